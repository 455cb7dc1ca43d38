"""Per-value error metrics of the paper's validation rule (section
"Refactoring the MURaM Code": a value passes at a relative difference of
1e-5 or an absolute difference of 1e-7).  The arrays here are in arbitrary
units, so the absolute threshold is taken relative to the array's largest
reference magnitude.  Shared by the GPU tests (not collected by pytest)."""
import numpy as np

REL = 1e-5
ABS_OF_MAX = 1e-7


def paper_rule(got, ref, rel=REL, abs_of_max=ABS_OF_MAX):
    """(failing values, normwise max|d|/max|ref|, largest relative error over
    the values with |ref| >= 1e-3 max|ref|) of got against ref."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    a = np.abs(ref)
    m = a.max() if a.size else 0.0
    ok = (d <= rel * a) | (d <= abs_of_max * m)
    big = a >= 1e-3 * m
    worst = float((d[big] / a[big]).max()) if m > 0 and big.any() else 0.0
    return int((~ok).sum()), float(d.max() / m) if m > 0 else float(d.max()), worst


def assert_paper_rule(name, got, ref, **kw):
    fails, norm, worst = paper_rule(got, ref, **kw)
    print(f"{name}: per-value failures {fails}, normwise {norm:.2e}, "
          f"max rel (|ref| >= 1e-3 max) {worst:.2e}", flush=True)
    assert fails == 0, (name, fails, norm, worst)
    return norm, worst
