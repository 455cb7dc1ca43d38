"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/rts.h, and rejects invalid problems before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2107_08145_amd import inputs, rts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rts.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rts_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = rts.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(rts.SYMBOLS)


def test_version_and_status_strings():
    L = rts.lib()
    assert b"gfx950" in L.rts_version()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert rts.status_string(code) != "unknown status"
    assert rts.status_string(-3).startswith("RTS_E_WORKSPACE")


def _desc_problem(**kw):
    p = inputs.workload("grey32", size=8)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [
    ("nx", 1), ("ny", 0), ("nz", 1), ("dx", 0.0), ("dz", -1.0), ("dy", float("nan")),
    ("n_iter", 0), ("bot", 2), ("top", -1), ("i_bot", float("inf")),
])
def test_plan_rejects_bad_fields(field, value):
    p = _desc_problem(**{field: value})
    with pytest.raises(rts.RTSError) as e:
        rts.Plan(p)
    assert e.value.status == rts.RTS_E_ARG


def test_plan_rejects_bad_directions():
    p = _desc_problem()
    mu = p.mu.copy()
    mu[3] = [1.0, 0.0, 0.0]                 # mu_z == 0: no vertical boundary
    with pytest.raises(rts.RTSError):
        rts.Plan(_desc_problem(mu=mu))
    mu = p.mu.copy()
    mu[0] *= 1.01                           # not a unit vector
    with pytest.raises(rts.RTSError):
        rts.Plan(_desc_problem(mu=mu))


def test_plan_unsupported_sizes_and_precision():
    with pytest.raises(rts.RTSError) as e:
        rts.Plan(_desc_problem(nx=1025))
    assert e.value.status == rts.RTS_E_UNSUPPORTED
    with pytest.raises(rts.RTSError) as e:
        rts.Plan(_desc_problem(), prec=7)
    assert e.value.status == rts.RTS_E_ARG


def test_null_arguments():
    L = rts.lib()
    h = ctypes.c_void_p()
    assert L.rts_plan_create(None, 1, ctypes.byref(h)) == rts.RTS_E_ARG
    assert L.rts_workspace_bytes(None, 0, None) == rts.RTS_E_ARG
    assert L.rts_solve(None, None, None, None, 0, None) == rts.RTS_E_ARG
    pl = rts.Plan(_desc_problem())
    n = ctypes.c_size_t()
    assert L.rts_workspace_bytes(pl.handle, 9, ctypes.byref(n)) == rts.RTS_E_ARG
    # calls with missing inputs or workspace are rejected before any HIP call
    ci, co = rts.Inputs(), rts.Outputs()
    assert L.rts_solve(pl.handle, ctypes.byref(ci), ctypes.byref(co), None, 0, None) == rts.RTS_E_ARG
    ci = rts.Inputs(16, 16, 16)
    co = rts.Outputs(16, None, None)
    assert L.rts_solve(pl.handle, ctypes.byref(ci), ctypes.byref(co), None, 0, None) == rts.RTS_E_WORKSPACE
    assert L.rts_solve(pl.handle, ctypes.byref(ci), ctypes.byref(co), ctypes.c_void_p(256 * 3 + 8),
                       1 << 40, None) == rts.RTS_E_WORKSPACE          # misaligned
    assert L.rts_solve(pl.handle, ctypes.byref(ci), ctypes.byref(co), ctypes.c_void_p(256 * 4),
                       16, None) == rts.RTS_E_WORKSPACE               # too small
    assert L.rts_solve_batched(pl.handle, 2, ctypes.byref(ci), ctypes.byref(co),
                               ctypes.c_void_p(256), 1 << 40, None) == rts.RTS_E_ARG


def test_static_solve_refuses_plans_beyond_its_array():
    # rts_solve_static checks the plan's workspace against its fixed array
    # (64 MiB) before any device call, so this runs without a GPU
    L = rts.lib()
    big = rts.Plan(inputs.random_problem(72, 72, 72, seed=1, bands=5), rts.RTS_FP32)
    assert big.workspace_bytes() > rts.RTS_STATIC_SCRATCH_BYTES
    ci = rts.Inputs(256, 256, 256)
    co = rts.Outputs(256, None, None)
    assert L.rts_solve_static(big.handle, 1, ctypes.byref(ci), ctypes.byref(co),
                              None) == rts.RTS_E_WORKSPACE
    small = rts.Plan(inputs.random_problem(16, 16, 16, seed=1), rts.RTS_FP32)
    assert small.workspace_bytes() <= rts.RTS_STATIC_SCRATCH_BYTES
    assert L.rts_solve_static(None, 1, ctypes.byref(ci), ctypes.byref(co), None) == rts.RTS_E_ARG
    assert L.rts_solve_static(small.handle, 2, ctypes.byref(ci), ctypes.byref(co),
                              None) == rts.RTS_E_ARG
    assert L.rts_solve_static(small.handle, 1, None, None, None) == rts.RTS_E_ARG


def test_workspace_and_schedule():
    p = inputs.workload("grey32", size=16)
    pl = rts.Plan(p, rts.RTS_FP32)
    n0 = pl.workspace_bytes()
    N = p.ncells
    assert n0 >= 4 * N * (3 + 6)            # chi, chi^T, S^T and six partial sums
    s = pl.schedule()
    assert s["rows_per_strip"] in (2, 4, 6, 8)
    pl.set_schedule(rows_per_strip=8)
    assert pl.schedule()["rows_per_strip"] == 8
    with pytest.raises(rts.RTSError):
        pl.set_schedule(rows_per_strip=3)
    assert s["single_launch"] == 0            # one sweep launch per workgroup width
    pl.set_schedule(single_launch=1)
    assert pl.schedule()["single_launch"] == 1
    with pytest.raises(rts.RTSError):
        pl.set_schedule(single_launch=2)
    p64 = rts.Plan(p, rts.RTS_FP64)
    with pytest.raises(rts.RTSError):
        p64.set_schedule(rows_per_strip=8)  # fp64 strips hold at most 4 rows
    assert p64.workspace_bytes() > n0


def test_adjoint_workspace_query():
    # grey S4 on a cube: two z-sweep tasks (one pass) and four x/y-sweep tasks
    # (n_iter passes); the adjoint stores D of every pass for four slots
    p = inputs.workload("grey32", size=16)
    for prec, esz in ((rts.RTS_FP32, 4), (rts.RTS_FP64, 8)):
        pl = rts.Plan(p, prec)
        n0 = pl.workspace_bytes(rts.RTS_OP_SOLVE)
        n1 = pl.workspace_bytes(rts.RTS_OP_ADJOINT)
        N = p.ncells
        assert n1 >= n0 + esz * 4 * N * (2 + 4 * p.n_iter)


def test_adjoint_argument_errors():
    p = inputs.workload("grey32", size=16)
    pl = rts.Plan(p, rts.RTS_FP64)
    L = rts.lib()
    ci = rts.Inputs(256, 256, 256)
    cs = rts.Seeds(None, None, None)
    cg = rts.Grads(256, 256)
    ws = ctypes.c_void_p(256)
    big = 1 << 40
    assert L.rts_adjoint(None, 1, ctypes.byref(ci), ctypes.byref(cs), ctypes.byref(cg), ws, big,
                         None) == rts.RTS_E_ARG
    assert L.rts_adjoint(pl.handle, 2, ctypes.byref(ci), ctypes.byref(cs), ctypes.byref(cg), ws,
                         big, None) == rts.RTS_E_ARG
    assert L.rts_adjoint(pl.handle, 1, None, ctypes.byref(cs), ctypes.byref(cg), ws, big,
                         None) == rts.RTS_E_ARG
    bad = rts.Grads(None, 256)
    assert L.rts_adjoint(pl.handle, 1, ctypes.byref(ci), ctypes.byref(cs), ctypes.byref(bad), ws,
                         big, None) == rts.RTS_E_ARG
    n0 = pl.workspace_bytes(rts.RTS_OP_SOLVE)
    assert L.rts_adjoint(pl.handle, 1, ctypes.byref(ci), ctypes.byref(cs), ctypes.byref(cg), ws,
                         n0, None) == rts.RTS_E_WORKSPACE
    assert L.rts_adjoint(pl.handle, 1, ctypes.byref(ci), ctypes.byref(cs), ctypes.byref(cg),
                         ctypes.c_void_p(100), big, None) == rts.RTS_E_WORKSPACE


def test_autotune_workspace_and_errors():
    p = inputs.workload("grey32", size=16)
    pl = rts.Plan(p, rts.RTS_FP32)
    n_tune = pl.workspace_bytes(rts.RTS_OP_AUTOTUNE)
    for h in (2, 4, 6, 8):
        pl.set_schedule(rows_per_strip=h)
        assert pl.workspace_bytes(rts.RTS_OP_SOLVE) <= n_tune
    L = rts.lib()
    ci = rts.Inputs(256, 256, 256)
    co = rts.Outputs(256, None, None)
    sch = rts.Schedule()
    assert L.rts_plan_autotune(None, 1, ctypes.byref(ci), ctypes.byref(co), ctypes.c_void_p(256),
                               n_tune, None, 1, ctypes.byref(sch)) == rts.RTS_E_ARG
    assert L.rts_plan_autotune(pl.handle, 1, ctypes.byref(ci), ctypes.byref(co),
                               ctypes.c_void_p(256), n_tune, None, 0,
                               ctypes.byref(sch)) == rts.RTS_E_ARG
    assert L.rts_plan_autotune(pl.handle, 1, ctypes.byref(ci), ctypes.byref(co),
                               ctypes.c_void_p(100), n_tune, None, 1,
                               ctypes.byref(sch)) == rts.RTS_E_WORKSPACE


def test_input_check_argument_errors():
    # rts_check_inputs validates its arguments before any device call
    p = inputs.workload("grey32", size=16)
    pl = rts.Plan(p, rts.RTS_FP32)
    L = rts.lib()
    ok = rts.Inputs(256, 256, 256)
    ws = ctypes.c_void_p(256)
    assert L.rts_check_inputs(None, 1, ctypes.byref(ok), ws, 256, None) == rts.RTS_E_ARG
    assert L.rts_check_inputs(pl.handle, 1, None, ws, 256, None) == rts.RTS_E_ARG
    assert L.rts_check_inputs(pl.handle, 2, ctypes.byref(ok), ws, 256, None) == rts.RTS_E_ARG
    for bad in (rts.Inputs(None, 256, 256), rts.Inputs(256, None, 256), rts.Inputs(256, 256, None)):
        assert L.rts_check_inputs(pl.handle, 1, ctypes.byref(bad), ws, 256, None) == rts.RTS_E_ARG
    assert L.rts_check_inputs(pl.handle, 1, ctypes.byref(ok), None, 256, None) == rts.RTS_E_WORKSPACE
    assert L.rts_check_inputs(pl.handle, 1, ctypes.byref(ok), ctypes.c_void_p(100), 256,
                              None) == rts.RTS_E_WORKSPACE
    assert L.rts_check_inputs(pl.handle, 1, ctypes.byref(ok), ws, 255, None) == rts.RTS_E_WORKSPACE
    # a scattering plan needs eps
    gs = rts.Plan(inputs.random_problem(6, 5, 4, seed=1), rts.RTS_FP64, gs_iter=2)
    assert L.rts_check_inputs(gs.handle, 1, ctypes.byref(ok), ws, 256, None) == rts.RTS_E_ARG


def test_size_limits_rejected():
    p = inputs.workload("grey32", size=8)
    for field, value, code in (("nx", 1025, rts.RTS_E_UNSUPPORTED), ("nx", 1, rts.RTS_E_ARG)):
        q = inputs.workload("grey32", size=8)
        setattr(q, field, value)
        q.kappa = np.ones((1, q.nz, q.ny, q.nx))
        q.S = np.ones((1, q.nz, q.ny, q.nx))
        q.rho = np.ones((q.nz, q.ny, q.nx))
        with pytest.raises(rts.RTSError) as e:
            rts.Plan(q)
        assert e.value.status == code
    q = inputs.random_problem(4, 4, 4, seed=1, bands=17)
    with pytest.raises(rts.RTSError) as e:
        rts.Plan(q)
    assert e.value.status == rts.RTS_E_UNSUPPORTED
    q = inputs.random_problem(4, 4, 4, seed=1)
    q.mu = np.array([[1.0, 0.0, 0.0]])  # mu_z = 0: no vertical boundary
    q.w = np.ones(1)
    with pytest.raises(rts.RTSError) as e:
        rts.Plan(q)
    assert e.value.status == rts.RTS_E_ARG


def test_flux_plan_workspace_and_argument_errors():
    # a flux plan keeps two more partial arrays per sweep task whose four rays
    # share |mu| (S4: six such tasks for grey on a cube; the plane-axis
    # component follows from the partial sum), three per other task; F needs
    # such a plan and QF needs F, checked before any HIP call
    p = inputs.workload("grey32", size=16)
    N = p.ncells
    for prec, esz in ((rts.RTS_FP32, 4), (rts.RTS_FP64, 8)):
        n0 = rts.Plan(p, prec).workspace_bytes()
        n1 = rts.Plan(p, prec, flux=True).workspace_bytes()
        assert 6 * 2 * N * esz <= n1 - n0 <= 6 * 2 * (N * esz + 256)
    q = inputs.workload("grey32", size=16)
    q.mu = np.array([[0.3, 0.2, np.sqrt(1 - 0.13)], [0.1, -0.4, -np.sqrt(1 - 0.17)]])
    q.w = np.array([0.5, 0.5])
    n0 = rts.Plan(q, rts.RTS_FP32).workspace_bytes()
    n1 = rts.Plan(q, rts.RTS_FP32, flux=True).workspace_bytes()
    assert 2 * 3 * N * 4 <= n1 - n0 <= 2 * 3 * (N * 4 + 256)   # two one-ray tasks
    L = rts.lib()
    ci = rts.Inputs(256, 256, 256)
    ws, big = ctypes.c_void_p(256), 1 << 40
    plain = rts.Plan(p, rts.RTS_FP32)
    co = rts.Outputs(256, None, None, 256, None)
    assert L.rts_solve(plain.handle, ctypes.byref(ci), ctypes.byref(co), ws, big,
                       None) == rts.RTS_E_ARG
    fl = rts.Plan(p, rts.RTS_FP32, flux=True)
    co = rts.Outputs(256, None, None, None, 256)
    assert L.rts_solve(fl.handle, ctypes.byref(ci), ctypes.byref(co), ws, big,
                       None) == rts.RTS_E_ARG
    # the flux flag is 0 or 1
    p2 = _desc_problem()
    mu = np.ascontiguousarray(p2.mu, dtype=np.float64)
    w = np.ascontiguousarray(p2.w, dtype=np.float64)
    descs = (rts.Desc * 1)()
    dd = descs[0]
    dd.g = rts.Grid(p2.nx, p2.ny, p2.nz, p2.dx, p2.dy, p2.dz)
    dd.nbands, dd.nrays = p2.nbands, p2.nrays
    dd.mu = mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    dd.w = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    dd.n_iter, dd.prec = 3, rts.RTS_FP64
    h = ctypes.c_void_p()
    for flag, want in ((2, rts.RTS_E_ARG), (1, rts.RTS_OK)):
        dd.flux = flag
        assert L.rts_plan_create(descs, 1, ctypes.byref(h)) == want
    L.rts_plan_destroy(h)


def test_tolerance_plan_checks():
    p = inputs.workload("grey32", size=16)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(rts.RTSError) as e:
            rts.Plan(p, rts.RTS_FP64, tol=bad)
        assert e.value.status == rts.RTS_E_ARG
    pl = rts.Plan(p, rts.RTS_FP64, tol=1e-6)       # S4: one task per dominant axis and direction
    # two rays with the same dominant axis, direction and in-plane signs need two tasks
    q = inputs.workload("grey32", size=16)
    q.mu = np.concatenate([q.mu, q.mu[:1]])
    q.w = np.concatenate([q.w, q.w[:1]]) / (1 + q.w[0])
    rts.Plan(q, rts.RTS_FP64)                       # fine without a tolerance
    with pytest.raises(rts.RTSError) as e:
        rts.Plan(q, rts.RTS_FP64, tol=1e-6)
    assert e.value.status == rts.RTS_E_UNSUPPORTED
    # the adjoint replays a fixed sweep count: rejected before any HIP call
    L = rts.lib()
    ci = rts.Inputs(256, 256, 256)
    cs = rts.Seeds(None, None, None)
    cg = rts.Grads(256, 256)
    assert L.rts_adjoint(pl.handle, 1, ctypes.byref(ci), ctypes.byref(cs), ctypes.byref(cg),
                         ctypes.c_void_p(256), 1 << 40, None) == rts.RTS_E_UNSUPPORTED


def test_kept_forward_and_backward_argument_errors():
    p = inputs.workload("grey32", size=16)
    pl = rts.Plan(p, rts.RTS_FP32)
    L = rts.lib()
    ci = rts.Inputs(256, 256, 256)
    co = rts.Outputs(256, None, None)
    cs = rts.Seeds(None, None, None)
    cg = rts.Grads(256, 256)
    n_solve = pl.workspace_bytes(rts.RTS_OP_SOLVE)
    # the kept forward needs the adjoint workspace; both check before any HIP call
    assert L.rts_solve_for_adjoint(pl.handle, 1, ctypes.byref(ci), ctypes.byref(co),
                                   ctypes.c_void_p(256), n_solve, None) == rts.RTS_E_WORKSPACE
    assert L.rts_solve_for_adjoint(pl.handle, 2, ctypes.byref(ci), ctypes.byref(co),
                                   ctypes.c_void_p(256), 1 << 40, None) == rts.RTS_E_ARG
    assert L.rts_adjoint_from_solve(pl.handle, 1, ctypes.byref(ci), ctypes.byref(cs),
                                    ctypes.byref(cg), ctypes.c_void_p(256), n_solve,
                                    None) == rts.RTS_E_WORKSPACE
    bad = rts.Grads(None, 256)
    assert L.rts_adjoint_from_solve(pl.handle, 1, ctypes.byref(ci), ctypes.byref(cs),
                                    ctypes.byref(bad), ctypes.c_void_p(256), 1 << 40,
                                    None) == rts.RTS_E_ARG
    tol = rts.Plan(p, rts.RTS_FP32, tol=1e-4)
    assert L.rts_solve_for_adjoint(tol.handle, 1, ctypes.byref(ci), ctypes.byref(co),
                                   ctypes.c_void_p(256), 1 << 40, None) == rts.RTS_E_UNSUPPORTED


def test_bench_refuses_more_than_one_gpu_and_entry_points_exist():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    sys.path.insert(0, ROOT)
    import __graft_entry__ as g
    assert callable(g.build) and callable(g.smoke)


def test_bench_trace_summary_groups_by_workgroup(tmp_path):
    # a kernel-trace database of the shape rocprofv3 writes: one table of
    # dispatches with the kernel name, duration (ns) and workgroup size
    import sqlite3
    import sys
    sys.path.insert(0, ROOT)
    import bench
    c = sqlite3.connect(tmp_path / "trace_results.db")
    c.execute("create table kernels (name text, duration integer, workgroup_x integer)")
    rows = [("k(A)", 3000, 576), ("k(A)", 5000, 576), ("k(A)", 1000, 64), ("z(B)", 2000, 256)]
    c.executemany("insert into kernels values (?, ?, ?)", rows)
    c.commit()
    c.close()
    plain = {n: (k, a) for n, k, a, _ in bench.trace_summary(str(tmp_path))}
    assert plain == {"k(A)": (3, 3.0), "z(B)": (1, 2.0)}
    by = {n: (k, a) for n, k, a, _ in bench.trace_summary(str(tmp_path), by_workgroup=True)}
    assert by == {"k(A) [workgroup 576]": (2, 4.0), "k(A) [workgroup 64]": (1, 1.0),
                  "z(B) [workgroup 256]": (1, 2.0)}
