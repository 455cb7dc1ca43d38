"""Parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py uses (autotuned schedule), against the FP64 oracle
run on the host's cores.

Bars: the FP64 path as in test_gpu_parity (per cell, |dQ| <= 1e-9 |Q| +
4 pi chi S 1e-13; J, I_top 1e-13 of max); the FP32 path within 1e-5 of
max|Q| in Q (the precision target of the FP32 storage design) and 2e-6 in J
and I_top.  The adjoint at 128^3: FP64 within 1e-10 of the oracle's reverse
mode per array, FP32 within 2e-4, and central differences of the FP64
forward solve at 64 seeded cells (relative step 1e-6) to 1e-6.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2107_08145_amd import inputs, rts
from percell import assert_paper_rule

pytestmark = pytest.mark.gpu
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _errs(got, ref):
    return tuple(float(np.abs(g - o).max() / max(np.abs(o).max(), 1e-300)) for g, o in zip(got, ref))


def _tuned_solve(p, prec):
    import torch
    pl = rts.Plan(p, prec)
    ins = pl.device_inputs(p)
    outs = pl.new_outputs(p)
    sched = pl.autotune([ins], [outs], reps=1)
    pl.solve_into([ins], [outs])
    pl.check_status()
    torch.cuda.synchronize()
    return tuple(o.double().cpu().numpy() for o in outs), sched


@pytest.mark.parametrize("name", ["grey288", "bands288"])
def test_full_size_fp32(name):
    p = inputs.workload(name).astype(np.float32)
    print("case full size fp32", name, flush=True)
    got, sched = _tuned_solve(p, rts.RTS_FP32)
    ref = oracle.solve(p.astype(np.float64), threads=THREADS)
    eq, ej, ei = _errs(got, ref)
    print(f"{name} fp32 {sched}: Q {eq:.2e} J {ej:.2e} I_top {ei:.2e}", flush=True)
    assert eq <= 1e-5 and ej <= 2e-6 and ei <= 2e-6
    for n, g, o in zip(("Q", "J", "I_top"), got, ref):
        assert_paper_rule(f"{name} {n}", g, o)


def test_full_size_boxes6_batched_fp32():
    # the six uneven boxes in one autotuned, graph-replayed rts_solve_batched
    # call (one persistent sweep launch per workgroup width), box by box
    import torch
    ps = [p.astype(np.float32) for p in inputs.workload("boxes6")]
    pl = rts.Plan(ps, rts.RTS_FP32)
    ins = [pl.device_inputs(p) for p in ps]
    outs = [pl.new_outputs(p) for p in ps]
    pl.autotune(ins, outs, reps=1)
    pl.set_schedule(use_graph=1)
    for rep in range(2):
        print("case full size boxes6 batched", rep, pl.schedule(), flush=True)
        pl.solve_into(ins, outs, batched=True)
        pl.check_status()
        torch.cuda.synchronize()
    got = [tuple(t.double().cpu().numpy() for t in o) for o in outs]
    del outs, ins, pl
    torch.cuda.empty_cache()
    for p, g in zip(ps, got):
        ref = oracle.solve(p.astype(np.float64), threads=THREADS)
        eq, ej, ei = _errs(g, ref)
        print(f"boxes6 {p.nx}x{p.ny}x{p.nz}: Q {eq:.2e} J {ej:.2e} I_top {ei:.2e}", flush=True)
        assert eq <= 1e-5 and ej <= 2e-6 and ei <= 2e-6
        for n, gg, o in zip(("Q", "J", "I_top"), g, ref):
            assert_paper_rule(f"boxes6 {p.nx}x{p.ny}x{p.nz} {n}", gg, o)


def test_full_size_grey288_fp64():
    p = inputs.workload("grey288")
    print("case full size fp64 grey288", flush=True)
    got, sched = _tuned_solve(p, rts.RTS_FP64)
    ref = oracle.solve(p, threads=THREADS)
    Qg, Jg, Ig = got
    Qo, Jo, Io = ref
    chi = oracle.chi_of(p)
    floor = 4 * math.pi * (np.abs(chi) * np.abs(p.S)).max(axis=0) * 1e-13
    print(f"grey288 fp64: Q {np.abs(Qg - Qo).max() / np.abs(Qo).max():.2e}", flush=True)
    assert np.all(np.abs(Qg - Qo) <= 1e-9 * np.abs(Qo) + floor)
    assert np.abs(Jg - Jo).max() <= 1e-13 * np.abs(Jo).max()
    assert np.abs(Ig - Io).max() <= 1e-13 * np.abs(Io).max()


def test_full_size_bands288_flux_fp32():
    # the flux vector and its divergence at 288^3 x 5 bands (bars as in
    # test_gpu_flux: F within 2e-6 of 4 pi max|J|, QF within sum_d 4/delta_d of that)
    import torch
    p = inputs.workload("bands288").astype(np.float32)
    print("case full size bands288 flux fp32", flush=True)
    pl = rts.Plan(p, rts.RTS_FP32, flux=True)
    ins = pl.device_inputs(p)
    outs = pl.new_outputs(p, want_flux=True)
    pl.solve_into([ins], [outs])
    pl.check_status()
    torch.cuda.synchronize()
    got = [o.double().cpu().numpy() for o in outs]
    ref = oracle.flux(p.astype(np.float64), threads=THREADS)
    scale = 4 * math.pi * np.abs(ref[1]).max()
    ef = np.abs(got[3] - ref[3]).max()
    eqf = np.abs(got[4] - ref[4]).max()
    print(f"bands288 flux fp32: F {ef / scale:.2e} of 4 pi max J ({ef / np.abs(ref[3]).max():.2e} "
          f"of max|F|), QF {eqf / np.abs(ref[4]).max():.2e} of max|QF|", flush=True)
    assert ef <= 2e-6 * scale
    assert eqf <= (4 / p.dx + 4 / p.dy + 4 / p.dz) * 2e-6 * scale
    eq, ej, ei = _errs(got[:3], ref[:3])
    assert eq <= 1e-5 and ej <= 2e-6 and ei <= 2e-6
    for n, g, o in zip(("Q", "J", "I_top"), got[:3], ref[:3]):
        assert_paper_rule(f"bands288 flux {n}", g, o)


def _adjoint128_seeds(p, prec):
    s_target, g = inputs.adjoint_seeds(p, 4000)
    t = p.astype(p.S.dtype)
    t.S = s_target.astype(p.S.dtype)
    _, _, it_target = rts.solve(t, prec)
    _, _, it = rts.solve(p, prec)
    return g, 2 * (it - it_target)


@pytest.mark.parametrize("prec", [rts.RTS_FP64, rts.RTS_FP32])
def test_adjoint128_full_size(prec):
    p = inputs.workload("adjoint128")
    if prec == rts.RTS_FP32:
        p = p.astype(np.float32)
    print("case adjoint128 full size", prec, flush=True)
    gQ, gI = _adjoint128_seeds(p, prec)
    got = rts.adjoint(p, prec, gQ, None, gI)
    ref = oracle.adjoint(p.astype(np.float64), gQ, None, gI.astype(p.S.dtype).astype(np.float64),
                         threads=THREADS)
    e = _errs(got, ref)
    print(f"adjoint128 prec {prec}: dS {e[0]:.2e} dchi {e[1]:.2e}", flush=True)
    assert max(e) <= (1e-10 if prec == rts.RTS_FP64 else 2e-4)


def test_adjoint128_finite_differences_64_cells():
    """Central differences of the FP64 forward solve with relative step 1e-6
    at 64 seeded cells (alternately in S and kappa).  The difference quotient
    carries the rounding of the two solves: with eps = 2.2e-16 its error bound
    is 2 eps sum(|g| (|out+| + |out-|)) / (2 h) over the cells the
    perturbation reaches (outputs rounded to within a few eps; the measured
    error stays below a tenth of this), so the check is
    |fd - ad| <= 1e-6 |ad| + that bound.  Four of the
    cells are also checked against the oracle's complex-step derivative, exact
    to rounding, to 1e-9."""
    p = inputs.workload("adjoint128")
    gQ, gI = _adjoint128_seeds(p, rts.RTS_FP64)
    dS, dchi = rts.adjoint(p, rts.RTS_FP64, gQ, None, gI)
    cells = inputs.fd_cells(p, 4000, 64)
    print("case adjoint128 finite differences", flush=True)

    def outputs():
        Q, J, It = rts.solve(p, rts.RTS_FP64)
        return Q, It

    eps = np.finfo(np.float64).eps
    worst, rel, nrel = 0.0, [], []
    for n, cell in enumerate(cells):
        z, y, x = np.unravel_index(int(cell), (p.nz, p.ny, p.nx))
        which = "S" if n % 2 == 0 else "kappa"
        arr = getattr(p, which)
        base = arr[0, z, y, x]
        h = 1e-6 * base
        arr[0, z, y, x] = base + h
        Qp, Ip = outputs()
        arr[0, z, y, x] = base - h
        Qm, Im = outputs()
        arr[0, z, y, x] = base
        # differenced cell by cell, so that only cells the perturbation reaches carry rounding
        fd = (float((gQ * (Qp - Qm)).sum()) + float((gI * (Ip - Im)).sum())) / (2 * h)
        mq, mi = Qp != Qm, Ip != Im
        noise = 2 * eps * (float((np.abs(gQ) * (np.abs(Qp) + np.abs(Qm)))[mq].sum())
                             + float((np.abs(gI) * (np.abs(Ip) + np.abs(Im)))[mi].sum())) / (2 * h)
        ad = dS[0, z, y, x] if which == "S" else dchi[0, z, y, x] * p.rho[z, y, x]
        worst = max(worst, abs(fd - ad) / (1e-6 * abs(ad) + noise))
        rel.append(abs(fd - ad) / abs(ad))
        nrel.append(noise / abs(ad))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + noise, (which, (z, y, x), fd, ad, noise)
        if n < 4:
            flat = (z * p.ny + y) * p.nx + x
            dQ, _, dI = oracle.complex_step(p, "S" if which == "S" else "chi", flat, threads=THREADS)
            cs = float((gQ * dQ).sum() + (gI * dI).sum())
            if which == "kappa":
                cs *= p.rho[z, y, x]
            assert abs(ad - cs) <= 1e-9 * abs(cs) + 1e-15, (which, (z, y, x), ad, cs)
    print(f"adjoint128 finite differences: worst |fd - ad| / bound {worst:.3f}; "
          f"|fd - ad| / |ad| median {np.median(rel):.1e} max {max(rel):.1e}; "
          f"noise bound / |ad| median {np.median(nrel):.1e} max {max(nrel):.1e}", flush=True)


def _boxes6_loss64(p64, seeds, rho_scale=1.0):
    q = p64 if rho_scale == 1.0 else p64.astype(np.float64)
    if rho_scale != 1.0:
        q.rho = p64.rho * rho_scale
    pl = rts.Plan(q, rts.RTS_FP64)
    pl.set_schedule(rows_per_strip=4)  # (576 rows: every strip of a z sweep resident)
    Q, J, It = rts.solve(q, rts.RTS_FP64, plan=pl)
    gQ, gJ, gI = seeds
    return float((gQ * Q).sum()) + float((gJ * J).sum()) + float((gI * It).sum())


@pytest.fixture(scope="module")
def boxes6_adjoint():
    """One batched FP32 rts_adjoint over the six uneven boxes at full size (the
    576^2 x 192 box's z sweeps take the two-pass reverse); U(0,1) seeds: gQ
    (FP64), gJ and gItop (FP32-representable).  Returns the FP32 problems, the
    seeds and the gradients (float64 on the host)."""
    import torch
    ps = [p.astype(np.float32) for p in inputs.workload("boxes6")]
    pl = rts.Plan(ps, rts.RTS_FP32)
    ins = [pl.device_inputs(p) for p in ps]
    host, seeds, grads = [], [], []
    for i, p in enumerate(ps):
        r = np.random.default_rng(7000 + i)
        gQ = r.random((p.nz, p.ny, p.nx))
        gJ = r.random(p.S.shape).astype(np.float32).astype(np.float64)
        gI = r.random((p.nbands, p.n_up, p.ny, p.nx)).astype(np.float32).astype(np.float64)
        host.append((gQ, gJ, gI))
        seeds.append((torch.as_tensor(gQ, device="cuda"),
                      torch.as_tensor(gJ.astype(np.float32), device="cuda"),
                      torch.as_tensor(gI.astype(np.float32), device="cuda")))
        grads.append((torch.empty(p.S.shape, dtype=torch.float32, device="cuda"),
                      torch.empty(p.S.shape, dtype=torch.float32, device="cuda")))
    print("case full size boxes6 adjoint", pl.workspace_bytes(rts.RTS_OP_ADJOINT), flush=True)
    pl.adjoint_into(ins, seeds, grads)
    pl.check_status()
    torch.cuda.synchronize()
    got = [tuple(t.double().cpu().numpy() for t in g) for g in grads]
    del grads, seeds, ins, pl
    torch.cuda.empty_cache()
    return ps, host, got


@pytest.mark.parametrize("box", range(6))
def test_full_size_boxes6_adjoint_fp32(boxes6_adjoint, box):
    """Box by box, of the one batched adjoint (fixture):
    * at any size: L is linear in S (bottom I = S, top I = 0), so
      <dL/dS, S> = L, with L from the FP64 forward on the same FP32-rounded
      inputs: |<dS, S> - L| <= 1e-5 sum|dS S|; and scaling rho by 1 +- h
      (h = 1e-3, every band's chi) gives the central difference
      dL/dh = sum_b <dL/dchi_b, chi_b> to 1e-4 sum|dchi chi| (truncation
      ~ h^2, FP64 rounding ~ 1e-13 / h);
    * the 64^3 box also against the oracle's reverse mode per array (2e-4 of
      max, as the other FP32 adjoint tests; the bench's --errors adds the
      96^2 x 512 box)."""
    ps, host, got = boxes6_adjoint
    p, sd, (dS, dchi) = ps[box], host[box], got[box]
    name = f"{p.nx}x{p.ny}x{p.nz}"
    p64 = p.astype(np.float64)
    L0 = _boxes6_loss64(p64, sd)
    sS = float((dS * p64.S).sum())
    aS = float(np.abs(dS * p64.S).sum())
    h = 1e-3
    fd = (_boxes6_loss64(p64, sd, 1 + h) - _boxes6_loss64(p64, sd, 1 - h)) / (2 * h)
    chi = oracle.chi_of(p64)
    ad = float((dchi * chi).sum())
    ac = float(np.abs(dchi * chi).sum())
    print(f"boxes6 adjoint {name}: <dS,S> - L {abs(sS - L0) / aS:.2e} of sum|dS S|, "
          f"d/drho {abs(fd - ad) / ac:.2e} of sum|dchi chi|", flush=True)
    assert abs(sS - L0) <= 1e-5 * aS, (name, sS, L0)
    assert abs(fd - ad) <= 1e-4 * ac, (name, fd, ad)
    if name == "64x64x64":
        ref = oracle.adjoint(p64, sd[0], sd[1], sd[2], threads=THREADS)
        e = _errs((dS, dchi), ref)
        print(f"boxes6 adjoint {name} vs oracle: dS {e[0]:.2e} dchi {e[1]:.2e}", flush=True)
        assert max(e) <= 2e-4, (name, e)
