"""GPU adjoint (rts_adjoint through the C ABI) against the FP64 CPU oracle's
reverse mode, finite differences of the GPU forward solve, and the autograd
binding.

Tolerances (derived from the arithmetic):
* FP64 vs oracle: both sides round at ~1e-16 per operation along paths of a
  few hundred steps; the GPU sweeps D = I - S with its own weight formulas and
  sums the per-task partials in another order.  Per array we require
  max|d_gpu - d_oracle| <= 1e-10 max|d_oracle|.
* FP32 vs oracle (same FP32-rounded inputs): FP32 state (6e-8 per operation)
  along the same paths, FP64 final sums: max|delta| <= 2e-4 max|d_oracle|.
* Finite differences of the FP64 forward with relative step 1e-6 (central):
  truncation ~1e-12 and cancellation ~1e-16 |L| / (1e-6 S); seeds are kept to
  a small block around the perturbed cell so that |L| stays small; the
  directional derivatives agree to 1e-6 relative.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_08145_amd import inputs, rts

pytestmark = pytest.mark.gpu


def _seeds(p, seed, gq=True, gj=True, gi=True):
    r = np.random.default_rng(seed)
    gQ = r.standard_normal((p.nz, p.ny, p.nx)) if gq else None
    gJ = r.standard_normal(p.S.shape) if gj else None
    gI = r.standard_normal((p.nbands, p.n_up, p.ny, p.nx)) if gi else None
    return gQ, gJ, gI


def _cmp(got, ref, tol):
    errs = []
    for g, o in zip(got, ref):
        for b in range(o.shape[0]):
            scale = np.abs(o[b]).max()
            e = np.abs(g[b] - o[b]).max() / max(scale, 1e-300)
            errs.append(e)
            assert e <= tol, (b, e)
    return max(errs)


def _run(p, prec, seeds, tol, threads=8):
    gQ, gJ, gI = seeds
    pp = p.astype(np.float32) if prec == rts.RTS_FP32 else p
    got = rts.adjoint(pp, prec, gQ, gJ, gI)
    ref = oracle.adjoint(pp.astype(np.float64), gQ,
                         None if gJ is None else gJ.astype(pp.S.dtype).astype(np.float64),
                         None if gI is None else gI.astype(pp.S.dtype).astype(np.float64),
                         threads=threads)
    return _cmp(got, ref, tol)


@pytest.mark.parametrize("shape", [(20, 13, 11), (2, 3, 2), (65, 64, 17), (64, 7, 33)])
def test_adjoint_fp64_matches_oracle(shape):
    nx, ny, nz = shape
    p = inputs.random_problem(nx, ny, nz, seed=nx + 3 * ny)
    print("case adjoint fp64", shape, flush=True)
    e = _run(p, rts.RTS_FP64, _seeds(p, 1), 1e-10)
    print(f"adjoint fp64 {shape}: {e:.2e}")


@pytest.mark.parametrize("bc", [(1, 1, 1.7, 3), (0, 1, 0.0, 1), (1, 0, 0.3, 4)])
def test_adjoint_boundary_variants(bc):
    bot, top, ib, nit = bc
    p = inputs.random_problem(24, 20, 14, seed=5, bot=bot, top=top, i_bot=ib, n_iter=nit)
    print("case adjoint bc", bc, flush=True)
    _run(p, rts.RTS_FP64, _seeds(p, 2), 1e-10)


def test_adjoint_multiband_and_partial_seeds():
    p = inputs.random_problem(26, 22, 15, seed=21, bands=3)
    p.qweight = np.array([1.0, 0.25, 0.0])
    print("case adjoint multiband", flush=True)
    _run(p, rts.RTS_FP64, _seeds(p, 3), 1e-10)
    _run(p, rts.RTS_FP64, _seeds(p, 4, gj=False, gi=False), 1e-10)
    _run(p, rts.RTS_FP64, _seeds(p, 5, gq=False), 1e-10)


def test_adjoint_general_directions():
    p = inputs.random_problem(18, 16, 12, seed=9)
    p.dx = p.dy = 3.0
    r = np.random.default_rng(3)
    extra = r.standard_normal((2, 3))
    extra /= np.linalg.norm(extra, axis=1, keepdims=True)
    p.mu = np.vstack([p.mu, extra])
    p.w = np.concatenate([p.w * 0.9, [0.05, 0.05]])
    print("case adjoint general directions", flush=True)
    _run(p, rts.RTS_FP64, _seeds(p, 6), 1e-10)


def test_adjoint_fp32_matches_oracle():
    p = inputs.random_problem(40, 36, 30, seed=12, lo=1e-3, hi=1e3)
    print("case adjoint fp32", flush=True)
    e = _run(p, rts.RTS_FP32, _seeds(p, 7), 2e-4)
    print(f"adjoint fp32: {e:.2e}")


# Every task is reversed as two slot-pair passes, one thread per column, with
# strips as tall as each width class allows (FP32: 6 rows up to 512 padded
# columns, 3 up to 768, 2 up to 1024; FP64: 2 rows up to 512, 1 up to 768):
# one case per class, with partial last strips and exchange rings that wrap.
@pytest.mark.parametrize("prec,shape", [(rts.RTS_FP32, (300, 20, 9)),
                                        (rts.RTS_FP64, (300, 12, 8)),
                                        (rts.RTS_FP32, (520, 10, 6)),
                                        (rts.RTS_FP32, (700, 9, 5)),
                                        (rts.RTS_FP32, (900, 7, 5)),
                                        (rts.RTS_FP64, (600, 7, 4))])
def test_adjoint_wide_planes(prec, shape):
    nx, ny, nz = shape
    p = inputs.random_problem(nx, ny, nz, seed=nx + ny, bands=2)
    print("case adjoint wide", prec, shape, flush=True)
    tol = 1e-10 if prec == rts.RTS_FP64 else 2e-4
    e = _run(p, prec, _seeds(p, 8), tol, threads=16)
    print(f"adjoint wide {shape}: {e:.2e}")


def test_adjoint_fp64_plane_beyond_the_reverse_shapes_is_unsupported():
    # FP64 reverse strips are at most 768 columns wide
    p = inputs.random_problem(800, 6, 4, seed=3)
    print("case adjoint fp64 800 columns", flush=True)
    with pytest.raises(rts.RTSError, match="UNSUPPORTED"):
        rts.adjoint(p, rts.RTS_FP64, *_seeds(p, 9))


# Strip chains: periodic rows (z planes), bounded rows (x and y planes) with
# partial last strips, one-strip tasks, and the schedule's split_reverse flag
# (accepted, no effect: results are bitwise those of the default).
@pytest.mark.parametrize("case", [
    dict(prec=rts.RTS_FP64, shape=(20, 13, 11), seed=51),
    dict(prec=rts.RTS_FP64, shape=(24, 20, 14), seed=52, bot=1, top=1, i_bot=1.7, n_iter=3),
    dict(prec=rts.RTS_FP64, shape=(33, 9, 17), seed=53, bands=2, top=0, n_iter=4),
    dict(prec=rts.RTS_FP32, shape=(40, 36, 30), seed=54, lo=1e-3, hi=1e3),
    dict(prec=rts.RTS_FP32, shape=(17, 5, 3), seed=56, n_iter=2),
    dict(prec=rts.RTS_FP32, shape=(64, 64, 61), seed=57, bands=2),
])
def test_adjoint_strip_chains_match_oracle(case):
    c = dict(case)
    prec, shape, seed = c.pop("prec"), c.pop("shape"), c.pop("seed")
    p = inputs.random_problem(*shape, seed=seed, **c)
    pp = p.astype(np.float32) if prec == rts.RTS_FP32 else p
    print("case adjoint strips", prec, shape, flush=True)
    tol = 1e-10 if prec == rts.RTS_FP64 else 2e-4
    gQ, gJ, gI = _seeds(p, seed)
    got = rts.adjoint(pp, prec, gQ, gJ, gI)
    ref = oracle.adjoint(pp.astype(np.float64), gQ, gJ.astype(pp.S.dtype).astype(np.float64),
                         gI.astype(pp.S.dtype).astype(np.float64), threads=8)
    e = _cmp(got, ref, tol)
    print(f"adjoint strips {shape}: {e:.2e}")
    pl = rts.Plan(pp, prec)
    pl.set_schedule(split_reverse=1)
    again = rts.adjoint(pp, prec, gQ, gJ, gI, plan=pl)
    for a, b in zip(got, again):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,shape", [(rts.RTS_FP64, (520, 6, 4)),
                                        (rts.RTS_FP32, (576, 576, 5))])
def test_adjoint_wide_and_tall_planes(prec, shape):
    # 520 FP64 columns; a 576 x 576 z plane (192 strips of 3 rows per pass)
    p = inputs.random_problem(*shape, seed=shape[0] + shape[2], bands=1)
    print("case adjoint wide and tall", prec, shape, flush=True)
    tol = 1e-10 if prec == rts.RTS_FP64 else 2e-4
    e = _run(p, prec, _seeds(p, 10), tol, threads=16)
    print(f"adjoint wide and tall {shape}: {e:.2e}")


def test_adjoint128_fp32_small_matches_oracle():
    p = inputs.workload("adjoint128", size=32)
    print("case adjoint128 size 32 fp32", flush=True)
    s_target, gq = inputs.adjoint_seeds(p, 4000)
    e = _run(p, rts.RTS_FP32, (gq, None, None), 2e-4)
    print(f"adjoint128/32 fp32: {e:.2e}")


def _loss(p, seeds):
    Q, J, I = rts.solve(p, rts.RTS_FP64)
    gQ, gJ, gI = seeds
    return float((gQ * Q).sum() + (gJ * J).sum() + (gI * I).sum())


def test_adjoint_matches_finite_differences():
    p = inputs.random_problem(12, 10, 9, seed=33, bands=2)
    r = np.random.default_rng(8)
    cells = [(0, 4, 5, 6), (1, 2, 3, 4), (0, 8, 0, 11), (1, 0, 9, 0)]
    for (b, z, y, x) in cells:
        # seeds on a 5^3 block around the cell (periodic in x, y)
        m3 = np.zeros((p.nz, p.ny, p.nx))
        for dz in range(-2, 3):
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    if 0 <= z + dz < p.nz:
                        m3[z + dz, (y + dy) % p.ny, (x + dx) % p.nx] = 1
        gQ = r.standard_normal(m3.shape) * m3
        gJ = r.standard_normal(p.S.shape) * m3[None]
        gI = r.standard_normal((p.nbands, p.n_up, p.ny, p.nx)) * m3[-1][None, None]
        seeds = (gQ, gJ, gI)
        dS, dchi = rts.adjoint(p, rts.RTS_FP64, *seeds)
        print("case fd", (b, z, y, x), flush=True)
        for which in ("S", "kappa"):
            arr = getattr(p, which)
            base = arr[b, z, y, x]
            h = 1e-6 * base
            arr[b, z, y, x] = base + h
            lp = _loss(p, seeds)
            arr[b, z, y, x] = base - h
            lm = _loss(p, seeds)
            arr[b, z, y, x] = base
            fd = (lp - lm) / (2 * h)
            ad = dS[b, z, y, x] if which == "S" else dchi[b, z, y, x] * p.rho[z, y, x]
            assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12, (which, (b, z, y, x), fd, ad)


def test_adjoint_batched_equals_single():
    import torch
    ps = [inputs.random_problem(40, 24, 18, seed=31, bands=2).astype(np.float32),
          inputs.random_problem(17, 33, 21, seed=32, bands=2).astype(np.float32)]
    pl = rts.Plan(ps, rts.RTS_FP32)
    ins = [pl.device_inputs(p) for p in ps]
    seeds, grads, host = [], [], []
    for i, p in enumerate(ps):
        gQ, gJ, gI = _seeds(p, 40 + i)
        host.append((gQ, gJ, gI))
        seeds.append((torch.as_tensor(gQ, device="cuda"),
                      torch.as_tensor(gJ.astype(np.float32), device="cuda"),
                      torch.as_tensor(gI.astype(np.float32), device="cuda")))
        grads.append((torch.empty(p.S.shape, dtype=torch.float32, device="cuda"),
                      torch.empty(p.S.shape, dtype=torch.float32, device="cuda")))
    for rep in range(2):
        pl.adjoint_into(ins, seeds, grads)
        pl.check_status()
        torch.cuda.synchronize()
        for p, h, g in zip(ps, host, grads):
            single = rts.adjoint(p, rts.RTS_FP32, h[0], h[1].astype(np.float32), h[2].astype(np.float32))
            for a, b in zip(g, single):
                assert np.array_equal(a.double().cpu().numpy(), b), rep


def test_adjoint_width_launches():
    # planes of 64 to 320 padded columns: with one reverse launch per width
    # a box's gradients are bitwise those of its own plan; one launch at the
    # widest width (single_launch) sums the slots of the narrow tasks in
    # another order and meets the same bar against the oracle
    import torch
    ps = [inputs.random_problem(300, 20, 9, seed=71, bands=2).astype(np.float32),
          inputs.random_problem(40, 70, 12, seed=72).astype(np.float32)]
    pl = rts.Plan(ps, rts.RTS_FP32)
    ins = [pl.device_inputs(p) for p in ps]
    seeds, grads, host, refs = [], [], [], []
    for i, p in enumerate(ps):
        gQ, gJ, gI = _seeds(p, 80 + i)
        gJ, gI = gJ.astype(np.float32), gI.astype(np.float32)
        host.append((gQ, gJ, gI))
        refs.append(oracle.adjoint(p.astype(np.float64), gQ, gJ.astype(np.float64),
                                   gI.astype(np.float64), threads=8))
        seeds.append((torch.as_tensor(gQ, device="cuda"), torch.as_tensor(gJ, device="cuda"),
                      torch.as_tensor(gI, device="cuda")))
        grads.append((torch.empty(p.S.shape, dtype=torch.float32, device="cuda"),
                      torch.empty(p.S.shape, dtype=torch.float32, device="cuda")))
    for single in (0, 1):
        pl.set_schedule(single_launch=single)
        print("case adjoint width launches", single, flush=True)
        pl.adjoint_into(ins, seeds, grads)
        pl.check_status()
        torch.cuda.synchronize()
        for p, h, g, ref in zip(ps, host, grads, refs):
            got = [t.double().cpu().numpy() for t in g]
            e = _cmp(got, ref, 2e-4)
            print(f"adjoint width launches single={single} {p.nx}x{p.ny}: {e:.2e}")
            if single == 0:
                alone = rts.adjoint(p, rts.RTS_FP32, *h)
                for a, b in zip(got, alone):
                    assert np.array_equal(a, b)


def test_autograd_chain_rule():
    import torch
    from paper_2107_08145_amd.autograd import rts_apply
    p = inputs.random_problem(16, 14, 12, seed=50, bands=2)
    pl = rts.Plan(p, rts.RTS_FP64)
    k = torch.tensor(p.kappa, device="cuda", requires_grad=True)
    rho = torch.tensor(p.rho, device="cuda", requires_grad=True)
    S = torch.tensor(p.S, device="cuda", requires_grad=True)
    gQ, gJ, gI = _seeds(p, 51)
    Q, J, It = rts_apply(k, rho, S, pl)
    loss = ((Q * torch.tensor(gQ, device="cuda")).sum() + (J * torch.tensor(gJ, device="cuda")).sum()
            + (It * torch.tensor(gI, device="cuda")).sum())
    loss.backward()
    dS, dchi = oracle.adjoint(p, gQ, gJ, gI, threads=8)
    ref_k = dchi * p.rho[None]
    ref_r = (dchi * p.kappa).sum(0)
    for got, ref in ((k.grad, ref_k), (rho.grad, ref_r), (S.grad, dS)):
        g = got.cpu().numpy()
        assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("prec,flux", [(rts.RTS_FP64, False), (rts.RTS_FP32, False),
                                       (rts.RTS_FP32, True)])
def test_solve_for_adjoint_and_adjoint_from_solve_are_bitwise(prec, flux):
    # the forward that keeps D gives rts_solve's outputs (with the flux vector
    # too), and the adjoint that reads it gives rts_adjoint's gradients, bit
    # for bit; a second call of the backward on the same kept forward gives
    # them again
    import torch
    dt = np.float32 if prec == rts.RTS_FP32 else np.float64
    ps = [inputs.random_problem(30, 22, 15, seed=71, bands=2).astype(dt),
          inputs.random_problem(19, 27, 12, seed=72, bands=2).astype(dt)]
    pl = rts.Plan(ps, prec, flux=flux)
    ins = [pl.device_inputs(p) for p in ps]
    outs_a = [pl.new_outputs(p, want_flux=flux) for p in ps]
    outs_b = [pl.new_outputs(p, want_flux=flux) for p in ps]
    seeds, ga, gb = [], [], []
    for i, p in enumerate(ps):
        gQ, gJ, gI = _seeds(p, 80 + i)
        seeds.append((torch.as_tensor(gQ, device="cuda"),
                      torch.as_tensor(gJ.astype(dt), device="cuda"),
                      torch.as_tensor(gI.astype(dt), device="cuda")))
        ga.append((torch.empty(p.S.shape, dtype=pl.dtype, device="cuda"),
                   torch.empty(p.S.shape, dtype=pl.dtype, device="cuda")))
        gb.append((torch.empty(p.S.shape, dtype=pl.dtype, device="cuda"),
                   torch.empty(p.S.shape, dtype=pl.dtype, device="cuda")))
    print("case kept forward + adjoint", prec, flux, flush=True)
    pl.solve_into(ins, outs_a, batched=True)
    pl.adjoint_into(ins, seeds, ga)
    pl.solve_for_adjoint_into(ins, outs_b)
    for rep in range(2):
        pl.adjoint_from_solve_into(ins, seeds, gb)
        pl.check_status()
        torch.cuda.synchronize()
        for oa, ob in zip(outs_a, outs_b):
            for a, b in zip(oa, ob):
                assert torch.equal(a, b)
        for a2, b2 in zip(ga, gb):
            for a, b in zip(a2, b2):
                assert torch.equal(a, b), rep
