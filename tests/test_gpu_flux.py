"""GPU radiative flux vector F = sum_b qweight_b 4 pi sum_r w_r mu_r I_r and its
divergence heating QF = -div F (rts_solve / rts_solve_batched through the C
ABI with a flux plan) against the FP64 CPU oracle.

Tolerances (derived from the arithmetic):
* F: |F| <= 4 pi max I, and the GPU forms it from the same intensities as J,
  so its error is bounded by the J bar times 4 pi max|J|: 1e-13 (FP64) and
  2e-6 (FP32, FP32 state along the sweep and FP32 sums over a task's four
  rays) of 4 pi max|J|.
* QF: each derivative combines F values with coefficients whose magnitudes
  sum to 4 / delta at most (the one-sided second-order differences), so
  |dQF| <= (4/dx + 4/dy + 4/dz) * (the F bound).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_08145_amd import inputs, rts
from percell import assert_paper_rule

pytestmark = pytest.mark.gpu


def _check(p, got, ref, rel):
    Qg, Jg, Ig, Fg, QFg = got
    Qo, Jo, Io, Fo, QFo = ref
    if rel > 1e-10:  # FP32: the paper's per-value rule on Q, J and I_top
        for name, g, o in (("Q", Qg, Qo), ("J", Jg, Jo), ("I_top", Ig, Io)):
            assert_paper_rule(name, g, o)
    scale = 4 * math.pi * np.abs(Jo).max()
    ef = np.abs(Fg - Fo).max()
    eqf = np.abs(QFg - QFo).max()
    fbound = rel * scale
    qbound = (4 / p.dx + 4 / p.dy + 4 / p.dz) * fbound
    assert ef <= fbound, (ef, fbound)
    assert eqf <= qbound, (eqf, qbound)
    return ef / scale, eqf / max(np.abs(QFo).max(), 1e-300)


@pytest.mark.parametrize("case", [
    dict(nx=20, ny=13, nz=11, seed=1),
    dict(nx=33, ny=17, nz=2, seed=2),                      # two layers: first-order ends
    dict(nx=24, ny=30, nz=19, seed=3, bands=3, qweight=np.array([1.0, 0.5, 0.0])),
    dict(nx=18, ny=16, nz=12, seed=4, bot=1, top=1, i_bot=2.5, n_iter=2),
])
def test_flux_fp64_matches_oracle(case):
    c = dict(case)
    shape = (c.pop("nx"), c.pop("ny"), c.pop("nz"))
    seed, bands = c.pop("seed"), c.pop("bands", 1)
    p = inputs.random_problem(*shape, seed=seed, bands=bands, **c)
    p.dz = 0.7                                            # uneven spacing
    print("case flux fp64", shape, seed, flush=True)
    got = rts.solve(p, rts.RTS_FP64, flux=True)
    ref = oracle.flux(p, threads=8)
    ef, eq = _check(p, got, ref, 1e-13)
    print(f"flux fp64 {shape}: F {ef:.2e}, QF {eq:.2e}")


def test_flux_general_directions_fp32():
    r = np.random.default_rng(7)
    p = inputs.random_problem(26, 22, 15, seed=8, bands=2)
    mu = r.standard_normal((10, 3))
    mu[:, 2] = np.where(np.abs(mu[:, 2]) < 0.1, 0.4, mu[:, 2])
    p.mu = mu / np.linalg.norm(mu, axis=1, keepdims=True)
    p.w = r.random(10)
    p.w /= p.w.sum()
    p32 = p.astype(np.float32)
    print("case flux fp32 random directions", flush=True)
    got = rts.solve(p32, rts.RTS_FP32, flux=True)
    ref = oracle.flux(p32.astype(np.float64), threads=8)
    ef, eq = _check(p32, got, ref, 2e-6)
    print(f"flux fp32 random directions: F {ef:.2e}, QF {eq:.2e}")


def test_flux_leaves_q_j_itop_bitwise_unchanged():
    p = inputs.random_problem(40, 36, 21, seed=12, bands=2).astype(np.float32)
    print("case flux on/off", flush=True)
    plain = rts.solve(p, rts.RTS_FP32)
    with_flux = rts.solve(p, rts.RTS_FP32, flux=True)
    for a, b in zip(plain, with_flux[:3]):
        assert np.array_equal(a, b)


def test_flux_batched_and_graph_replays():
    import torch
    ps = [inputs.random_problem(40, 24, 18, seed=31, bands=2).astype(np.float32),
          inputs.random_problem(17, 33, 21, seed=32, bands=2).astype(np.float32)]
    refs = [oracle.flux(p.astype(np.float64), threads=8) for p in ps]
    pl = rts.Plan(ps, rts.RTS_FP32, flux=True)
    ins = [pl.device_inputs(p) for p in ps]
    outs = [pl.new_outputs(p, want_flux=True) for p in ps]
    first = None
    for use_graph in (0, 1):
        pl.set_schedule(use_graph=use_graph)
        for rep in range(3):
            print("case flux batched", use_graph, rep, flush=True)
            pl.solve_into(ins, outs, batched=True)
            pl.check_status()
            torch.cuda.synchronize()
            got = [[t.double().cpu().numpy() for t in o] for o in outs]
            for p, g, ref in zip(ps, got, refs):
                _check(p, g, ref, 2e-6)
            if first is None:
                first = got
            for g, f in zip(got, first):
                for a, b in zip(g, f):
                    assert np.array_equal(a, b), (use_graph, rep)


def test_flux_on_one_box_of_two():
    # a plan whose second box has no flux partials: the flux launch must leave
    # that box's results as in a plain solve
    import torch
    ps = [inputs.random_problem(30, 20, 14, seed=41, bands=2).astype(np.float32),
          inputs.random_problem(22, 26, 12, seed=42, bands=2).astype(np.float32)]
    pl = rts.Plan(ps, rts.RTS_FP32, flux=[True, False])
    ins = [pl.device_inputs(p) for p in ps]
    outs = [pl.new_outputs(ps[0], want_flux=True), pl.new_outputs(ps[1])]
    print("case flux on one box of two", flush=True)
    pl.solve_into(ins, outs, batched=True)
    pl.check_status()
    torch.cuda.synchronize()
    got0 = [t.double().cpu().numpy() for t in outs[0]]
    _check(ps[0], got0, oracle.flux(ps[0].astype(np.float64), threads=8), 2e-6)
    plain = rts.solve(ps[1], rts.RTS_FP32)
    for a, b in zip(outs[1], plain):
        assert np.array_equal(a.double().cpu().numpy(), b)


@pytest.mark.parametrize("prec", [rts.RTS_FP64, rts.RTS_FP32])
def test_flux_mixed_uniform_and_general_tasks(prec):
    # S4 without one ray: one three-ray task, the others four-ray tasks whose
    # rays share |mu| (two flux partials, the plane-axis one from the partial
    # sum) swept by the kernel for general tasks
    p = inputs.random_problem(22, 19, 13, seed=61, bands=2)
    p.mu = np.delete(p.mu, 5, axis=0)
    p.w = np.delete(p.w, 5)
    p.w = p.w / p.w.sum()
    pp = p.astype(np.float32) if prec == rts.RTS_FP32 else p
    print("case flux mixed tasks", prec, flush=True)
    got = rts.solve(pp, prec, flux=True)
    ref = oracle.flux(pp.astype(np.float64), threads=8)
    ef, eq = _check(pp, got, ref, 1e-13 if prec == rts.RTS_FP64 else 2e-6)
    print(f"flux mixed tasks {prec}: F {ef:.2e}, QF {eq:.2e}")
