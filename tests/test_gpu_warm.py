"""Warm start of the periodic boundary iteration (rts_inputs.ghost /
rts_outputs.ghost through the C ABI) against the FP64 oracle's solve_warm.

* The cold start's ghost planes given explicitly (I = S of each outflow plane,
  boundary layers at their values) reproduce the cold solve bitwise (the
  warm-start arithmetic is I - S = 0 exactly).
* From the ghost planes of another atmosphere (a 1 % perturbation of this
  one, converged): the result and the final ghost planes against the oracle
  started from the same planes: FP64 per cell as test_gpu_parity, FP32 within
  2e-5 / 2e-6 and the paper's per-value rule.
* Under a tolerance: tolerances whose oracle sweep counts are stable within
  +-10 % (as test_gpu_tol); a warm start from the previous atmosphere's planes
  takes fewer sweeps than a cold start in the oracle, and the GPU result
  matches the oracle's warm result (a different sweep count would differ by
  about tol).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_08145_amd import inputs, rts
from percell import assert_paper_rule

pytestmark = pytest.mark.gpu


def _pair(shape, seed, **kw):
    p = inputs.random_problem(*shape, seed=seed, lo=0.02, hi=0.5, **kw)
    prev = p.astype(np.float64)
    prev.S = p.S * (1 + 0.01 * np.random.default_rng(seed + 7).standard_normal(p.S.shape))
    return p, prev


def _check64(p, got, ref):
    chi = oracle.chi_of(p)
    floor = 4 * math.pi * (np.abs(chi) * np.abs(p.S)).max(axis=0) * 1e-13
    assert np.all(np.abs(got[0] - ref[0]) <= 1e-9 * np.abs(ref[0]) + floor)
    for g, o in zip(got[1:3], ref[1:3]):
        assert np.abs(g - o).max() <= 1e-13 * np.abs(o).max()


def _check32(got, ref):
    for name, g, o, bar in zip(("Q", "J", "I_top"), got[:3], ref[:3], (2e-5, 2e-6, 2e-6)):
        assert np.abs(g - o).max() <= bar * np.abs(o).max(), name
        assert_paper_rule(name, g, o)


@pytest.mark.parametrize("prec", [rts.RTS_FP64, rts.RTS_FP32])
def test_warm_start_cold_planes_equal_cold_solve(prec):
    p = inputs.random_problem(22, 17, 12, seed=801, bands=2)
    pp = p.astype(np.float32) if prec == rts.RTS_FP32 else p
    print("case warm cold planes", prec, flush=True)
    got = rts.solve_warm(pp, prec, ghost_in=_initial_ghost(pp))
    ref = rts.solve(pp, prec)
    for a, b in zip(got[:3], ref):
        assert np.array_equal(a, b)


def _initial_ghost(p):
    # I = S of each x or y dominant ray's outflow plane, boundary layers at
    # their values (thermal bottom: S; zero top: 0)
    M = max(p.nx, p.ny)
    g = np.zeros((p.nbands, p.nrays, p.nz, M))
    for r, m in enumerate(p.mu):
        s = [d / abs(c) if c != 0 else np.inf for d, c in zip((p.dx, p.dy, p.dz), m)]
        ax = max(a for a in range(3) if s[a] == min(s))
        if ax == 2:
            continue
        if ax == 0:
            plane = p.S[:, :, :, p.nx - 1 if m[0] > 0 else 0]
        else:
            plane = p.S[:, :, p.ny - 1 if m[1] > 0 else 0, :]
        w = plane.shape[2]
        g[:, r, :, :w] = plane
        if m[2] > 0:
            g[:, r, 0, :w] = plane[:, 0] if p.bot == 0 else p.i_bot
        else:
            g[:, r, -1, :w] = 0.0 if p.top == 0 else plane[:, -1]
    return g.astype(p.S.dtype)


@pytest.mark.parametrize("prec,shape", [(rts.RTS_FP64, (20, 17, 11)), (rts.RTS_FP32, (26, 19, 13))])
def test_warm_start_matches_oracle(prec, shape):
    p, prev = _pair(shape, 802, bands=2, n_iter=2)
    pp = p.astype(np.float32) if prec == rts.RTS_FP32 else p
    conv = prev.astype(np.float64)
    conv.n_iter = 60
    gin = oracle.solve_warm(conv)[3].astype(pp.S.dtype)
    print("case warm start", prec, shape, flush=True)
    got = rts.solve_warm(pp, prec, ghost_in=gin)
    ref = oracle.solve_warm(pp.astype(np.float64), gin.astype(np.float64))
    if prec == rts.RTS_FP64:
        _check64(pp, got, ref)
        assert np.abs(got[3] - ref[3]).max() <= 1e-13 * np.abs(ref[3]).max()
    else:
        _check32(got, ref)
        assert np.abs(got[3] - ref[3]).max() <= 2e-6 * np.abs(ref[3]).max()


def test_warm_start_saves_sweeps_under_tolerance():
    p, prev = _pair((24, 18, 12), 803, bands=2, n_iter=12)
    conv = prev.astype(np.float64)
    conv.n_iter = 60
    gin = oracle.solve_warm(conv)[3]
    tol = None
    for t in (1e-3, 3e-4, 1e-4, 3e-5):
        s = [oracle.solve_warm(p, gin, tol=x)[4] for x in (t, 0.9 * t, 1.1 * t)]
        c = oracle.solve_warm(p, None, tol=t)[4]
        if all(np.array_equal(s[0], x) for x in s[1:]) and s[0].sum() < c.sum() and s[0].max() > 1:
            tol, warm_sweeps, cold_sweeps = t, s[0], c
            break
    assert tol is not None, "no tolerance with stable, fewer warm sweeps"
    print("case warm tol", tol, warm_sweeps.sum(), cold_sweeps.sum(), flush=True)
    got = rts.solve_warm(p, rts.RTS_FP64, ghost_in=gin, tol=tol)
    ref = oracle.solve_warm(p, gin, tol=tol)
    _check64(p, got, ref)
    # and the ghost planes out are those of the oracle's last sweeps
    assert np.abs(got[3] - ref[3]).max() <= 1e-13 * np.abs(ref[3]).max()
