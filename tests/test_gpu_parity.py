"""GPU parity: librts (through the C ABI) against the FP64 CPU oracle.

Tolerances (derived from the arithmetic):
* FP64 path vs oracle.  The library sweeps D = I - S, the oracle I; both
  round at ~1e-16 per operation.  J and I_top agree to a few 1e-15 relative.
  Q = 4 pi chi (J - S): the oracle forms J - S by subtraction, which loses
  up to 1e-16 * S absolutely, so the per-cell bound is
  |dQ| <= 1e-9 |Q| + 4 pi chi S * 1e-13.
* FP32 path vs oracle on the same (FP32-rounded) inputs: D is carried in
  FP32 (6e-8 per operation, transcendental ops ~1 ulp), accumulated with a
  compensated sum and reduced in FP64; we require max|dQ|/max|Q| <= 2e-5 and
  J, I_top within 2e-6 relative of max.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_08145_amd import inputs, rts
from percell import assert_paper_rule

pytestmark = pytest.mark.gpu


def _rand_problem(nx, ny, nz, seed, **kw):
    return inputs.random_problem(nx, ny, nz, seed, **kw)


def _check64(p, got, ref):
    Qg, Jg, Ig = got
    Qo, Jo, Io = ref
    chi = oracle.chi_of(p)
    floor = 4 * math.pi * (np.abs(chi) * np.abs(p.S)).max(axis=0) * 1e-13
    assert np.all(np.abs(Qg - Qo) <= 1e-9 * np.abs(Qo) + floor), np.abs(Qg - Qo).max()
    assert np.abs(Jg - Jo).max() <= 1e-13 * np.abs(Jo).max()
    assert np.abs(Ig - Io).max() <= 1e-13 * max(np.abs(Io).max(), 1e-300)


def _check32(p32, got, ref, q_tol=2e-5, j_tol=2e-6):
    # normwise bars, then the paper's per-value rule (relative 1e-5 or
    # absolute 1e-7 of the largest value) on every cell of Q, J and I_top
    Qg, Jg, Ig = got
    Qo, Jo, Io = ref
    eq = np.abs(Qg - Qo).max() / np.abs(Qo).max()
    ej = np.abs(Jg - Jo).max() / np.abs(Jo).max()
    ei = np.abs(Ig - Io).max() / max(np.abs(Io).max(), 1e-300)
    assert eq <= q_tol and ej <= j_tol and ei <= j_tol, (eq, ej, ei)
    for name, g, o in (("Q", Qg, Qo), ("J", Jg, Jo), ("I_top", Ig, Io)):
        assert_paper_rule(name, g, o)
    return eq, ej, ei


def test_grey32_fp64_matches_oracle():
    p = inputs.workload("grey32")
    print("case grey32 fp64", flush=True)
    got = rts.solve(p, rts.RTS_FP64)
    _check64(p, got, oracle.solve(p, threads=8))


def test_grey32_fp32_matches_oracle():
    p = inputs.workload("grey32").astype(np.float32)
    print("case grey32 fp32", flush=True)
    got = rts.solve(p, rts.RTS_FP32)
    eq, ej, ei = _check32(p, got, oracle.solve(p.astype(np.float64), threads=8))
    print(f"grey32 fp32: Q {eq:.2e} J {ej:.2e} I_top {ei:.2e}")


@pytest.mark.parametrize("shape", [(20, 13, 11), (130, 70, 9), (64, 7, 33), (2, 3, 2), (65, 64, 17)])
def test_ragged_shapes_fp64(shape):
    nx, ny, nz = shape
    p = _rand_problem(nx, ny, nz, seed=nx * 7 + ny)
    print("case ragged", shape, flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))


@pytest.mark.parametrize("shape", [(20, 13, 11), (130, 70, 9), (97, 33, 40)])
def test_ragged_shapes_fp32(shape):
    nx, ny, nz = shape
    p = _rand_problem(nx, ny, nz, seed=nx * 11 + nz).astype(np.float32)
    print("case ragged fp32", shape, flush=True)
    _check32(p, rts.solve(p, rts.RTS_FP32), oracle.solve(p.astype(np.float64), threads=8))


@pytest.mark.parametrize("bc", [(1, 1, 1.7, 3), (0, 1, 0.0, 1), (1, 0, 0.3, 4)])
def test_boundary_variants_and_iterations(bc):
    bot, top, ib, nit = bc
    p = _rand_problem(24, 20, 14, seed=5, bot=bot, top=top, i_bot=ib, n_iter=nit)
    print("case bc", bc, flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))


def test_general_directions_nonuniform_path():
    # dx = dy = 3 dz: every S4 ray is z-dominant with its own fractions, so
    # tasks are not uniform; plus two random directions leave slots unused
    p = _rand_problem(18, 16, 12, seed=9)
    p.dx = p.dy = 3.0
    r = np.random.default_rng(3)
    extra = r.standard_normal((2, 3))
    extra /= np.linalg.norm(extra, axis=1, keepdims=True)
    p.mu = np.vstack([p.mu, extra])
    p.w = np.concatenate([p.w * 0.9, [0.05, 0.05]])
    print("case general directions", flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))
    p32 = p.astype(np.float32)
    _check32(p32, rts.solve(p32, rts.RTS_FP32), oracle.solve(p32.astype(np.float64), threads=8))


def test_multiband_qweight():
    p = _rand_problem(26, 22, 15, seed=21, bands=3)
    p.qweight = np.array([1.0, 0.25, 0.0])
    print("case multiband", flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))


def test_isothermal_exact_on_gpu():
    p = _rand_problem(40, 36, 30, seed=2, lo=1e-3, hi=1e3)
    p.S = np.full_like(p.S, 2.5)
    p.top = inputs.TOP_THERMAL
    Q, J, I = rts.solve(p, rts.RTS_FP64)
    assert np.abs(J - 2.5).max() < 1e-13 and np.abs(I - 2.5).max() < 1e-13
    Q, J, I = rts.solve(p.astype(np.float32), rts.RTS_FP32)
    assert np.abs(J - 2.5).max() < 1e-5


def test_schedules_are_bitwise_identical():
    p = _rand_problem(70, 40, 37, seed=4).astype(np.float32)
    ref = None
    for h in (2, 4, 6, 8):
        pl = rts.Plan(p, rts.RTS_FP32)
        pl.set_schedule(rows_per_strip=h)
        got = rts.solve(p, rts.RTS_FP32, plan=pl)
        if ref is None:
            ref = got
        else:
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), h
    pl = rts.Plan(p, rts.RTS_FP32)
    pl.set_schedule(max_workgroups=7, order=1)
    got = rts.solve(p, rts.RTS_FP32, plan=pl)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_fp64_schedules_bitwise_and_repeatable():
    p = _rand_problem(33, 30, 19, seed=8)
    pl = rts.Plan(p, rts.RTS_FP64)
    a = rts.solve(p, rts.RTS_FP64, plan=pl)
    b = rts.solve(p, rts.RTS_FP64, plan=pl)
    pl.set_schedule(rows_per_strip=4)
    c = rts.solve(p, rts.RTS_FP64, plan=pl)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_batched_equals_single():
    import torch
    ps = [_rand_problem(40, 24, 18, seed=31, bands=2), _rand_problem(17, 33, 21, seed=32, bands=2)]
    ps = [p.astype(np.float32) for p in ps]
    pl = rts.Plan(ps, rts.RTS_FP32)
    ins = [pl.device_inputs(p) for p in ps]
    outs = [pl.new_outputs(p) for p in ps]
    for use_graph in (0, 1):
        pl.set_schedule(use_graph=use_graph)
        for rep in range(3):
            pl.solve_into(ins, outs, batched=True)
            pl.check_status()
            torch.cuda.synchronize()
            for p, o in zip(ps, outs):
                single = rts.solve(p, rts.RTS_FP32)
                for a, b in zip(o, single):
                    assert np.array_equal(a.double().cpu().numpy(), b), (use_graph, rep)


@pytest.mark.parametrize("extra", ["plain", "flux", "tol"])
def test_width_launches_equal_single_launch(extra):
    # sweep planes of 64 to 256 padded columns (nx != ny: one box has two
    # widths): one launch per width and one launch at the widest width give
    # the same bits, eagerly and in graph replays, and match the oracle
    import torch
    ps = [_rand_problem(130, 40, 20, seed=51, bands=2), _rand_problem(70, 200, 15, seed=52),
          _rand_problem(20, 17, 9, seed=53, bands=3)]
    if extra == "tol":
        ps = [inputs.random_problem(p.nx, p.ny, p.nz, seed=60 + i, lo=0.02, hi=0.5, n_iter=6,
                                    bands=p.nbands) for i, p in enumerate(ps)]
    ps = [p.astype(np.float32) for p in ps]
    flux = extra == "flux"
    tol = 1e30 if extra == "tol" else 0.0     # the first sweep meets it: one sweep each
    pl = rts.Plan(ps, rts.RTS_FP32, flux=flux, tol=tol)
    ins = [pl.device_inputs(p) for p in ps]
    res = {}
    for single in (0, 1):
        for use_graph in (0, 1):
            pl.set_schedule(single_launch=single, use_graph=use_graph)
            outs = [pl.new_outputs(p, want_flux=flux) for p in ps]
            for rep in range(2):
                print("case width launches", extra, single, use_graph, rep, flush=True)
                pl.solve_into(ins, outs, batched=True)
                pl.check_status()
                torch.cuda.synchronize()
                res[(single, use_graph, rep)] = [[t.double().cpu().numpy() for t in o]
                                                 for o in outs]
    first = res[(0, 0, 0)]
    for k, got in res.items():
        for g, f in zip(got, first):
            for a, b in zip(g, f):
                assert np.array_equal(a, b), k
    for p, g in zip(ps, first):
        q = p.astype(np.float64)
        if extra == "tol":
            q.n_iter = 1
        ref = oracle.flux(q, threads=8) if flux else oracle.solve(q, threads=8)
        _check32(p, g[:3], ref[:3])


def test_autotune_keeps_results():
    p = _rand_problem(70, 40, 37, seed=4).astype(np.float32)
    ref = rts.solve(p, rts.RTS_FP32)
    pl = rts.Plan(p, rts.RTS_FP32)
    ins = pl.device_inputs(p)
    outs = pl.new_outputs(p)
    chosen = pl.autotune([ins], [outs], reps=2)
    print("autotune chose", chosen, flush=True)
    assert chosen["rows_per_strip"] in (2, 4, 6, 8) and chosen["order"] in (0, 1)
    assert chosen["single_launch"] in (0, 1)    # planes of 128 and 64 columns: both tried
    assert pl.schedule() == chosen
    got = rts.solve(p, rts.RTS_FP32, plan=pl)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    # cached: a second plan of the same shape takes the same schedule without timing
    pl2 = rts.Plan(p, rts.RTS_FP32)
    assert pl2.autotune([ins], [outs], reps=1) == chosen


def test_autotune_persisted_cache(tmp_path, monkeypatch):
    # RTS_TUNE_CACHE names a file that is the cache: a tuning run appends one line
    # "<key> <rows> <order> <single_launch>"; a later call (a fresh plan, or another
    # process) whose key has a valid line applies it without timing
    import torch
    p = _rand_problem(52, 33, 21, seed=6).astype(np.float32)
    ref = rts.solve(p, rts.RTS_FP32)
    first = tmp_path / "a.txt"
    monkeypatch.setenv("RTS_TUNE_CACHE", str(first))
    pl = rts.Plan(p, rts.RTS_FP32)
    ins = pl.device_inputs(p)
    chosen = pl.autotune([ins], [pl.new_outputs(p)], reps=1)
    lines = first.read_text().splitlines()
    assert len(lines) == 1, lines
    key, *vals = lines[0].split(" ")
    assert key.startswith("gfx950") and [int(v) for v in vals] == [
        chosen["rows_per_strip"], chosen["order"], chosen["single_launch"]]
    # another file: a different valid schedule for this key, between lines to ignore
    h = 2 if chosen["rows_per_strip"] != 2 else 6
    second = tmp_path / "b.txt"
    text = "\n".join([f"{key} 5 0 0", "garbage", f"{key} {h} {1 - chosen['order']} 0",
                      f"{key}x 8 1 0", f"{key} 4 x 0"]) + "\n"
    second.write_text(text)
    monkeypatch.setenv("RTS_TUNE_CACHE", str(second))
    pl2 = rts.Plan(p, rts.RTS_FP32)
    outs = pl2.new_outputs(p)
    for t in outs:
        t.fill_(float("nan"))
    got = pl2.autotune([ins], [outs], reps=1)
    torch.cuda.synchronize()
    assert (got["rows_per_strip"], got["order"], got["single_launch"]) == (
        h, 1 - chosen["order"], 0)
    assert all(bool(torch.isnan(t).all()) for t in outs)   # applied without a timed call
    assert second.read_text() == text                       # a hit records nothing
    for a, b in zip(ref, rts.solve(p, rts.RTS_FP32, plan=pl2)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [rts.RTS_FP32, rts.RTS_FP64])
def test_input_check_finds_nonfinite_values(prec):
    # rts_check_inputs scans kappa, rho and S of every box (and eps of a scattering plan)
    import torch
    boxes = [_rand_problem(19, 11, 7, seed=21, bands=3), _rand_problem(9, 30, 12, seed=22),
             _rand_problem(33, 5, 9, seed=23, bands=2)]
    pl = rts.Plan(boxes, prec)
    ins = [pl.device_inputs(b) for b in boxes]
    print("case input check", prec, flush=True)
    big = 3e38 if prec == rts.RTS_FP32 else 1e308
    ins[1][2].view(-1)[5] = big                      # large and tiny finite values pass
    ins[1][2].view(-1)[6] = 1e-40 if prec == rts.RTS_FP32 else 1e-310
    pl.check_inputs(ins)
    rng = np.random.default_rng(5)
    for box, arr, val in ((2, 2, float("nan")), (0, 1, float("inf")), (1, 0, -float("inf")),
                          (2, 2, float("-nan")), (0, 0, float("nan"))):
        t = ins[box][arr].view(-1)
        for k in (int(rng.integers(t.numel())), t.numel() - 1):   # anywhere, and the last value
            keep = t[k].item()
            t[k] = val
            with pytest.raises(rts.RTSError) as e:
                pl.check_inputs(ins)
            assert e.value.status == rts.RTS_E_NONFINITE, (box, arr, k)
            t[k] = keep
            pl.check_inputs(ins)
    torch.cuda.synchronize()


def test_input_check_scans_eps_of_a_scattering_plan():
    import torch
    p = _rand_problem(8, 7, 6, seed=24)
    pl = rts.Plan(p, rts.RTS_FP64, gs_iter=2)
    kap, rho, S = pl.device_inputs(p)
    eps = torch.full(S.shape, 0.5, dtype=torch.float64, device="cuda")
    pl.check_inputs([(kap, rho, S, eps)])
    eps.view(-1)[100] = float("nan")
    with pytest.raises(rts.RTSError) as e:
        pl.check_inputs([(kap, rho, S, eps)])
    assert e.value.status == rts.RTS_E_NONFINITE


@pytest.mark.parametrize("rows", [4, 6, 8])
@pytest.mark.parametrize("shape", [(17, 5, 3), (9, 2, 7), (6, 3, 2)])
def test_tasks_with_fewer_rows_than_a_strip(rows, shape):
    # a task whose plane has fewer rows than the strip height is one strip of
    # all its rows (the x and y sweeps of a 3-layer box, the z sweeps of a box
    # 2 or 3 cells deep in y)
    p = _rand_problem(*shape, seed=rows + shape[2], bands=2, n_iter=2)
    p32 = p.astype(np.float32)
    pl = rts.Plan(p32, rts.RTS_FP32)
    pl.set_schedule(rows_per_strip=rows)
    print("case few rows", shape, rows, flush=True)
    _check32(p32, rts.solve(p32, rts.RTS_FP32, plan=pl), oracle.solve(p32.astype(np.float64)))
    if rows == 4:
        pl64 = rts.Plan(p, rts.RTS_FP64)
        pl64.set_schedule(rows_per_strip=4)
        _check64(p, rts.solve(p, rts.RTS_FP64, plan=pl64), oracle.solve(p))


def test_max_columns_and_extreme_opacity():
    # 1024 columns (the largest supported row), 16 + 1 threads' waves per strip;
    # opacities from 1e-6 (optically thin: x << 0.1, the series branch) to 1e4
    # (optically thick: e underflows to 0)
    p = _rand_problem(1024, 6, 5, seed=77, lo=1e-6, hi=1e4)
    print("case max columns", flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))
    p32 = p.astype(np.float32)
    _check32(p32, rts.solve(p32, rts.RTS_FP32), oracle.solve(p32.astype(np.float64), threads=8))


def test_many_bands_and_rays():
    # the largest band count (16) and a 64-ray quadrature of random directions
    r = np.random.default_rng(5)
    p = _rand_problem(12, 10, 9, seed=78, bands=16)
    mu = r.standard_normal((64, 3))
    mu[:, 2] = np.where(np.abs(mu[:, 2]) < 0.05, 0.3, mu[:, 2])
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    p.mu = mu
    p.w = np.full(64, 1 / 64)
    p.qweight = r.uniform(0, 1, 16)
    print("case 16 bands 64 rays", flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))


def test_axis_aligned_in_plane_components():
    # rays with a zero in-plane component (f = 0: the upwind point is on a
    # grid line) and exactly diagonal ones (ties of the dominant axis)
    p = _rand_problem(14, 12, 10, seed=79)
    s = 1 / math.sqrt(2)
    t = 1 / math.sqrt(3)
    p.mu = np.array([[0, 0, 1.0], [0, 0, -1.0], [s, 0, s], [0, -s, -s], [t, t, t], [-t, t, -t]])
    p.w = np.full(6, 1 / 6)
    print("case axis-aligned rays", flush=True)
    _check64(p, rts.solve(p, rts.RTS_FP64), oracle.solve(p, threads=8))
