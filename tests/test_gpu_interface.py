"""GPU tests of the call interface: general quadrature weights, the task
table upload on re-used workspace addresses, status checks of the autograd
binding's private workspaces, and graph-replayed calls with device timing.

Bars as in test_gpu_parity / test_gpu_adjoint (FP64 per cell against the
oracle, FP32 within 2e-5 of max|Q|, adjoint FP64 1e-10 of max per array);
graph replays and repeated autograd steps are compared bit for bit with
eager calls (the same kernels on the same data).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2107_08145_amd import inputs, rts

pytestmark = pytest.mark.gpu


def _weighted(p, seed):
    # positive weights that do not sum to 1 (J = sum_r w_r I_r as written)
    p.w = p.w * (0.9 + 0.6 * np.random.default_rng(seed).random(p.nrays))
    assert abs(p.w.sum() - 1) > 1e-2
    return p


def test_weights_not_summing_to_one_forward():
    p = _weighted(inputs.random_problem(23, 17, 14, seed=301, bands=2), 302)
    p.qweight = np.array([1.0, 0.5])
    print("case general weights fp64", flush=True)
    Qg, Jg, Ig = rts.solve(p, rts.RTS_FP64)
    Qo, Jo, Io = oracle.solve(p, threads=8)
    chi = oracle.chi_of(p)
    floor = 4 * math.pi * (np.abs(chi) * np.abs(p.S)).max(axis=0) * 1e-13
    assert np.all(np.abs(Qg - Qo) <= 1e-9 * np.abs(Qo) + floor)
    assert np.abs(Jg - Jo).max() <= 1e-13 * np.abs(Jo).max()
    assert np.abs(Ig - Io).max() <= 1e-13 * np.abs(Io).max()
    print("case general weights fp32", flush=True)
    p32 = p.astype(np.float32)
    Qf, Jf, If = rts.solve(p32, rts.RTS_FP32)
    Qo, Jo, Io = oracle.solve(p32.astype(np.float64), threads=8)
    assert np.abs(Qf - Qo).max() <= 2e-5 * np.abs(Qo).max()
    assert np.abs(Jf - Jo).max() <= 2e-6 * np.abs(Jo).max()


@pytest.mark.parametrize("prec", [rts.RTS_FP64, rts.RTS_FP32])
def test_weights_not_summing_to_one_adjoint(prec):
    p = _weighted(inputs.random_problem(20, 18, 12, seed=303, bands=2), 304)
    p.qweight = np.array([0.75, 1.0])
    pp = p.astype(np.float32) if prec == rts.RTS_FP32 else p
    r = np.random.default_rng(305)
    gQ = r.standard_normal((p.nz, p.ny, p.nx))
    gJ = r.standard_normal(p.S.shape).astype(pp.S.dtype)
    gI = r.standard_normal((p.nbands, p.n_up, p.ny, p.nx)).astype(pp.S.dtype)
    print("case general weights adjoint", prec, flush=True)
    got = rts.adjoint(pp, prec, gQ, gJ, gI)
    ref = oracle.adjoint(pp.astype(np.float64), gQ, gJ.astype(np.float64), gI.astype(np.float64),
                         threads=8)
    tol = 1e-10 if prec == rts.RTS_FP64 else 2e-4
    for g, o in zip(got, ref):
        for b in range(o.shape[0]):
            assert np.abs(g[b] - o[b]).max() <= tol * np.abs(o[b]).max(), b


def test_autograd_steps_with_reused_workspace_address():
    # Two training steps: between them a large temporary is written and
    # freed, so that the caching allocator hands the private adjoint
    # workspace's block out again with other contents.  The second step's
    # outputs and gradients equal the first's bit for bit.
    import torch
    from paper_2107_08145_amd.autograd import rts_apply
    p = inputs.random_problem(24, 20, 14, seed=311, bands=2)
    pl = rts.Plan(p, rts.RTS_FP64)
    r = np.random.default_rng(312)
    gQ = torch.tensor(r.standard_normal((p.nz, p.ny, p.nx)), device="cuda")
    res = []
    for step in range(2):
        print("case autograd step", step, flush=True)
        k = torch.tensor(p.kappa, device="cuda", requires_grad=True)
        rho = torch.tensor(p.rho, device="cuda", requires_grad=True)
        S = torch.tensor(p.S, device="cuda", requires_grad=True)
        Q, J, It = rts_apply(k, rho, S, pl)
        (Q * gQ).sum().backward()
        res.append([t.detach().clone() for t in (Q, J, It, k.grad, rho.grad, S.grad)])
        del Q, J, It, k, rho, S
        junk = torch.full((pl.workspace_bytes(rts.RTS_OP_ADJOINT) // 8 + 4096,), 7.0,
                          dtype=torch.float64, device="cuda")
        junk.mul_(3.0)
        torch.cuda.synchronize()
        del junk
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_graph_replays_with_timing_equal_eager():
    # rts_solve honours use_graph; timed replays record the sweep through
    # event-record nodes.  Every replay (with eager work and synchronisation
    # in between) equals the eager result bit for bit.
    import torch
    for prec, dt in ((rts.RTS_FP32, np.float32), (rts.RTS_FP64, np.float64)):
        p = inputs.random_problem(40, 33, 21, seed=321, bands=2).astype(dt)
        pl = rts.Plan(p, prec)
        ins = pl.device_inputs(p)
        ref = pl.new_outputs(p)
        pl.solve_into([ins], [ref])
        pl.check_status()
        torch.cuda.synchronize()
        pl.set_schedule(use_graph=1)
        outs = pl.new_outputs(p)
        for timing in (False, True):
            pl.enable_timing(timing)
            for rep in range(3):
                print("case graph replay", prec, timing, rep, flush=True)
                for o in outs:
                    o.fill_(-1.0)
                pl.solve_into([ins], [outs])
                pl.check_status()
                torch.cuda.synchronize()
                for a, b in zip(ref, outs):
                    assert torch.equal(a, b), (timing, rep)
            if timing:
                sweep_ms, call_ms = pl.last_timing()
                assert 0 < sweep_ms <= call_ms, (sweep_ms, call_ms)
        pl.enable_timing(False)
