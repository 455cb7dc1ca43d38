"""rts_solve_static, the forward solve on the library's fixed device array
(for callers that cannot allocate), against rts_solve_batched on a caller's
workspace: the same plan and schedule give bitwise the same Q, J and I_top.
Two calls in a row on one array, the second on a smaller problem (the array
keeps the first call's contents), in both precisions and on a two-box plan."""
import numpy as np
import pytest

from paper_2107_08145_amd import inputs, rts

pytestmark = pytest.mark.gpu


def _plan_pair(problems, prec, dt):
    ps = [p.astype(dt) for p in problems]
    pl = rts.Plan(ps if len(ps) > 1 else ps[0], prec)
    assert pl.workspace_bytes(rts.RTS_OP_SOLVE) <= rts.RTS_STATIC_SCRATCH_BYTES
    ins = [pl.device_inputs(p) for p in ps]
    return ps, pl, ins


@pytest.mark.parametrize("prec,dt", [(rts.RTS_FP32, np.float32), (rts.RTS_FP64, np.float64)])
def test_static_solve_equals_workspace_solve(prec, dt):
    import torch
    # a larger problem first, then a smaller one: the second call must not
    # see the first call's exchange words, tickets or partials
    cases = [[inputs.random_problem(40, 36, 28, seed=701, bands=2)],
             [inputs.random_problem(20, 18, 13, seed=702, bands=1)],
             [inputs.random_problem(24, 24, 16, seed=703, bands=2),
              inputs.random_problem(17, 30, 9, seed=704, bands=1)]]
    for k, probs in enumerate(cases):
        print("case static solve", prec, k, [(p.nx, p.ny, p.nz, p.nbands) for p in probs],
              flush=True)
        ps, pl, ins = _plan_pair(probs, prec, dt)
        ref = [pl.new_outputs(p) for p in ps]
        pl.solve_into(ins, ref, batched=True)
        pl.check_status()
        got = [pl.new_outputs(p) for p in ps]
        for o in got:
            for t in o:
                t.fill_(-1.0)
        pl.solve_static_into(ins, got)
        pl.check_static_status()
        torch.cuda.synchronize()
        for b in range(len(ps)):
            for name, a, g in zip(("Q", "J", "I_top"), ref[b], got[b]):
                assert torch.equal(a, g), (k, b, name)
