"""torch.autograd binding of the librts forward solve and its adjoint.

`rts_apply(kappa, rho, S, plan)` returns (Q, J, I_top) of one box.  When any
input requires a gradient the forward is `rts_solve_for_adjoint` on a private
adjoint workspace (it keeps D of every plane, as a tape keeps activations)
and the backward is `rts_adjoint_from_solve` on that workspace: the
transposed recursion swept in reverse, giving dL/dS and dL/dchi,
chi = kappa rho.  Each call owns its workspace, so several graphs may be in
flight.  The chain rule to the caller's inputs is
dL/dkappa_b = rho dL/dchi_b and dL/drho = sum_b kappa_b dL/dchi_b.

Argument marshalling only: every step runs in librts (no CPU fallback).
"""
from __future__ import annotations

import torch

from . import rts


def _dev(t, dtype):
    return None if t is None else t.to(device="cuda", dtype=dtype).contiguous()


class RTSFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, rho, S, plan):
        p = plan.problems[0]
        dt = plan.dtype
        ins = (_dev(kappa, dt), _dev(rho, dt), _dev(S, dt))
        Q, J, It = plan.new_outputs(p)
        if any(ctx.needs_input_grad[:3]):
            ws_t, w, nbytes = plan.adjoint_workspace()
            plan.solve_for_adjoint_into([ins], [(Q, J, It)], ws=(w, nbytes))
            # the status word of the private workspace (a neighbour-wait
            # timeout leaves partial outputs): checked before anything reads them
            plan.check_status(ws=w)
            ctx.ws = (ws_t, w, nbytes)
        else:
            plan.solve_into([ins], [(Q, J, It)])
            plan.check_status()
        ctx.plan = plan
        ctx.save_for_backward(*ins)
        return Q, J, It

    @staticmethod
    def backward(ctx, gQ, gJ, gIt):
        plan = ctx.plan
        kappa, rho, S = ctx.saved_tensors
        dt = plan.dtype
        dS = torch.empty_like(S)
        dchi = torch.empty_like(S)
        seeds = (_dev(gQ, torch.float64), _dev(gJ, dt), _dev(gIt, dt))
        ws_t, w, nbytes = ctx.ws
        plan.adjoint_from_solve_into([(kappa, rho, S)], [seeds], [(dS, dchi)], ws=(w, nbytes))
        plan.check_status(ws=w)
        del ctx.ws
        dkappa = dchi * rho.unsqueeze(0) if ctx.needs_input_grad[0] else None
        drho = (dchi * kappa).sum(0) if ctx.needs_input_grad[1] else None
        return dkappa, drho, (dS if ctx.needs_input_grad[2] else None), None


def rts_apply(kappa: torch.Tensor, rho: torch.Tensor, S: torch.Tensor, plan: "rts.Plan"):
    """(Q [nz,ny,nx] float64, J [B,nz,ny,nx], I_top [B,n_up,ny,nx]) of the plan's box,
    differentiable in kappa [B,nz,ny,nx], rho [nz,ny,nx] and S [B,nz,ny,nx]."""
    if len(plan.problems) != 1:
        raise ValueError("rts_apply takes a single-box plan")
    return RTSFunction.apply(kappa, rho, S, plan)
