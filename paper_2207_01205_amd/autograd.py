"""torch.autograd binding of the FOFSE forward and adjoint kernels.

``fofse_extrapolate(areas, rho_gamma, plan, known)`` returns g on the missing
area of every block and records the selection; its backward runs the adjoint
kernel (``fofse_backward``) for that record, so gradients flow to the known
samples and to (rho_hat, gamma).  The selection itself is piecewise constant in
the inputs and is held fixed, as in any argmax-based model."""

from __future__ import annotations

import torch

from .fofse import Plan


class FofseExtrapolate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, areas, rho_gamma, plan: Plan, known=None):
        out, sel, coef, status = plan.extrapolate(areas.detach(), rho_gamma.detach(), known=known,
                                                  record=True, status=True)
        ctx.plan = plan
        ctx.known = known
        ctx.save_for_backward(areas.detach(), rho_gamma.detach(), sel, coef)
        ctx.mark_non_differentiable(status)
        return out, status

    @staticmethod
    def backward(ctx, grad_out, grad_status):
        areas, rho_gamma, sel, coef = ctx.saved_tensors
        need_f, need_p = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_f or need_p):
            return None, None, None, None
        ga, grg, _ = ctx.plan.backward(areas, rho_gamma, sel, coef,
                                       grad_out.to(torch.float32).contiguous(), known=ctx.known,
                                       grad_areas=need_f)
        return (ga if need_f else None), (grg if need_p else None), None, None


def fofse_extrapolate(areas: torch.Tensor, rho_gamma: torch.Tensor, plan: Plan, known=None):
    """Differentiable extrapolation: returns (g on B [n, nB] float32,
    per-block status [n] int32)."""
    return FofseExtrapolate.apply(areas, rho_gamma, plan, known)
