"""Differentiation form: the MDC operator as a torch.autograd.Function.

U_b = P+_b R (time in, time out; Theory section, the operator of the
time-domain functional, applied as transform / per-frequency product /
inverse transform as in Appendix A) runs in `mdc_forward`; its backward is the
hand-written adjoint kernel `mdc_adjoint`, so any loss built in torch on U_b
(and any preconditioner applied in torch before it, e.g. reciprocity
(z + z^T)/2) differentiates through the library.  Only the batch indices are
saved for backward: the operator is linear in R, so neither R nor its spectra
are kept between forward and backward.
"""
from __future__ import annotations

import torch

from .plan import Plan


class MDC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, R: torch.Tensor, idx: torch.Tensor, plan: Plan):
        ctx.plan = plan
        ctx.save_for_backward(idx)
        return plan.mdc_forward(R.contiguous(), idx)

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        (idx,) = ctx.saved_tensors
        grad_r = None
        if ctx.needs_input_grad[0]:
            grad_r = ctx.plan.mdc_adjoint(grad_u.contiguous(), idx)
        return grad_r, None, None


def mdc(R: torch.Tensor, idx: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable U_b = P+_b R for the batch `idx` (int32 device tensor)."""
    return MDC.apply(R, idx, plan)


def reciprocity(z: torch.Tensor) -> torch.Tensor:
    """Reciprocity preconditioner C_r z = (z + z^T)/2 over (receiver, virtual source),
    in-graph (Theory section, preconditioned functional); self-adjoint."""
    return 0.5 * (z + z.transpose(0, 1))
