"""Differentiation form: the MDC operator as a torch.autograd.Function.

U_b = P+_b R (time in, time out; Theory section, the operator of the
time-domain functional, applied as transform / per-frequency product /
inverse transform as in Appendix A) runs in `mdc_forward`; its backward is the
hand-written adjoint kernel `mdc_adjoint`, so any loss built in torch on U_b
(and the reciprocity preconditioner C_r below, or any preconditioner applied
in torch before it) differentiates through the library.  Only the batch indices are
saved for backward: the operator is linear in R, so neither R nor its spectra
are kept between forward and backward.
"""
from __future__ import annotations

import ctypes

import torch

from . import native

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


class Reciprocity(torch.autograd.Function):
    """C_r z = (z + z^T)/2 over (receiver, virtual source) by the library's kernel
    (mdd_reciprocity); C_r is self-adjoint, so its backward is the same kernel."""

    @staticmethod
    def forward(ctx, z: torch.Tensor):
        return _reciprocity(z)

    @staticmethod
    def backward(ctx, grad: torch.Tensor):
        return _reciprocity(grad)


def _reciprocity(z: torch.Tensor) -> torch.Tensor:
    if z.dim() != 3 or z.shape[0] != z.shape[1] or z.dtype != torch.float32 or not z.is_cuda:
        raise ValueError("reciprocity needs a float32 CUDA tensor [n][n][nt]")
    z = z.contiguous()
    out = torch.empty_like(z)
    lib = native.load()
    stream = torch.cuda.current_stream(z.device).cuda_stream
    native.check("mdd_reciprocity", lib.mdd_reciprocity(
        ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(out.data_ptr()), z.shape[0], z.shape[2],
        ctypes.c_void_p(stream)))
    return out


def reciprocity(z: torch.Tensor) -> torch.Tensor:
    """Reciprocity preconditioner C_r z = (z + z^T)/2 over (receiver, virtual source),
    in-graph (Theory section, preconditioned functional); self-adjoint."""
    return Reciprocity.apply(z)


class MDCRec(torch.autograd.Function):
    """U_b = P+_b C_r z in one operator (mdc_forward_rec); the backward is C_r P+_b^H
    (mdc_adjoint_rec).  The same value as mdc(reciprocity(z)), with C_r applied to the
    retained spectra inside the operator instead of to the traces."""

    @staticmethod
    def forward(ctx, z: torch.Tensor, idx: torch.Tensor, plan: Plan):
        ctx.plan = plan
        ctx.save_for_backward(idx)
        return plan.mdc_forward_rec(z.contiguous(), idx)

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        (idx,) = ctx.saved_tensors
        grad_z = None
        if ctx.needs_input_grad[0]:
            grad_z = ctx.plan.mdc_adjoint_rec(grad_u.contiguous(), idx)
        return grad_z, None, None


def mdc_rec(z: torch.Tensor, idx: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable U_b = P+_b C_r z (nr == nvs) for the batch `idx`."""
    return MDCRec.apply(z, idx, plan)
