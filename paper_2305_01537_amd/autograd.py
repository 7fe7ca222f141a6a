"""Differentiation through the double FFT filter.

The filter F = Phi o Theta is linear, and each pass is a real symmetric
operator (a block-diagonal set of real circulants, conjugated by the
pole-extension permutation for Theta), so the vector-Jacobian product of F is
F^T = Theta o Phi: the library's adjoint call.  Nothing needs to be saved for
the backward -- except with hybrid fields, whose per-line choice between the
Gaussian and the exponential filter depends on the data: the forward records
the choices and the backward applies the transpose of the filter with those
choices frozen (the filter is piecewise linear in its input).

filter_chain applies y_{k+1} = tanh(F y_k) K times, optionally under
activation checkpointing (each application's input is kept; the forward of
that segment is recomputed during the backward).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint as _checkpoint

from .filter import Plan


def _aligned(t: torch.Tensor) -> torch.Tensor:
    """A contiguous tensor whose data starts on a 16-byte boundary, as the
    library requires: a copy only for a view that starts mid-way."""
    t = t.contiguous()
    return t if t.data_ptr() % 16 == 0 else t.clone()


class SphFilter(torch.autograd.Function):
    """y = F x on the GPU; the backward applies F^T through the adjoint kernels."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        x = _aligned(x)
        if plan.has_hybrid:
            th, ph = plan.decision_buffers(x.device)
            y = plan.apply_ex(x, theta_dec=th, phi_dec=ph, replay=False)
            ctx.save_for_backward(th, ph)
            return y
        return plan.apply(x)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = _aligned(grad_out)
        if ctx.plan.has_hybrid:
            th, ph = ctx.saved_tensors
            return ctx.plan.apply_ex(g, adjoint=True, theta_dec=th, phi_dec=ph, replay=True), None
        return ctx.plan.apply_adjoint(g), None


def sph_filter(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    return SphFilter.apply(x, plan)


def _step(y: torch.Tensor, plan: Plan) -> torch.Tensor:
    return torch.tanh(SphFilter.apply(y, plan))


def filter_chain(x: torch.Tensor, plan: Plan, K: int, checkpoint: bool = True) -> torch.Tensor:
    """y_K with y_0 = x and y_{k+1} = tanh(F y_k)."""
    y = x
    for _ in range(int(K)):
        if checkpoint and torch.is_grad_enabled():
            y = _checkpoint(_step, y, plan, use_reentrant=False)
        else:
            y = _step(y, plan)
    return y
