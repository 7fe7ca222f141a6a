"""Differentiation through the double FFT filter.

The filter F = Phi o Theta is linear, and each pass is a real symmetric
operator (a block-diagonal set of real circulants, conjugated by the
pole-extension permutation for Theta), so the vector-Jacobian product of F is
F^T = Theta o Phi: the library's adjoint call.  Nothing needs to be saved for
the backward.

filter_chain applies y_{k+1} = tanh(F y_k) K times, optionally under
activation checkpointing (each application's input is kept; the forward of
that segment is recomputed during the backward).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint as _checkpoint

from .filter import Plan


class SphFilter(torch.autograd.Function):
    """y = F x on the GPU; the backward applies F^T through the adjoint kernels."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.apply(x.contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        return ctx.plan.apply_adjoint(grad_out.contiguous()), None


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
