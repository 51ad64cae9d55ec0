"""Differentiable forward projector: the Siddon projector as a ``torch.autograd.Function`` whose
backward pass is the library's exact transpose (CT_BP_ADJOINT), so gradients of losses of A x are
exact up to FP32 rounding.  Both passes run on torch's current stream.
"""
from __future__ import annotations

import torch

from .operators import Plan


class SiddonProjection(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan):
        ctx.plan = plan
        return plan.forward(x.contiguous(), "siddon", out_dtype=torch.float32)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        gx = ctx.plan.backproject(g.contiguous().float(), "adjoint", out_dtype=torch.float32)
        return gx, None


def project(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    """A x with a hand-written backward A^T g."""
    return SiddonProjection.apply(x, plan)
