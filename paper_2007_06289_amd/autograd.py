"""Differentiable reconstruction: a torch.autograd.Function around the C ABI.

The forward pass is ``fbp_reconstruct`` (recursive ramp pair, then the transposed FHT of the
four classes and their sum).  Both stages are linear, so the backward pass is the adjoint chain:
the adjoint of the class sum and transposed FHT is the forward FHT of the image gradient on the
four classes (``fht_forward``), and the recursive pair with its row scale is self-adjoint (the
causal and anticausal recursions are each other's transpose, and the row scale is constant
along the row), so the same ``fbp_filter`` finishes the gradient.  Both run in the library's
HIP kernels.
"""
from __future__ import annotations

import torch

from . import api


class FBPReconstruct(torch.autograd.Function):
    """img = FBP(lino) with gradient d lino = filter(fht_forward(d img))."""

    @staticmethod
    def forward(ctx, lino: torch.Tensor, plan: "api.Plan") -> torch.Tensor:
        ctx.plan = plan
        return api.fbp_reconstruct(plan, lino.contiguous())

    @staticmethod
    def backward(ctx, grad_img: torch.Tensor):
        plan = ctx.plan
        g = api.fht_forward(plan, grad_img.contiguous())
        api.fbp_filter(plan, g, g)
        return g, None


def fbp_reconstruct_autograd(plan: "api.Plan", lino: torch.Tensor) -> torch.Tensor:
    """Differentiable ``fbp_reconstruct`` (gradient with respect to the linogram)."""
    return FBPReconstruct.apply(lino, plan)
