"""Differentiable dose operator: dose = K P^T p (Eq. 3) as a torch.autograd.Function.

Forward runs the HIP backprojector and blur; the hand-written backward is the
adjoint P K (Eq. 51 applies the same operator to the dual variables):

    grad_p = P (K grad_dose)        (K symmetric, so K^T = K)

The map is linear, so the backward keeps nothing from the forward: the
projector recomputes the Beer-Lambert factors of every (voxel, view) pair on
the fly, and memory use does not grow with the number of checkpointed calls.
"""
from __future__ import annotations

import torch

from .binding import Plan


class SipoDose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        d = plan.backproject(p.contiguous())
        return plan.blur(d) if plan.taps is not None else d

    @staticmethod
    def backward(ctx, grad_dose: torch.Tensor):
        plan = ctx.plan
        g = grad_dose.contiguous()
        if plan.taps is not None:
            g = plan.blur(g)
        return plan.project(g), None


def dose(p: torch.Tensor, plan: Plan) -> torch.Tensor:
    """dose = K P^T p for a sinogram-shaped projection p, differentiable in p."""
    return SipoDose.apply(p, plan)
