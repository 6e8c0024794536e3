"""Differentiable ICR sample s = L xi for PyTorch.

The backward of the forward sweep is the hand-written adjoint sweep (icr_adjoint),
so gradients with respect to xi come from the same HIP kernels. The matrices
(R, sqrtD, L00) are constants of the plan: no gradient flows to the kernel's
hyperparameters.
"""

from __future__ import annotations

import torch

from .icr import Plan, icr_adjoint, icr_forward


class ICRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return icr_forward(plan, xi.contiguous())

    @staticmethod
    def backward(ctx, grad_s: torch.Tensor):
        return icr_adjoint(ctx.plan, grad_s.contiguous()), None


def icr_sample(plan: Plan, xi: torch.Tensor) -> torch.Tensor:
    """s = L xi with autograd support (gradient with respect to xi)."""
    return ICRFunction.apply(xi, plan)
