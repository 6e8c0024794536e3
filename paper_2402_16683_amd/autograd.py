"""Differentiable ICR sample s = L xi for PyTorch.

The backward of the forward sweep is the hand-written adjoint sweep (icr_adjoint),
so gradients with respect to xi come from the same HIP kernels. icr_sample treats
the matrices (R, sqrtD, L00) as constants of the plan. icr_sample_hyper also returns
gradients with respect to the kernel's scale and length scale (a tensor theta that
must hold the plan's values), through icr_hyper_grad and the FP64 length derivatives
of a plan built with hypergrad=True; a new theta needs a new plan.
"""

from __future__ import annotations

import torch

from .icr import Plan, icr_adjoint, icr_forward, icr_hyper_grad, workspace_for


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


class ICRHyperFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi: torch.Tensor, theta: torch.Tensor, plan: Plan) -> torch.Tensor:
        scale, length = (float(v) for v in theta.detach().cpu().tolist())
        if abs(scale - plan.cfg.scale) > 1e-12 * abs(plan.cfg.scale) or \
                abs(length - plan.cfg.length) > 1e-12 * abs(plan.cfg.length):
            raise ValueError("theta must hold the plan's (scale, length)")
        xi = xi.contiguous()
        batch = 1 if xi.dim() == 1 else xi.shape[0]
        ws = workspace_for(plan, batch)
        s = icr_forward(plan, xi, workspace=ws)
        ctx.plan = plan
        ctx.theta_dtype = theta.dtype
        ctx.save_for_backward(xi, s, ws)
        return s

    @staticmethod
    def backward(ctx, grad_s: torch.Tensor):
        xi, s, ws = ctx.saved_tensors
        grad_s = grad_s.contiguous()
        batch = 1 if xi.dim() == 1 else xi.shape[0]
        ws_a = workspace_for(ctx.plan, batch)
        grad_xi = icr_adjoint(ctx.plan, grad_s, workspace=ws_a)
        g = icr_hyper_grad(ctx.plan, xi, s, ws, grad_s, ws_a)
        return grad_xi, g.sum(dim=0).to(ctx.theta_dtype).cpu(), None


def icr_sample_hyper(plan: Plan, xi: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """s = L(theta) xi with gradients for xi and theta = (scale, length) (a CPU tensor)."""
    return ICRHyperFunction.apply(xi, theta, plan)

