"""torch.autograd.Function around the hand-written adjoint.

forward() evaluates the objective and its gradient in one call of
air_objective_and_grad and keeps the gradient; backward() multiplies a copy
of the kept gradient by the incoming scalar with air_scale, so the kept
gradient is never changed (a second backward over a retained graph sees it
intact). PyTorch's tape never differentiates the registration itself (it
replaces the automatic differentiation of the paper's Sec. III-A with a
hand-written adjoint).
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import api


class ObjectiveFn(torch.autograd.Function):
    """L(theta) for a one-pair plan; fixed and moving are not differentiated."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, plan: api.Plan, fixed: torch.Tensor,
                moving: torch.Tensor) -> torch.Tensor:
        value, grad = api.objective_and_grad(plan, fixed, moving, theta.detach().contiguous())
        ctx.save_for_backward(grad)
        return value

    @staticmethod
    @once_differentiable
    def backward(ctx, grad_out: torch.Tensor):
        (grad,) = ctx.saved_tensors
        out = grad.clone()
        api.scale_(out, grad_out.detach().to(torch.float32).contiguous())
        return out, None, None, None


def objective(theta: torch.Tensor, plan: api.Plan, fixed: torch.Tensor,
              moving: torch.Tensor) -> torch.Tensor:
    return ObjectiveFn.apply(theta, plan, fixed, moving)
