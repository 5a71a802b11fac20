"""Wavespeed -> misfit as a torch.autograd.Function.

When the gradient is needed, the forward pass runs, per problem, the GPU forward
solve, the float64 misfit J (eq. l2error without a dt factor) and the fused adjoint
+ gradient sweep (eq. gradient3) in one call of kmv_misfit_gradient_accumulate,
which adds J and dJ/dc to running sums held on the device; the backward pass
returns grad_output * dJ/dc.  When it is not (no input requires a gradient, as in
a line-search or finite-difference probe under torch.no_grad), only the forward
solve and the misfit run (kmv_misfit).  Several shots (one Problem each, or
Problems holding several shots each) are summed.
"""
from __future__ import annotations

import torch


class FWIMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, problems, observed):
        total = 0.0
        if not ctx.needs_input_grad[0]:
            for prob, obs in zip(problems, observed):
                total += prob.misfit(c.detach(), obs)
            ctx.save_for_backward(None)
            return torch.tensor(total, dtype=torch.float64, device=c.device)
        grad = torch.zeros_like(c)
        for prob, obs in zip(problems, observed):
            total = prob.misfit_gradient_accumulate(c.detach(), obs, total, grad)
        ctx.save_for_backward(grad)
        return torch.tensor(total, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, grad_output):
        (grad,) = ctx.saved_tensors
        if grad is None:
            raise RuntimeError("FWIMisfit was evaluated without a gradient (no input required one)")
        return grad_output * grad, None, None


def fwi_misfit(c, problems, observed):
    """J(c) summed over shots; differentiable in c (float64 CUDA tensor)."""
    if not isinstance(problems, (list, tuple)):
        problems, observed = [problems], [observed]
    return FWIMisfit.apply(c, list(problems), list(observed))
