"""Wavespeed -> misfit as a torch.autograd.Function.

The forward pass runs the GPU forward solve, the float64 misfit J (eq. l2error
without a dt factor) and the fused adjoint + gradient sweep (eq. gradient3) in one
call of kmv_misfit_gradient, and keeps dJ/dc for the backward pass, which returns
grad_output * dJ/dc.  Several shots (one Problem each, or Problems holding several
shots each) are summed.
"""
from __future__ import annotations

import torch


class FWIMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, problems, observed):
        total = 0.0
        grad = torch.zeros_like(c)
        for prob, obs in zip(problems, observed):
            J, g, _ = prob.misfit_gradient(c.detach(), obs)
            total += J
            grad += g
        ctx.save_for_backward(grad)
        return torch.tensor(total, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, grad_output):
        (grad,) = ctx.saved_tensors
        return grad_output * grad, None, None


def fwi_misfit(c, problems, observed):
    """J(c) summed over shots; differentiable in c (float64 CUDA tensor)."""
    if not isinstance(problems, (list, tuple)):
        problems, observed = [problems], [observed]
    return FWIMisfit.apply(c, list(problems), list(observed))
