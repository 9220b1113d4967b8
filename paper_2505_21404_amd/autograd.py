"""torch.autograd.Function of the residual map r(theta) (Section 2.2).

forward: r = r(theta) (dngd_residual_jacobian with J = NULL).
backward: theta_bar = J^T r_bar by the reverse pass over the stored
activations (dngd_vjp): J is never formed, so the memory is that of the
activations, not m x n. The gradient of the PINN loss L = 0.5 ||r||^2 is
J^T r.
"""
from __future__ import annotations

import torch

from . import dngd as D


class ResidualFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, prob: "D.Problem"):
        th = theta.detach().to(torch.float64).contiguous()
        ctx.prob = prob
        ctx.save_for_backward(th)
        return prob.residual(th)

    @staticmethod
    def backward(ctx, r_bar: torch.Tensor):
        (th,) = ctx.saved_tensors
        g = ctx.prob.vjp(th, r_bar.detach().to(torch.float64).contiguous())
        return g.to(r_bar.dtype), None


def residual(prob: "D.Problem", theta: torch.Tensor) -> torch.Tensor:
    """r(theta) with a hand-written backward (theta_bar = J^T r_bar)."""
    return ResidualFunction.apply(theta, prob)


def loss(prob: "D.Problem", theta: torch.Tensor) -> torch.Tensor:
    """L(theta) = 0.5 ||r(theta)||^2; its gradient is J^T r."""
    r = residual(prob, theta)
    return 0.5 * (r * r).sum()
