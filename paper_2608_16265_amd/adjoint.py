"""Differentiation with respect to the model parameters (binding only).

:class:`LagrangianGradient` is a ``torch.autograd.Function`` mapping the
parameter vector theta of a parametric NLP (eq. nlp) to the Lagrangian
gradient

    F(theta) = grad_x L(x, y; theta) = sigma grad_x f(x; theta) + J(x; theta)^T y

at fixed (x, y, sigma).  Its forward runs exa_lag_grad (the gradient and
J^T y terms and their sum, in the library's kernels); its backward runs the
hand-written adjoint kernel exa_adjoint_theta, which returns
(dF/dtheta)^T w from the mixed second derivatives of every pattern
instance.
"""
from __future__ import annotations

import torch

from .model import ExaModel


class LagrangianGradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, model: ExaModel, x: torch.Tensor, y: torch.Tensor,
                sigma: float):
        theta_c = theta.detach().contiguous()
        model.set_theta(theta_c)
        out = model.lag_grad(x, y, float(sigma))
        ctx.model, ctx.sigma = model, float(sigma)
        ctx.save_for_backward(theta_c, x, y)
        return out

    @staticmethod
    def backward(ctx, w: torch.Tensor):
        theta, x, y = ctx.saved_tensors
        model = ctx.model
        model.set_theta(theta)  # the model may have been used with another theta meanwhile
        tbar = model.adjoint_theta(x, y, ctx.sigma, w.contiguous())
        return tbar, None, None, None, None


def lagrangian_gradient(theta, model, x, y, sigma=1.0):
    """grad_x L as a differentiable function of theta."""
    return LagrangianGradient.apply(theta, model, x, y, sigma)
