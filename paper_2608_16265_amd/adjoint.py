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
from .batch import ExaBatch


class LagrangianGradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, model: ExaModel, x: torch.Tensor, y: torch.Tensor,
                sigma: float):
        # the backward differentiates with respect to theta only: (x, y) are
        # held fixed, so a graph that needs their gradients is refused here
        # rather than given silent zeros
        if (isinstance(x, torch.Tensor) and x.requires_grad) or (isinstance(y, torch.Tensor) and y.requires_grad):
            raise NotImplementedError("LagrangianGradient differentiates with respect to theta only; "
                                      "x and y must not require grad")
        theta_c = theta.detach().contiguous()
        model.set_theta(theta_c)
        out = model.lag_grad(x, y, float(sigma))
        ctx.model, ctx.sigma = model, float(sigma)
        ctx.save_for_backward(theta_c, x, y)
        return out

    @staticmethod
    def backward(ctx, w: torch.Tensor):
        if any(ctx.needs_input_grad[1:]):
            raise NotImplementedError("LagrangianGradient differentiates with respect to theta only")
        theta, x, y = ctx.saved_tensors
        model = ctx.model
        model.set_theta(theta)  # the model may have been used with another theta meanwhile
        tbar = model.adjoint_theta(x, y, ctx.sigma, w.contiguous())
        return tbar, None, None, None, None


def lagrangian_gradient(theta, model, x, y, sigma=1.0):
    """grad_x L as a differentiable function of theta."""
    return LagrangianGradient.apply(theta, model, x, y, sigma)


class BatchLagrangianGradient(torch.autograd.Function):
    """The same map for every instance of a batch at once: theta_cat (the
    concatenated parameters) -> lag_cat (the concatenated Lagrangian
    gradients).  Forward: exa_batch_set_theta and one batched evaluation of
    the Lagrangian gradient (EXA_EV_LAG); backward: one batched evaluation
    of the parameter adjoint (EXA_EV_ADJ).  One autograd node, two batched
    calls, whatever the number of instances."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, batch: ExaBatch, x: torch.Tensor, y: torch.Tensor,
                sigma: float):
        if (isinstance(x, torch.Tensor) and x.requires_grad) or (isinstance(y, torch.Tensor) and y.requires_grad):
            raise NotImplementedError("BatchLagrangianGradient differentiates with respect to theta only; "
                                      "x and y must not require grad")
        theta_c = theta.detach().contiguous()
        batch.set_theta(theta_c)
        out = batch.empty("x", device=x.device)
        batch.evaluate(x, y, float(sigma), lag=out)
        ctx.batch, ctx.sigma = batch, float(sigma)
        ctx.save_for_backward(theta_c, x, y)
        return out

    @staticmethod
    def backward(ctx, w: torch.Tensor):
        if any(ctx.needs_input_grad[1:]):
            raise NotImplementedError("BatchLagrangianGradient differentiates with respect to theta only")
        theta, x, y = ctx.saved_tensors
        batch = ctx.batch
        batch.set_theta(theta)  # the batch may have been used with another theta meanwhile
        tbar = batch.empty("theta", device=x.device)
        batch.evaluate(x, y, ctx.sigma, wx=w.contiguous(), theta_bar=tbar)
        return tbar, None, None, None, None


def batch_lagrangian_gradient(theta, batch, x, y, sigma=1.0):
    """grad_x L of every instance as a differentiable function of the
    concatenated parameters."""
    return BatchLagrangianGradient.apply(theta, batch, x, y, sigma)
