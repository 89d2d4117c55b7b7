"""torch.autograd wrappers: the estimator and the receive model as
differentiable operators, so they can sit inside receiver chains.

  correlate(Y)   H = Y P / N       (Eq. 3 / Eq. 10)   backward: g P^T / N
  synthesize(X)  Yhat = P X        (Eq. 9, noiseless)  backward: g P

P is real, so under PyTorch's convention for complex autograd (the gradient of
a real loss is dL/dRe + i dL/dIm) each backward is the plain transpose, with
no conjugation. Forward and backward both run in libpnce.so: the correlator
kernel and its adjoint kernel; nothing here computes.
"""
from __future__ import annotations

import torch

from .api import Plan


def _plain(t: torch.Tensor) -> torch.Tensor:
    """Contiguous memory holding the tensor's values (conjugate and negative
    views resolved): the library reads memory, not view flags."""
    return t.resolve_conj().resolve_neg().contiguous()


class PnceCorrelate(torch.autograd.Function):
    """H = Y P / N; grad_Y = grad_H P^T / N (pnce_adjoint with alpha = 1/N)."""

    @staticmethod
    def forward(ctx, Y, plan: Plan, precision: str):
        ctx.plan = plan
        ctx.precision = precision
        return plan.estimate(_plain(Y), precision)

    @staticmethod
    def backward(ctx, gH):
        gY = None
        if ctx.needs_input_grad[0]:
            gY = ctx.plan.adjoint(_plain(gH), ctx.precision)
        return gY, None, None


class PnceSynthesize(torch.autograd.Function):
    """Yhat = P X (pnce_adjoint with alpha = 1); grad_X = grad_Yhat P
    (pnce_estimate with alpha = 1)."""

    @staticmethod
    def forward(ctx, X, plan: Plan, precision: str):
        ctx.plan = plan
        ctx.precision = precision
        return plan.adjoint(_plain(X), precision, alpha=1.0)

    @staticmethod
    def backward(ctx, gY):
        gX = None
        if ctx.needs_input_grad[0]:
            gX = ctx.plan.estimate(_plain(gY), ctx.precision, alpha=1.0)
        return gX, None, None


def correlate(Y: torch.Tensor, plan: Plan, precision: str = "f32s") -> torch.Tensor:
    return PnceCorrelate.apply(Y, plan, precision)


def synthesize(X: torch.Tensor, plan: Plan, precision: str = "f32s") -> torch.Tensor:
    return PnceSynthesize.apply(X, plan, precision)


def residual_loss(y: torch.Tensor, X: torch.Tensor, plan: Plan,
                  precision: str = "f32s") -> torch.Tensor:
    """||y - P X||^2 summed over every frame, antenna and sample."""
    r = y - synthesize(X, plan, precision)
    return (r.real ** 2 + r.imag ** 2).sum()


def refine_by_gradient(y: torch.Tensor, plan: Plan, steps: int, precision: str = "f32s"):
    """Least-squares refinement as gradient descent on ||y - P x||^2 with step
    1/(2N), gradients from autograd through the library's kernels:
    x_0 = correlate(y); x_{j+1} = x_j - grad/(2N) = x_j + P^T (y - P x_j)/N.
    Returns (iterates [x_0 .. x_steps], losses at each iterate)."""
    x = correlate(y, plan, precision).detach()
    xs, losses = [x], []
    for _ in range(steps + 1):
        xg = x.detach().requires_grad_(True)
        loss = residual_loss(y, xg, plan, precision)
        losses.append(float(loss.detach()))
        if len(xs) > steps:
            break
        (g,) = torch.autograd.grad(loss, xg)
        x = (xg - g / (2.0 * plan.N)).detach()
        xs.append(x)
    return xs, losses
