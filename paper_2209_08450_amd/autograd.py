"""Differentiable projector pair and gradient least squares.

``radon(x, plan)`` is the forward projector R (tp_radon); its gradient is the
hand-written adjoint R^T (tp_backproject with scale 1).  ``backproject(q,
plan, scale)`` is the reverse pair.  Both kernels evaluate the same FP32
coordinate expression, so R^T is the exact transpose of R up to summation
rounding (the paper names iterative reconstruction as the use of such a pair,
Sections 1 and 5).

``ls_solve`` minimises ||R x - y||^2 by gradient descent with the gradient from
autograd, x_{k+1} = x_k - eta * 2 R^T (R x_k - y), x_0 = 0, with
eta = 1 / (2 lambda_max(R^T R)) from power iteration on the device.  R acts on
each slice alone and is the same for every slice, so one step size serves all.
"""
from __future__ import annotations

import math

import torch

from . import tp


class RadonFn(torch.autograd.Function):
    """y = R x for x [rows][N][N] float32 -> y [rows][n_angles][n_det]."""

    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return tp.radon(plan, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return tp.backproject(ctx.plan, g.contiguous(), scale=1.0), None


class BackprojectFn(torch.autograd.Function):
    """f = scale R^T q for q [rows][n_angles][n_det] float32 -> f [rows][N][N]."""

    @staticmethod
    def forward(ctx, q, plan, scale):
        ctx.plan, ctx.scale = plan, float(scale)
        return tp.backproject(plan, q.contiguous(), scale=scale)

    @staticmethod
    def backward(ctx, g):
        return tp.radon(ctx.plan, g.contiguous()) * ctx.scale, None, None


def radon(x, plan):
    return RadonFn.apply(x, plan)


def backproject(q, plan, scale=1.0):
    return BackprojectFn.apply(q, plan, scale)


def power_lambda_max(plan, iters: int = 30, seed: int = 0, device="cuda") -> float:
    """Largest eigenvalue of R^T R (one slice) by power iteration from a seeded start."""
    g = torch.Generator(device=device).manual_seed(seed)
    v = torch.randn((1, plan.n_vox, plan.n_vox), generator=g, device=device)
    v /= torch.linalg.vector_norm(v)
    lam = 0.0
    for _ in range(iters):
        w = tp.backproject(plan, tp.radon(plan, v), scale=1.0)
        lam = float(torch.sum(v.double() * w.double()))
        v = w / torch.linalg.vector_norm(w)
    return lam


def ls_solve(plan, y, steps: int, eta: float | None = None, x0=None, callback=None):
    """Gradient descent on ||R x - y||^2 (summed over all slices).

    y: [rows][n_angles][n_det] float32 on the device.  Returns (x, losses) with
    losses[k] = ||R x_k - y||^2 (FP64 sum of the FP32 residual) before step k.
    """
    if eta is None:
        eta = 1.0 / (2.0 * power_lambda_max(plan, device=y.device))
    rows = y.shape[0]
    x = torch.zeros((rows, plan.n_vox, plan.n_vox), dtype=torch.float32, device=y.device) if x0 is None \
        else x0.detach().clone()
    losses = []
    for k in range(steps):
        x.requires_grad_(True)
        r = radon(x, plan) - y
        loss = torch.sum(r.double() ** 2)
        loss.backward()
        losses.append(float(loss))
        with torch.no_grad():
            x = x - eta * x.grad
        if callback is not None:
            callback(k, x, losses[-1])
    return x.detach(), losses


def step_size(plan, iters: int = 30) -> float:
    """eta = 1 / (2 lambda_max(R^T R))."""
    lam = power_lambda_max(plan, iters=iters)
    if not math.isfinite(lam) or lam <= 0:
        raise RuntimeError("power iteration failed")
    return 1.0 / (2.0 * lam)
