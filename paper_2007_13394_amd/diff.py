"""Differentiable particle-mesh run behind torch.autograd.Function.

Argument marshalling only: the forward passes call pm_ic / pm_step /
pm_density and the backward passes call their hand-written reverse modes
(pm_ic_vjp, pm_step_vjp, pm_density_vjp) in libpm.  Checkpointing is per step:
each step saves its input positions (the force meshes are recomputed in the
reverse pass), so a run of n steps keeps n + 1 position arrays.  The context
must be configured with PM_FLAG_NO_SORT so that particles keep their order.
"""
import torch

from . import pm


class ICFunction(torch.autograd.Function):
    """white noise [n_cdm]^3 -> (x, p) [3, P] (Zel'dovich initial conditions)."""

    @staticmethod
    def forward(fctx, white, ctx):
        x, p = ctx.particles()
        pm.pm_ic(ctx, white.contiguous(), x, p)
        fctx.pmctx = ctx
        fctx.wshape = white.shape
        return x, p

    @staticmethod
    def backward(fctx, xbar, pbar):
        ctx = fctx.pmctx
        wbar = torch.empty(fctx.wshape, dtype=torch.float32, device=xbar.device)
        pm.pm_ic_vjp(ctx, xbar.contiguous(), pbar.contiguous(), wbar)
        return wbar, None


class StepFunction(torch.autograd.Function):
    """(x, p) -> (x', p') for one pm_step call with scale factors `call`."""

    @staticmethod
    def forward(fctx, x, p, ctx, call):
        x1, p1 = x.clone(), p.clone()
        pm.pm_step(ctx, x1, p1, *call)
        fctx.save_for_backward(x)
        fctx.pmctx, fctx.call = ctx, call
        return x1, p1

    @staticmethod
    def backward(fctx, xbar, pbar):
        (x,) = fctx.saved_tensors
        xb, pb = xbar.contiguous().clone(), pbar.contiguous().clone()
        pm.pm_step_vjp(fctx.pmctx, x, *fctx.call, xb, pb)
        return xb, pb, None, None


class DensityFunction(torch.autograd.Function):
    """x -> painted density contrast delta [N, N, N]."""

    @staticmethod
    def forward(fctx, x, ctx):
        n = ctx.n
        delta = torch.empty((n, n, n), dtype=torch.float32, device=x.device)
        pm.pm_density(ctx, x, delta)
        fctx.save_for_backward(x)
        fctx.pmctx = ctx
        return delta

    @staticmethod
    def backward(fctx, dd):
        (x,) = fctx.saved_tensors
        xb = torch.zeros_like(x)
        pm.pm_density_vjp(fctx.pmctx, x, dd.contiguous(), xb)
        return xb, None


def final_density(ctx, white, calls):
    """White noise -> initial conditions -> the KDK calls -> final density."""
    x, p = ICFunction.apply(white, ctx)
    for c in calls:
        x, p = StepFunction.apply(x, p, ctx, tuple(c))
    return DensityFunction.apply(x, ctx)
