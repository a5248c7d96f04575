"""Differentiable filter: a torch.autograd.Function around the library's
forward and hand-written adjoint (r3d_filter_forward / r3d_filter_backward).

``filter_posterior`` maps the model parameters (beta, IRF taps, sigma_rw2,
nu) to every frame's posterior mean and variance; any torch loss of those
outputs can be back-propagated to the parameters. The adjoint runs on the
device; this module only marshals arguments. ``gaussian_irf`` gives the
bin-integrated Gaussian pulse as a differentiable function of its width, so
gradients reach the IRF sigma through the chain rule over the W taps.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import r3d

THETA_FIXED = 11  # beta, sigma_rw2, nu[0..8] ahead of the IRF taps in the gradient


def gaussian_irf(sigma: torch.Tensor, W: int, c: int) -> torch.Tensor:
    """Bin-integrated Gaussian pulse of width sigma with its peak at tap c,
    renormalised over the W taps (float64, differentiable in sigma)."""
    j = torch.arange(W, dtype=torch.float64, device=sigma.device)
    pmf = torch.special.ndtr((j - c + 0.5) / sigma) - torch.special.ndtr((j - c - 0.5) / sigma)
    return pmf / pmf.sum()


class _FilterFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta, irf, sigma_rw2, nu, base, frames, ckpt_every, device):
        params = dict(base)
        params.update(beta=float(beta), irf=irf.detach().cpu().double().numpy(),
                      sigma_rw2=float(sigma_rw2), nu=nu.detach().cpu().double().numpy())
        c = r3d.Context(params)
        N, P = len(frames), c.P
        init = r3d.State.empty(P, device)
        c.state_init(init)
        ws = torch.empty(c.grad_workspace_size(N, ckpt_every), dtype=torch.uint8, device=device)
        mean = torch.empty(N * P, dtype=torch.float32, device=device)
        var = torch.empty(N * P, dtype=torch.float32, device=device)
        c.filter_forward(frames, ckpt_every, init, mean, var, ws)
        ctx.lib_ctx, ctx.frames, ctx.ws, ctx.ckpt = c, frames, ws, ckpt_every
        ctx.W, ctx.device = irf.shape[0], device
        ctx.dtypes = (beta.dtype, irf.dtype, sigma_rw2.dtype, nu.dtype)
        return mean.view(N, P), var.view(N, P)

    @staticmethod
    def backward(ctx, gmean, gvar):
        c = ctx.lib_ctx
        gm = gmean.to(torch.float32).contiguous().view(-1)
        gv = None if gvar is None else gvar.to(torch.float32).contiguous().view(-1)
        grad = torch.empty(THETA_FIXED + ctx.W, dtype=torch.float64, device=ctx.device)
        c.filter_backward(ctx.frames, ctx.ckpt, gm, gv, ctx.ws, grad)
        g = grad.cpu()
        tb, ti, ts, tn = ctx.dtypes
        return (g[0].to(tb), g[THETA_FIXED:].to(ti), g[1].to(ts), g[2:THETA_FIXED].to(tn),
                None, None, None, None)


def filter_posterior(beta: torch.Tensor, irf: torch.Tensor, sigma_rw2: torch.Tensor,
                     nu: torch.Tensor, base: dict, frames: "r3d.Frames", ckpt_every: int = 5,
                     device="cuda"):
    """Posterior means and variances [nframes, P] of the filter run from the
    initial state with these parameters (beta, sigma_rw2: scalars; irf [W];
    nu [9]); the other model fields come from ``base`` (a parameter dict)."""
    return _FilterFunction.apply(beta, irf, sigma_rw2, nu, base, frames, ckpt_every,
                                 torch.device(device))
