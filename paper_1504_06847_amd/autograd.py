"""``MuffinUnroll``: K unrolled passes of Algorithm 1 as a differentiable
torch operation of (mu_s, mu_nu, rho).  The backward pass is the library's
hand-written reverse sweep (muffin_grad in VJP mode)."""
from __future__ import annotations

import torch

from .solver import Solver


class MuffinUnroll(torch.autograd.Function):
    """x_K = MuffinUnroll.apply(psf, dirty, mu_s, mu_nu, rho, K[, ckpt_every, mu_eps])

    mu_s, mu_nu, rho: 0-d tensors (or floats); rho is the common value of
    rho_P = rho_T = rho_V = rho_S.  x_K has the dtype of psf (float32 or
    float64) and lives on its device.  ckpt_every: the reverse sweep's
    checkpoint spacing (default: Solver.sweep_ckpt_every).  Gradients flow to mu_s, mu_nu and
    rho; psf and dirty get none."""

    @staticmethod
    def forward(ctx, psf, dirty, mu_s, mu_nu, rho, K, ckpt_every=None, mu_eps=1e-3):
        dtype = psf.dtype if psf.dtype in (torch.float32, torch.float64) else torch.float32
        dev = psf.device if psf.device.type == "cuda" else torch.device("cuda")
        s = Solver(psf.detach(), dirty.detach(), dtype=dtype, device=dev, mu_eps=float(mu_eps),
                   mu_s=float(mu_s), mu_nu=float(mu_nu), rho=float(rho))
        s.iterate(int(K))
        ctx.solver, ctx.K = s, int(K)
        ctx.ckpt = None if ckpt_every is None else int(ckpt_every)
        ctx.kinds = tuple(torch.is_tensor(v) for v in (mu_s, mu_nu, rho))
        return s.x

    @staticmethod
    def backward(ctx, gx):
        s = ctx.solver
        _, g = s.grad(ctx.K, gx=gx.detach().contiguous(), ckpt_every=ctx.ckpt)
        s.close()
        ctx.solver = None
        grads = [torch.tensor(float(v), dtype=gx.dtype, device=gx.device) if t else None
                 for v, t in zip(g, ctx.kinds)]
        return (None, None, *grads, None, None, None)
