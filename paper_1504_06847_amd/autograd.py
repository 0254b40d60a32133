"""``MuffinUnroll``: K unrolled passes of Algorithm 1 as a differentiable
torch operation of (mu_s, mu_nu, rho, mu_eps) and of the dirty images.  The
forward runs the K passes once, checkpointed (muffin_grad_record); the
backward is the reverse half of the library's hand-written sweep
(muffin_grad_replay), which reuses those checkpoints."""
from __future__ import annotations

import torch

from .solver import Solver


class MuffinUnroll(torch.autograd.Function):
    """x_K = MuffinUnroll.apply(psf, dirty, mu_s, mu_nu, rho, K[, ckpt_every, mu_eps])

    mu_s, mu_nu, rho, mu_eps: 0-d tensors (or floats); rho is the common
    value of rho_P = rho_T = rho_V = rho_S.  x_K has the dtype of psf
    (float32 or float64) and lives on its device.  ckpt_every: the reverse
    sweep's checkpoint spacing (default: Solver.sweep_ckpt_every).  Gradients
    flow to mu_s, mu_nu, rho and mu_eps when they are tensors, and to dirty
    when it requires them (the cotangent of the dirty images, muffin_grad_dirty's
    dL/dY); psf gets none."""

    @staticmethod
    def forward(ctx, psf, dirty, mu_s, mu_nu, rho, K, ckpt_every=None, mu_eps=1e-3):
        dtype = psf.dtype if psf.dtype in (torch.float32, torch.float64) else torch.float32
        dev = psf.device if psf.device.type == "cuda" else torch.device("cuda")
        s = Solver(psf.detach(), dirty.detach(), dtype=dtype, device=dev, mu_eps=float(mu_eps),
                   mu_s=float(mu_s), mu_nu=float(mu_nu), rho=float(rho))
        ctx.want_dirty = bool(ctx.needs_input_grad[1])
        s.grad_record(int(K), ckpt_every=None if ckpt_every is None else int(ckpt_every),
                      dirty=ctx.want_dirty)
        ctx.solver = s
        ctx.kinds = tuple(torch.is_tensor(v) for v in (mu_s, mu_nu, rho, mu_eps))
        ctx.dirty_dtype = dirty.dtype
        return s.x

    @staticmethod
    def backward(ctx, gx):
        s = ctx.solver
        _, g, gy = s.grad_replay(gx=gx.detach().contiguous())
        s.close()
        ctx.solver = None
        vals = (g["mu_s"], g["mu_nu"], g["rho_P"] + g["rho_T"] + g["rho_V"] + g["rho_S"], g["mu_eps"])
        mu_s, mu_nu, rho, mu_eps = [torch.tensor(float(v), dtype=gx.dtype, device=gx.device) if t else None
                                    for v, t in zip(vals, ctx.kinds)]
        gdirty = gy.to(ctx.dirty_dtype) if (ctx.want_dirty and gy is not None) else None
        return (None, gdirty, mu_s, mu_nu, rho, None, None, mu_eps)
