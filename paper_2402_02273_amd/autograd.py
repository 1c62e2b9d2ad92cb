"""``torch.autograd`` wrapper of the library's multi-step advance.

``advance(ctx, u0, rho, class_D, nsteps)`` returns u after ``nsteps`` exponential
Euler steps; its backward calls ``expint_vjp`` (the library's discrete adjoint
with checkpointed recomputation) for the gradients with respect to u0, rho
and the class diffusivities.  The (s, m) plan of the context is kept fixed
while the parameters change, so the map being differentiated is smooth.
"""

from __future__ import annotations

import torch

from .expint import ExpInt


class ExpIntAdvance(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: ExpInt, u0, rho, class_D, nsteps: int, ckpt_every: int):
        ctx.set_params(rho=float(rho), class_D=[float(v) for v in class_D], replan=False)
        u0c = u0.detach().contiguous()
        u = u0c.clone()
        ctx.advance(u, int(nsteps))
        fctx.ctx = ctx
        fctx.nsteps = int(nsteps)
        fctx.ckpt_every = int(ckpt_every)
        fctx.param_state = (float(rho), [float(v) for v in class_D])
        fctx.rho_like = rho
        fctx.cd_like = class_D
        fctx.save_for_backward(u0c)
        return u

    @staticmethod
    def backward(fctx, gout):
        (u0,) = fctx.saved_tensors
        ctx = fctx.ctx
        rho, cd = fctx.param_state
        ctx.set_params(rho=rho, class_D=cd, replan=False)
        gu, grho, gD = ctx.vjp(u0, fctx.nsteps, gout.contiguous(), ckpt_every=fctx.ckpt_every)
        g_rho = torch.as_tensor(grho, dtype=fctx.rho_like.dtype, device=fctx.rho_like.device)
        g_cd = torch.as_tensor(gD, dtype=fctx.cd_like.dtype, device=fctx.cd_like.device)
        return None, gu, g_rho, g_cd, None, None


def advance(ctx: ExpInt, u0, rho, class_D, nsteps: int, ckpt_every: int = 10):
    """Differentiable u_T = advance(u0; rho, class_D) for a label-form context."""
    rho = torch.as_tensor(rho, dtype=torch.float64)
    class_D = torch.as_tensor(class_D, dtype=torch.float64)
    return ExpIntAdvance.apply(ctx, u0, rho, class_D, nsteps, ckpt_every)
