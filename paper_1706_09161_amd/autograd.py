"""torch.autograd access to the solver: forward = n steps of the HIP time step,
backward = the library's hand-written adjoint (lbm_fade_adjoint) with
checkpoint-and-recompute.

    C_n = fade_solve(C0, S, D, u, p, alpha=(1.6, 1.4), steps=500, ckpt_every=50)
    loss = 0.5 * ((C_n - C_obs) ** 2).sum()
    loss.backward()      # gradients for C0, S, D, u, p

D, u, p are small tensors (any device); C0 and S are node fields on the GPU.
Every call creates a solver for the given parameters (they are create-time
constants of the library), so keep one call per optimisation step.
"""
from __future__ import annotations

import numpy as np
import torch

from .solver import LbmFade


def _vals(t) -> list:
    return [float(v) for v in torch.as_tensor(t).detach().double().cpu().reshape(-1)]


class FadeSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C0, S, D, u, p, opts: dict):
        dim = C0.dim()
        n = list(reversed(C0.shape))
        Dm = np.array(_vals(D)).reshape(dim, dim)
        solver = LbmFade(dim, n, alpha=opts["alpha"], p=_vals(p), D=Dm, u=_vals(u), g=opts.get("g"),
                         dx=opts.get("dx", 1.0), dt=opts.get("dt", 1.0), tau_free=opts.get("tau_free"),
                         tau0=opts.get("tau0", 1.0), c_wall=opts.get("c_wall", 0.0),
                         collision=opts.get("collision", "MRT"), precision=opts.get("precision", "fp32"))
        C0c = C0.detach().float().contiguous()
        Sc = None if S is None else S.detach().float().contiguous()
        solver.set_C(C0c)
        solver.set_source(Sc)
        solver.step(opts["steps"])
        out = solver.get_C()
        ctx.solver = solver
        ctx.saved = (C0c, Sc)
        ctx.opts = opts
        ctx.meta = (D, u, p, S is not None)
        return out

    @staticmethod
    def backward(ctx, gC):
        solver, (C0c, Sc), opts = ctx.solver, ctx.saved, ctx.opts
        D, u, p, has_S = ctx.meta
        solver.set_C(C0c)
        solver.set_source(Sc)
        grads, dC0, dS = solver.adjoint(opts["steps"], opts.get("ckpt_every", 50), gC.detach().float().contiguous())
        solver.close()
        ctx.solver = None

        def like(val, ref):
            t = torch.as_tensor(np.asarray(val, dtype=np.float64))
            r = torch.as_tensor(ref)
            return t.reshape(r.shape).to(dtype=r.dtype if r.is_floating_point() else torch.float64, device=r.device)

        return (dC0, dS if has_S else None, like(grads["D"], D), like(grads["u"], u), like(grads["p"], p), None)


def fade_solve(C0, S, D, u, p, *, alpha, steps: int, ckpt_every: int = 50, **opts):
    """C after `steps` time steps, differentiable in C0, S, D, u and p."""
    o = dict(opts)
    o.update(alpha=list(alpha), steps=int(steps), ckpt_every=int(ckpt_every))
    return FadeSolve.apply(C0, S, D, u, p, o)
