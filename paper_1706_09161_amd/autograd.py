"""torch.autograd access to the solver: forward = n steps of the HIP time step,
backward = the library's hand-written adjoint (lbm_fade_adjoint) with
checkpoint-and-recompute.

    C_n = fade_solve(C0, S, D, u, p, alpha=(1.6, 1.4), steps=500, ckpt_every=50)
    loss = 0.5 * ((C_n - C_obs) ** 2).sum()
    loss.backward()      # gradients for C0, S, D, u, p

D (d x d, symmetric), u and p (d values each) are small tensors on any
device; C0 and S (S may be None) are node fields on the GPU, slowest axis
first.  C_n is float32 (the step computes in FP32).  Each gradient has the
dtype and device of its input; D's gradient is the symmetrised one (a
symmetric perturbation dD changes the loss by sum_ab grad_ab dD_ab), so a D
built from tied off-diagonal parameters receives their full derivative.
Every other keyword (g, dx, dt, tau_free, tau0, c_wall, collision,
precision, flux_form, nonfinite_check_every) goes to the solver unchanged.
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
        kw = {k: v for k, v in opts.items() if k not in ("alpha", "steps", "ckpt_every")}
        solver = LbmFade(dim, n, alpha=opts["alpha"], p=_vals(p), D=Dm, u=_vals(u), **kw)
        try:
            solver.set_C(C0.detach().float().contiguous())
            solver.set_source(None if S is None else S.detach().float().contiguous())
            solver.step(opts["steps"])
            out = solver.get_C()
        except Exception:
            solver.close()
            raise
        # the inputs themselves are saved, so an in-place change before
        # backward() is caught by autograd's version check
        ctx.save_for_backward(C0, S, D, u, p)
        ctx.solver = solver
        ctx.opts = opts
        return out

    @staticmethod
    def backward(ctx, gC):
        C0, S, D, u, p = ctx.saved_tensors
        solver, opts = ctx.solver, ctx.opts
        ctx.solver = None
        try:
            solver.set_C(C0.detach().float().contiguous())
            solver.set_source(None if S is None else S.detach().float().contiguous())
            grads, dC0, dS = solver.adjoint(opts["steps"], opts.get("ckpt_every", 50),
                                            gC.detach().float().contiguous())
        finally:
            solver.close()

        def like(val, ref):
            t = torch.as_tensor(np.asarray(val, dtype=np.float64))
            return t.reshape(ref.shape).to(dtype=ref.dtype, device=ref.device)

        need = ctx.needs_input_grad
        return (dC0.to(C0.dtype) if need[0] else None,
                dS.to(S.dtype) if (S is not None and need[1]) else None,
                like(grads["D"], D) if need[2] else None,
                like(grads["u"], u) if need[3] else None,
                like(grads["p"], p) if need[4] else None,
                None)


def fade_solve(C0, S, D, u, p, *, alpha, steps: int, ckpt_every: int = 50, **opts):
    """C after `steps` time steps, differentiable in C0, S, D, u and p."""
    o = dict(opts)
    o.update(alpha=list(alpha), steps=int(steps), ckpt_every=int(ckpt_every))
    D, u, p = (torch.as_tensor(x, dtype=torch.float64) if not isinstance(x, torch.Tensor) else x for x in (D, u, p))
    return FadeSolve.apply(C0, S, D, u, p, o)
