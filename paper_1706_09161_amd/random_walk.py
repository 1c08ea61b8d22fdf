"""Levy-stable random walk on the GPU (lbm_rw_* of the C ABI): the paper's
statistical counterpart of the LB solution (Sec. 3.1, equations
(RW_STABLE), (distri); killed at the first exit from the box).  Thin
marshalling: positions (dim, n) float64 and alive flags (n,) uint8 live in
torch CUDA tensors; every step runs in the library's kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from .solver import _stream_ptr, _torch


class RandomWalk:
    """Walk parameters of one box: see lbm_rw_params in include/lbm_fade.h."""

    def __init__(self, dim: int, lo, hi, *, alpha, p, D, g=None, u=None, dt: float = 1e-3, seed: int = 1):
        P = L.lbm_rw_params()
        P.dim = int(dim)
        for mu in range(P.dim):
            P.lo[mu], P.hi[mu] = float(lo[mu]), float(hi[mu])
            P.alpha[mu], P.p[mu], P.D[mu] = float(alpha[mu]), float(p[mu]), float(D[mu])
            P.g[mu] = 1.0 if g is None else float(g[mu])
            P.u[mu] = 0.0 if u is None else float(u[mu])
        P.dt = float(dt)
        P.seed = int(seed)
        self.P = P
        self.dim = P.dim

    def init_gaussian(self, center, sigma0: float, n: int, first: int = 0, stream=None):
        """Positions (dim, n) float64 and alive flags (n,) uint8 on the current device."""
        torch = _torch()
        x = torch.empty((self.dim, int(n)), dtype=torch.float64, device="cuda")
        alive = torch.empty(int(n), dtype=torch.uint8, device="cuda")
        c = (ctypes.c_double * 3)(*([float(v) for v in center] + [0.0] * (3 - len(center))))
        L.check(L.lib().lbm_rw_init_gaussian(ctypes.byref(self.P), c, float(sigma0), int(n), int(first),
                                             ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(alive.data_ptr()),
                                             _stream_ptr(stream)))
        return x, alive

    def walk(self, x, alive, nsteps: int, first: int = 0, step0: int = 0, stream=None):
        """Steps step0 + 1 .. step0 + nsteps in place on (x, alive)."""
        self._check(x, alive)
        L.check(L.lib().lbm_rw_walk(ctypes.byref(self.P), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(alive.data_ptr()), int(alive.numel()), int(first), int(step0),
                                    int(nsteps), _stream_ptr(stream)))

    def histogram(self, x, alive, nodes, dx: float, stream=None):
        """Counts of living particles per node (torch int32 view of the uint32
        counts, shape reversed(nodes))."""
        self._check(x, alive)
        torch = _torch()
        nn = (ctypes.c_int32 * 3)(*([int(v) for v in nodes] + [1] * (3 - len(nodes))))
        counts = torch.empty(int(np.prod(nodes)), dtype=torch.int32, device="cuda")
        L.check(L.lib().lbm_rw_histogram(ctypes.byref(self.P), ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(alive.data_ptr()), int(alive.numel()), nn, float(dx),
                                         ctypes.c_void_p(counts.data_ptr()), _stream_ptr(stream)))
        return counts.reshape(tuple(reversed([int(v) for v in nodes])))

    def _check(self, x, alive):
        torch = _torch()
        if not (x.is_cuda and alive.is_cuda and x.dtype == torch.float64 and alive.dtype == torch.uint8
                and x.is_contiguous() and alive.is_contiguous() and tuple(x.shape) == (self.dim, alive.numel())):
            raise ValueError("x must be a contiguous (dim, n) float64 CUDA tensor and alive a (n,) uint8 one")


def main():
    """Throughput of the walk on the paper's validation 1 (Omega = [0, 2]^2,
    alpha = (1.5, 1.99), D = 0.5 Id, p = 1/2, dt = 1e-3, t = 0.1): 4e6
    particles, 100 steps, timed with HIP events on the launch stream."""
    import argparse

    ap = argparse.ArgumentParser()
    ap.add_argument("--particles", type=int, default=4_000_000)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    torch = _torch()
    W = RandomWalk(2, [0, 0], [2, 2], alpha=[1.5, 1.99], p=[0.5, 0.5], D=[0.5, 0.5], dt=1e-3, seed=2024)
    stream = torch.cuda.current_stream()
    best = None
    for _ in range(args.reps):
        x, a = W.init_gaussian([1.0, 1.0], 0.05, args.particles)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        W.walk(x, a, args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    draws = args.particles * args.steps * 2
    print(f"{args.particles} particles x {args.steps} steps: {best:.2f} ms, {draws / best / 1e6:.2f} G stable draws/s, "
          f"survival {float(a.float().mean()):.5f}")


if __name__ == "__main__":
    main()
