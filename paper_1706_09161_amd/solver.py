"""Thin Python binding over the C ABI: same entry points, argument marshalling only.

Every step of the method runs in the HIP kernels of liblbmfade.so; this module
turns Python values into the ABI's structs, passes tensor addresses and the
current torch stream, and raises on error codes.  Device memory comes from
torch (``torch.cuda`` tensors) or numpy arrays (host memory).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L

_COLLISION = {"BGK": L.LBM_BGK, "MRT": L.LBM_MRT}
_PRECISION = {"fp32": L.LBM_FP32, "bf16x3": L.LBM_BF16X3, "fp32_simt": L.LBM_FP32_SIMT}
_FLUX_FORM = {"rl": L.LBM_FLUX_RL, "caputo": L.LBM_FLUX_CAPUTO}


def _torch():
    import torch

    return torch


def _is_cuda_tensor(x) -> bool:
    try:
        torch = _torch()
    except ImportError:  # pragma: no cover
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


def _stream_ptr(stream):
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    try:
        torch = _torch()
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:  # pragma: no cover
        pass
    return ctypes.c_void_p(0)


def make_structs(dim: int, n, *, alpha, p, D, g=None, u=None, dx: float = 1.0, dt: float = 1.0, tau_free=None,
                 tau0: float = 1.0, c_wall: float = 0.0, collision: str = "MRT", precision: str = "fp32",
                 nonfinite_check_every: int = 0, flux_form: str = "rl"):
    """The ABI's lbm_grid and lbm_params for these arguments (see LbmFade)."""
    d = int(dim)
    n = [int(v) for v in n][:d]
    grid = L.lbm_grid()
    grid.dim = d
    for mu in range(3):
        grid.n[mu] = n[mu] if mu < d else 1
    grid.dx, grid.dt = float(dx), float(dt)
    P = L.lbm_params()
    g = [1.0] * d if g is None else list(g)
    u = [0.0] * d if u is None else list(u)
    tf = [1.0] * 4 if tau_free is None else list(tau_free) + [1.0] * (4 - len(tau_free))
    Dm = np.asarray(D, dtype=np.float64).reshape(d, d)
    for mu in range(d):
        P.alpha[mu] = float(alpha[mu])
        P.p[mu] = float(p[mu])
        P.g[mu] = float(g[mu])
        P.u[mu] = float(u[mu])
    for a in range(d):
        for b in range(d):
            P.D[a * d + b] = float(Dm[a, b])
    for k in range(4):
        P.tau_free[k] = float(tf[k])
    P.tau0 = float(tau0)
    P.c_wall = float(c_wall)
    P.collision = _COLLISION[collision]
    P.precision = _PRECISION[precision]
    P.nonfinite_check_every = int(nonfinite_check_every)
    P.flux_form = _FLUX_FORM[flux_form]
    return grid, P


def config_kwargs(cfg: dict) -> dict:
    """Solver keyword arguments of a plain configuration dict (see ``synth``)."""
    return dict(alpha=cfg["alpha"], p=cfg["p"], D=cfg["D"], g=cfg.get("g"), u=cfg.get("u"), dx=cfg.get("dx", 1.0),
                dt=cfg.get("dt", 1.0), tau_free=cfg.get("tau_free"), tau0=cfg.get("tau0", 1.0),
                c_wall=cfg.get("c_wall", 0.0), collision=cfg.get("collision", "MRT"),
                flux_form=cfg.get("flux_form", "rl"))


class LbmFade:
    """One solver (one grid, one parameter set) on the current HIP device."""

    def __init__(self, dim: int, n, *, alpha, p, D, g=None, u=None, dx: float = 1.0, dt: float = 1.0,
                 tau_free=None, tau0: float = 1.0, c_wall: float = 0.0, collision: str = "MRT",
                 precision: str = "fp32", nonfinite_check_every: int = 0, flux_form: str = "rl"):
        lib = L.lib()
        self.dim = int(dim)
        self.n = [int(v) for v in n][: self.dim]
        self.Q = 2 * self.dim + 1
        self.nodes = int(np.prod(self.n))
        self.shape = tuple(reversed(self.n))  # slowest axis first
        grid, P = make_structs(dim, n, alpha=alpha, p=p, D=D, g=g, u=u, dx=dx, dt=dt, tau_free=tau_free, tau0=tau0,
                               c_wall=c_wall, collision=collision, precision=precision,
                               nonfinite_check_every=nonfinite_check_every, flux_form=flux_form)
        h = ctypes.c_void_p()
        L.check(lib.lbm_fade_create(ctypes.byref(grid), self.Q, ctypes.byref(P), ctypes.byref(h)))
        self._h = h
        self.precision = precision
        self.collision = collision

    @classmethod
    def from_config(cls, cfg: dict, precision: str = "fp32", **kw) -> "LbmFade":
        d = cfg["dim"]
        return cls(d, cfg["n"][:d], precision=precision, **config_kwargs(cfg), **kw)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            L.lib().lbm_fade_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- marshalling ------------------------------------------------------------
    def _in(self, x, count: int):
        """(address, on_device, keepalive) of an input buffer of `count` float32."""
        if _is_cuda_tensor(x):
            t = x.detach()
            if t.dtype != _torch().float32 or not t.is_contiguous():
                t = t.to(_torch().float32).contiguous()
            if t.numel() != count:
                raise ValueError(f"expected {count} values, got {t.numel()}")
            return ctypes.c_void_p(t.data_ptr()), 1, t
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        if a.size != count:
            raise ValueError(f"expected {count} values, got {a.size}")
        return ctypes.c_void_p(a.ctypes.data), 0, a

    def _out(self, out, count: int, shape, device: bool):
        if out is None:
            if device:
                torch = _torch()
                out = torch.empty(shape, dtype=torch.float32, device="cuda")
            else:
                out = np.empty(shape, dtype=np.float32)
        if _is_cuda_tensor(out):
            if out.dtype != _torch().float32 or not out.is_contiguous() or out.numel() != count:
                raise ValueError("output tensor must be contiguous float32 of the right size")
            return out, ctypes.c_void_p(out.data_ptr()), 1
        if not (isinstance(out, np.ndarray) and out.dtype == np.float32 and out.flags.c_contiguous
                and out.size == count):
            raise ValueError("output array must be contiguous float32 of the right size")
        return out, ctypes.c_void_p(out.ctypes.data), 0

    # -- ABI calls --------------------------------------------------------------
    def set_C(self, C0, stream=None):
        ptr, dev, keep = self._in(C0, self.nodes)
        L.check(L.lib().lbm_fade_set_C(self._h, ptr, dev, _stream_ptr(stream)))

    def set_source(self, S, stream=None):
        if S is None:
            L.check(L.lib().lbm_fade_set_source(self._h, None, 0, _stream_ptr(stream)))
            return
        ptr, dev, keep = self._in(S, self.nodes)
        L.check(L.lib().lbm_fade_set_source(self._h, ptr, dev, _stream_ptr(stream)))

    def set_diffusion(self, D, stream=None):
        """Space-dependent diffusion tensor: D of shape (d, d, *grid shape), or None
        for the constant tensor of the handle (MRT only)."""
        if D is None:
            L.check(L.lib().lbm_fade_set_diffusion(self._h, None, 0, _stream_ptr(stream)))
            return
        ptr, dev, keep = self._in(D, self.dim * self.dim * self.nodes)
        L.check(L.lib().lbm_fade_set_diffusion(self._h, ptr, dev, _stream_ptr(stream)))

    def set_wall(self, Cw, stream=None):
        """Dirichlet value of every wall node (a node field), or None for c_wall."""
        if Cw is None:
            L.check(L.lib().lbm_fade_set_wall(self._h, None, 0, _stream_ptr(stream)))
            return
        ptr, dev, keep = self._in(Cw, self.nodes)
        L.check(L.lib().lbm_fade_set_wall(self._h, ptr, dev, _stream_ptr(stream)))

    def step(self, n: int = 1, stream=None):
        L.check(L.lib().lbm_fade_step(self._h, int(n), _stream_ptr(stream)))

    def get_C(self, out=None, device: bool = True, stream=None):
        out, ptr, dev = self._out(out, self.nodes, self.shape, device)
        L.check(L.lib().lbm_fade_get_C(self._h, ptr, dev, _stream_ptr(stream)))
        return out

    def get_f(self, out=None, device: bool = True, stream=None):
        out, ptr, dev = self._out(out, self.Q * self.nodes, (self.Q,) + self.shape, device)
        L.check(L.lib().lbm_fade_get_f(self._h, ptr, dev, _stream_ptr(stream)))
        return out

    def set_f(self, f, stream=None):
        ptr, dev, keep = self._in(f, self.Q * self.nodes)
        L.check(L.lib().lbm_fade_set_f(self._h, ptr, dev, _stream_ptr(stream)))

    def apply_phi(self, C, out=None, stream=None):
        """Phi of every axis for the field C; C = None uses the solver's own
        current concentration (device output; the GEMM launch of a step)."""
        if C is None:
            out, optr, odev = self._out(out, self.dim * self.nodes, (self.dim,) + self.shape, True)
            if not odev:
                raise ValueError("C = None needs a device output")
            L.check(L.lib().lbm_fade_apply_phi(self._h, None, optr, 1, _stream_ptr(stream)))
            return out
        dev_in = _is_cuda_tensor(C)
        ptr, dev, keep = self._in(C, self.nodes)
        out, optr, odev = self._out(out, self.dim * self.nodes, (self.dim,) + self.shape, bool(dev_in))
        if odev != dev:
            raise ValueError("C and Phi must both be host or both be device buffers")
        L.check(L.lib().lbm_fade_apply_phi(self._h, ptr, optr, dev, _stream_ptr(stream)))
        return out

    def adjoint(self, n: int, ckpt_every: int, gC, want_fields: bool = True, stream=None):
        """Gradients of <gC, C_n>: returns (dict of FP64 scalars, dC0, dS)."""
        dev_in = _is_cuda_tensor(gC)
        ptr, dev, keep = self._in(gC, self.nodes)
        dC0 = dS = None
        p0 = p1 = None
        if want_fields:
            dC0, p0, _ = self._out(None, self.nodes, self.shape, bool(dev_in))
            dS, p1, _ = self._out(None, self.nodes, self.shape, bool(dev_in))
        g = L.lbm_grads()
        L.check(L.lib().lbm_fade_adjoint(self._h, int(n), int(ckpt_every), ptr, dev, ctypes.byref(g), p0, p1,
                                         _stream_ptr(stream)))
        d = self.dim
        grads = {
            "D": np.array(g.dD[: d * d]).reshape(d, d),
            "u": np.array(g.du[:d]),
            "p": np.array(g.dp[:d]),
        }
        return grads, dC0, dS


def apply_phi_noalloc(dim: int, n, C, out=None, stream=None, **params):
    """lbm_fade_apply_phi_noalloc: the fractional operator of every axis for the
    device field C without a handle (no device allocation in the library).
    params are LbmFade's keyword arguments; C and out are CUDA tensors (out:
    float32, contiguous, shape (dim, *C.shape); allocated here when None)."""
    grid, P = make_structs(dim, n, **params)
    if not _is_cuda_tensor(C):
        raise ValueError("C must be a CUDA tensor")
    torch = _torch()
    c = C.detach()
    if c.dtype != torch.float32 or not c.is_contiguous():
        c = c.to(torch.float32).contiguous()
    nodes = int(np.prod([int(v) for v in n][: int(dim)]))
    if c.numel() != nodes:
        raise ValueError(f"expected {nodes} values, got {c.numel()}")
    if out is None:
        out = torch.empty((int(dim),) + tuple(c.shape), dtype=torch.float32, device=c.device)
    if not (_is_cuda_tensor(out) and out.dtype == torch.float32 and out.is_contiguous()
            and out.numel() == int(dim) * nodes):
        raise ValueError("out must be a contiguous float32 CUDA tensor of dim * nodes values")
    L.check(L.lib().lbm_fade_apply_phi_noalloc(ctypes.byref(grid), ctypes.byref(P), ctypes.c_void_p(c.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def version() -> str:
    return L.lib().lbm_fade_version().decode()
