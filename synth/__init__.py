"""Seeded synthetic workloads shared by the oracle side and the GPU side.

This module holds configuration data (grid, lattice, fractional orders,
skewness, diffusion tensor, velocity, relaxation times) and seeded generators
of initial concentrations and sources.  It contains none of the method's
arithmetic: no fractional weights, no equilibrium, no relaxation, no
streaming.  The workload shapes follow the paper's tests: Gaussian plumes in a
square or cubic box with homogeneous Dirichlet walls (Sec. 3.2, Gaussian hill
initial condition), written here in lattice units (dx = dt = 1).

Readings used for every workload (the paper fixes none of them in lattice
units): g = 1 on every axis, every free relaxation time = 1, the relaxation
time of the mass moment = 1 (it has no effect), wall value 0.
"""
from __future__ import annotations

import copy
import math

import numpy as np

_COMMON = dict(dx=1.0, dt=1.0, collision="MRT", tau_free=[1.0, 1.0, 1.0, 1.0], tau0=1.0, c_wall=0.0)


def _rot30_D(l1: float, l2: float):
    """R(+30 deg) diag(l1, l2) R(+30 deg)^T: a rotated anisotropic tensor."""
    c, s = math.cos(math.pi / 6), math.sin(math.pi / 6)
    R = np.array([[c, -s], [s, c]])
    D = R @ np.diag([l1, l2]) @ R.T
    return (0.5 * (D + D.T)).tolist()


CONFIGS = {
    # small case the oracle finishes in seconds
    "c1_64sq": dict(_COMMON, dim=2, n=[64, 64], steps=200, alpha=[1.5, 1.5], p=[0.5, 0.5], g=[1.0, 1.0],
                    D=[[0.1, 0.0], [0.0, 0.1]], u=[0.0, 0.0],
                    init=dict(kind="gauss", sigma=3.0, center=[31.5, 31.5], amp=1.0)),
    # the benchmark workload
    "c2_1024sq": dict(_COMMON, dim=2, n=[1024, 1024], steps=2000, alpha=[1.3, 1.7], p=[0.3, 0.8], g=[1.0, 1.0],
                      D=_rot30_D(0.05, 0.2), u=[0.05, 0.02],
                      init=dict(kind="pulses", count=8, sigma=[4.0, 20.0], amp=[0.5, 1.0], seed=2)),
    "c3_256cube": dict(_COMMON, dim=3, n=[256, 256, 256], steps=500, alpha=[1.5, 1.6, 1.8], p=[0.5, 0.2, 0.9],
                       g=[1.0, 1.0, 1.0], D=[[0.1, 0, 0], [0, 0.05, 0], [0, 0, 0.02]], u=[0.03, 0.0, 0.0],
                       init=dict(kind="gauss", sigma=6.0, center=[127.5, 127.5, 127.5], amp=1.0),
                       source=dict(kind="point", node=[64, 128, 128], value=1e-3)),
    "c4_4096sq": dict(_COMMON, dim=2, n=[4096, 4096], steps=1000, alpha=[1.2, 1.9], p=[1.0, 0.0], g=[1.0, 1.0],
                      D=[[0.1, 0.0], [0.0, 0.1]], u=[0.02, 0.02],
                      init=dict(kind="pulses", count=8, sigma=[4.0, 20.0], amp=[0.5, 1.0], seed=4)),
    # adjoint workload: hidden parameters that generate the observed plume ...
    "c5_512sq_hidden": dict(_COMMON, dim=2, n=[512, 512], steps=500, alpha=[1.6, 1.4], p=[0.6, 0.4], g=[1.0, 1.0],
                            D=[[0.08, 0.03], [0.03, 0.15]], u=[0.04, -0.01], ckpt_every=50,
                            init=dict(kind="pulses", count=8, sigma=[4.0, 20.0], amp=[0.5, 1.0], seed=5)),
    # ... and the point at which the gradient is evaluated
    "c5_512sq_eval": dict(_COMMON, dim=2, n=[512, 512], steps=500, alpha=[1.6, 1.4], p=[0.5, 0.5], g=[1.0, 1.0],
                          D=[[0.1, 0.0], [0.0, 0.1]], u=[0.0, 0.0], ckpt_every=50,
                          init=dict(kind="pulses", count=8, sigma=[4.0, 20.0], amp=[0.5, 1.0], seed=5)),
}


def config(name: str, **overrides) -> dict:
    """A deep copy of a named configuration with optional overrides."""
    cfg = copy.deepcopy(CONFIGS[name])
    cfg["name"] = name
    cfg.update(copy.deepcopy(overrides))
    return cfg


def shape(cfg: dict):
    """Array shape of a node field, slowest axis first: (ny, nx) or (nz, ny, nx)."""
    return tuple(int(v) for v in reversed(cfg["n"][: cfg["dim"]]))


def nodes(cfg: dict) -> int:
    return int(np.prod(cfg["n"][: cfg["dim"]]))


def _coords(cfg: dict):
    d = cfg["dim"]
    axes = [np.arange(cfg["n"][mu], dtype=np.float64) for mu in range(d)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")  # slowest first
    return list(reversed(grids))  # grids[mu] = coordinate along axis mu


def gaussian(cfg: dict, center, sigma: float, amp: float = 1.0) -> np.ndarray:
    """Peak-amp Gaussian hill (the paper's initial condition, Sec. 3.2) in node units."""
    X = _coords(cfg)
    r2 = sum((X[mu] - center[mu]) ** 2 for mu in range(cfg["dim"]))
    return amp * np.exp(-0.5 * r2 / sigma**2)


def initial_C(cfg: dict) -> np.ndarray:
    """Seeded initial concentration in FP64, shape ``shape(cfg)``."""
    spec = cfg["init"]
    if spec["kind"] == "gauss":
        return gaussian(cfg, spec["center"], spec["sigma"], spec.get("amp", 1.0))
    if spec["kind"] == "pulses":
        rng = np.random.default_rng(spec["seed"])
        C = np.zeros(shape(cfg))
        for _ in range(spec["count"]):
            sig = rng.uniform(*spec["sigma"])
            amp = rng.uniform(*spec["amp"])
            ctr = [rng.uniform(3 * sig, cfg["n"][mu] - 1 - 3 * sig) for mu in range(cfg["dim"])]
            C += gaussian(cfg, ctr, sig, amp)
        return C
    if spec["kind"] == "random":
        rng = np.random.default_rng(spec["seed"])
        return rng.uniform(spec.get("low", 0.0), spec.get("high", 1.0), size=shape(cfg))
    raise ValueError(spec["kind"])


def source(cfg: dict):
    """Constant-in-time source field S (FP64) or None."""
    spec = cfg.get("source")
    if not spec:
        return None
    S = np.zeros(shape(cfg))
    if spec["kind"] == "point":
        idx = tuple(reversed(spec["node"]))
        S[idx] = spec["value"]
        return S
    if spec["kind"] == "random":
        rng = np.random.default_rng(spec["seed"])
        return rng.uniform(-spec["scale"], spec["scale"], size=shape(cfg))
    raise ValueError(spec["kind"])


def small(dim: int, n, *, seed: int = 0, collision: str = "MRT", alpha=None, p=None, D=None, u=None,
          with_source: bool = False, **kw) -> dict:
    """A small random test problem (several GEMM tiles plus a ragged tail when n is odd-sized)."""
    rng = np.random.default_rng(seed)
    d = dim
    cfg = dict(_COMMON, dim=d, n=list(n), steps=kw.pop("steps", 10), collision=collision,
               alpha=list(alpha) if alpha is not None else list(rng.uniform(1.2, 1.95, d)),
               p=list(p) if p is not None else list(rng.uniform(0.0, 1.0, d)),
               g=[1.0] * d,
               u=list(u) if u is not None else list(rng.uniform(-0.03, 0.03, d)),
               init=dict(kind="random", seed=seed + 1000, low=0.0, high=1.0))
    if D is None:
        A = rng.uniform(-0.03, 0.03, (d, d))
        D = (np.diag(rng.uniform(0.05, 0.2, d)) + 0.5 * (A + A.T)).tolist()
        if collision == "BGK":
            v = float(rng.uniform(0.05, 0.2))
            D = (v * np.eye(d)).tolist()
    cfg["D"] = D
    if with_source:
        cfg["source"] = dict(kind="random", seed=seed + 2000, scale=1e-3)
    cfg.update(kw)
    return cfg


# ---------------------------------------------------------------------------
# Power-law problems with an exact solution (Sec. 3.4, equations (Def_D_AS)
# and (exsolFADE_3D)): on [0, L]^d with p = 1, u = 0, g = 1,
#   D_mumu(x) = x_mu^alpha_mu Gamma(a_mu + 2 - alpha_mu) / Gamma(a_mu + 2),
#   S(x, t)   = -(d + 1) e^-t prod_mu x_mu^a_mu,
#   C(x, t)   = e^-t prod_mu x_mu^a_mu  (also the initial and wall values).
# With eps != 0 (2D only) the tensor also gets the off-diagonal entry
# D_01 = D_10 = eps x_0 x_1, and the source gains the divergence of the extra
# flux, S -= e^-t eps [G_1 (a_0 + 1) x_0^a_0 x_1^(a_1 + 2 - alpha_1)
#                      + G_0 (a_1 + 1) x_1^a_1 x_0^(a_0 + 2 - alpha_0)],
# G_mu = Gamma(a_mu + 1) / Gamma(a_mu + 2 - alpha_mu), because the left
# Riemann-Liouville derivative of order alpha - 1 of x^a is
# G x^(a + 1 - alpha).  These fields are problem data, not the method.

class PowerLawProblem:
    """Fields of the exact-solution workload on an n^d grid (walls included)."""

    def __init__(self, dim: int, n: int, dt: float, *, alpha=None, a=None, eps: float = 0.0, length: float = 1.0,
                 D_const: float = 0.5, tau_free: float = 1.0):
        if eps != 0.0 and dim != 2:
            raise ValueError("the off-diagonal variant is 2D")
        self.dim = d = dim
        self.alpha = list(alpha) if alpha is not None else ([1.5, 1.7] if d == 2 else [1.5, 1.7, 1.9])
        self.a = list(a) if a is not None else ([0.4, 0.7] if d == 2 else [2.0, 2.0, 2.0])
        self.eps = float(eps)
        dx = length / (n - 1)
        self.cfg = dict(dim=d, n=[n] * d, dx=dx, dt=float(dt), collision="MRT", alpha=self.alpha, p=[1.0] * d,
                        g=[1.0] * d, u=[0.0] * d, D=(D_const * np.eye(d)).tolist(), tau_free=[tau_free] * 4,
                        tau0=1.0, c_wall=0.0, steps=0, name=f"powerlaw_{d}d_{n}")
        x = np.arange(n, dtype=np.float64) * dx
        grids = np.meshgrid(*([x] * d), indexing="ij")  # slowest first
        X = list(reversed(grids))                        # X[mu]: coordinate along axis mu
        al, aa = self.alpha, self.a
        self.base = np.ones(X[0].shape)
        for mu in range(d):
            self.base = self.base * X[mu] ** aa[mu]
        self.D = np.zeros((d, d) + self.base.shape)
        for mu in range(d):
            self.D[mu, mu] = X[mu] ** al[mu] * math.gamma(aa[mu] + 2 - al[mu]) / math.gamma(aa[mu] + 2)
        self.extra = np.zeros(self.base.shape)
        if self.eps != 0.0:
            self.D[0, 1] = self.D[1, 0] = self.eps * X[0] * X[1]
            G0 = math.gamma(aa[0] + 1) / math.gamma(aa[0] + 2 - al[0])
            G1 = math.gamma(aa[1] + 1) / math.gamma(aa[1] + 2 - al[1])
            self.extra = self.eps * (G1 * (aa[0] + 1) * X[0] ** aa[0] * X[1] ** (aa[1] + 2 - al[1])
                                     + G0 * (aa[1] + 1) * X[1] ** aa[1] * X[0] ** (aa[0] + 2 - al[0]))

    def exact(self, t: float) -> np.ndarray:
        return math.exp(-t) * self.base

    def source(self, t: float) -> np.ndarray:
        return -math.exp(-t) * ((self.dim + 1) * self.base + self.extra)

    def schedule32(self, m: int):
        """The FP32 fields an FP32 run receives before step m: the source at
        t_m and the wall values at t_{m+1} (t = m dt), each formed in FP32
        from the FP32-rounded base fields and time factors.  Giving these to
        both sides keeps input rounding out of a parity comparison."""
        dt = self.cfg["dt"]
        e0, e1 = np.float32(math.exp(-m * dt)), np.float32(math.exp(-(m + 1) * dt))
        b, x = self.base.astype(np.float32), self.extra.astype(np.float32)
        S = np.float32(-(self.dim + 1)) * e0 * b - e0 * x
        return S.astype(np.float32), (e1 * b).astype(np.float32)


def random_tensor_field(cfg: dict, seed: int, zero_fraction: float = 0.05) -> np.ndarray:
    """Seeded field of symmetric positive semi-definite d x d tensors, shape
    (d, d, *shape): diagonal entries in [0.02, 0.3], off-diagonal entries
    scaled to keep every node's tensor definite, and a fraction of nodes with
    D = 0 (the semi-definite limit).  Values are FP32-representable."""
    d = cfg["dim"]
    shp = shape(cfg)
    rng = np.random.default_rng(seed)
    diag = rng.uniform(0.02, 0.3, (d,) + shp)
    D = np.zeros((d, d) + shp)
    for a in range(d):
        D[a, a] = diag[a]
    for a in range(d):
        for b in range(a + 1, d):
            r = rng.uniform(-0.45, 0.45, shp) / max(d - 1, 1)
            D[a, b] = D[b, a] = r * np.sqrt(diag[a] * diag[b])
    zero = rng.random(shp) < zero_fraction
    D[:, :, zero] = 0.0
    return D.astype(np.float32).astype(np.float64)


def random_wall_values(cfg: dict, seed: int) -> np.ndarray:
    """Seeded field of Dirichlet values in [-0.5, 1] (only wall entries matter)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5, 1.0, shape(cfg)).astype(np.float32).astype(np.float64)


class CaputoPowerLawProblem:
    """Exact-solution workload of the Caputo-type flux variant (Sec. 3.5,
    equations (Fg2), (SourceTerm_PS)): on [0, 1]^d with p = 1, u = 0, g = 1,
    constant diagonal D = diag(D_mu),
        C(x, t) = e^-t prod_mu (x_mu^beta_mu + a_mu),
        S(x, t) = -C - e^-t sum_mu D_mu Gamma(beta_mu + 1) / Gamma(beta_mu + 1 - alpha_mu)
                        x_mu^(beta_mu - alpha_mu) prod_{nu != mu} (x_nu^beta_nu + a_nu),
    because I+^(2-alpha) d/dx x^beta = Gamma(beta + 1) / Gamma(beta + 2 - alpha)
    x^(beta + 1 - alpha).  beta = alpha is the paper's case (the source then
    has the constant factors Gamma(alpha_mu + 1)).  Problem data, not the method."""

    def __init__(self, dim: int, n: int, dt: float, *, alpha=None, a=None, beta=None, Dmu=None,
                 tau_free: float = 1.0):
        self.dim = d = dim
        self.alpha = list(alpha) if alpha is not None else ([1.7, 1.2] if d == 2 else [1.7, 1.2, 1.5])
        self.a = list(a) if a is not None else ([0.3, 1.2] if d == 2 else [0.3, 1.2, 0.5])
        self.beta = list(beta) if beta is not None else list(self.alpha)
        self.Dmu = list(Dmu) if Dmu is not None else [1.0] * d
        dx = 1.0 / (n - 1)
        self.cfg = dict(dim=d, n=[n] * d, dx=dx, dt=float(dt), collision="MRT", alpha=self.alpha, p=[1.0] * d,
                        g=[1.0] * d, u=[0.0] * d, D=np.diag(self.Dmu).tolist(), tau_free=[tau_free] * 4, tau0=1.0,
                        c_wall=0.0, flux_form="caputo", steps=0, name=f"caputo_{d}d_{n}")
        x = np.arange(n, dtype=np.float64) * dx
        grids = np.meshgrid(*([x] * d), indexing="ij")
        X = list(reversed(grids))
        fac = [X[mu] ** self.beta[mu] + self.a[mu] for mu in range(d)]
        self.base = np.ones(X[0].shape)
        for mu in range(d):
            self.base = self.base * fac[mu]
        self.flux_div = np.zeros(self.base.shape)
        for mu in range(d):
            b, al = self.beta[mu], self.alpha[mu]
            term = self.Dmu[mu] * math.gamma(b + 1) / math.gamma(b + 1 - al) * X[mu] ** (b - al)
            for nu in range(d):
                if nu != mu:
                    term = term * fac[nu]
            self.flux_div += term

    def exact(self, t: float) -> np.ndarray:
        return math.exp(-t) * self.base

    def source(self, t: float) -> np.ndarray:
        return -math.exp(-t) * (self.base + self.flux_div)

    def schedule32(self, m: int):
        """The FP32 source (t_m) and wall values (t_{m+1}) an FP32 run receives
        before step m, formed in FP32 from the FP32-rounded base fields."""
        dt = self.cfg["dt"]
        e0, e1 = np.float32(math.exp(-m * dt)), np.float32(math.exp(-(m + 1) * dt))
        b, fl = self.base.astype(np.float32), self.flux_div.astype(np.float32)
        S = -(e0 * (b + fl))
        return S.astype(np.float32), (e1 * b).astype(np.float32)


# ---------------------------------------------------------------------------
# High-Peclet stability workload of Sec. 3.3: Omega = [0, 2] x [0, 1],
# dx = 0.01 (201 x 101 nodes), dt = 8e-4, D = 2e-3 Id (BGK relaxation time
# 0.548), p = 1/2, g = 1, u = (u1, 0), homogeneous Dirichlet walls, and the
# paper's Gaussian hill (Gaussian_IC_3D) with sigma_0 = 0.002, C_0 = 5 centred
# at (0.5, 0.5).  alpha = 2 is the advection-diffusion case.

def stability_config(alpha: float, u1: float, collision: str, tau_free: float = 1.0) -> dict:
    return dict(dim=2, n=[201, 101], dx=0.01, dt=8e-4, alpha=[alpha, alpha], p=[0.5, 0.5], g=[1.0, 1.0],
                D=[[2e-3, 0.0], [0.0, 2e-3]], u=[u1, 0.0], collision=collision, tau_free=[tau_free] * 4,
                tau0=1.0, c_wall=0.0, steps=1250,
                name=f"stability_a{alpha}_u{u1}_{collision}_{tau_free}")


def paper_gaussian(cfg: dict, center, sigma0: float = 0.002, C0: float = 5.0) -> np.ndarray:
    """Equation (Gaussian_IC_3D) sampled at the nodes (physical coordinates)."""
    d = cfg["dim"]
    dx = cfg["dx"]
    X = _coords(cfg)
    r2 = sum((X[mu] * dx - center[mu]) ** 2 for mu in range(d))
    return C0 / (2 * math.pi * sigma0 ** 2) ** (d / 2) * np.exp(-0.5 * r2 / sigma0 ** 2)
