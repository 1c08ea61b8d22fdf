"""ORACLE -- test infrastructure only.

Python access to the plain FP64 CPU implementation in ``fade_oracle.c`` of the
lattice Boltzmann scheme for the space-fractional advection-diffusion equation
(Cartalade, Younsi, Neel, arXiv:1706.09161).  Only ``tests/``, the smoke check
and the benchmark's CPU-baseline leg import this package; the GPU library never
does.  It shares no code with the GPU path: both sides read their inputs from
``synth`` (seeded generators that hold none of the method's arithmetic).

``adjoint`` is the hand-written FP64 adjoint (vector-Jacobian product) of n steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfade_oracle.so")
_SOURCES = ["fade_oracle.c", "random_walk.c"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
               "-o", tmp, *srcs, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Problem(ctypes.Structure):
    """Mirror of ``fo_problem`` in fade_oracle.c."""

    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("collision", ctypes.c_int32),
        ("flux_form", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("alpha", ctypes.c_double * 3),
        ("p", ctypes.c_double * 3),
        ("g", ctypes.c_double * 3),
        ("D", ctypes.c_double * 9),
        ("u", ctypes.c_double * 3),
        ("tau_free", ctypes.c_double * 4),
        ("tau0", ctypes.c_double),
        ("c_wall", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        sig = {
            "fo_lattice": (ctypes.c_int, [ctypes.c_int32, i32p, i32p, dp, dp]),
            "fo_cplus": (ctypes.c_double, [ctypes.c_int64, ctypes.c_int64, ctypes.c_double]),
            "fo_cminus": (ctypes.c_double, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_double]),
            "fo_phi": (ctypes.c_int, [P, dp, dp]),
            "fo_phi_at": (ctypes.c_int, [P, dp, ip, ctypes.c_int64, dp]),
            "fo_collision_matrices": (ctypes.c_int, [P, dp, dp, dp, dp]),
            "fo_equilibrium": (ctypes.c_int, [P, ctypes.c_double, dp, dp]),
            "fo_collide_node": (ctypes.c_int, [P, dp, ctypes.c_double, dp, ctypes.c_double, dp]),
            "fo_moment": (ctypes.c_int, [P, dp, dp]),
            "fo_init": (ctypes.c_int, [P, dp, dp]),
            "fo_init_var": (ctypes.c_int, [P, dp, dp, dp]),
            "fo_step": (ctypes.c_int, [P, dp, dp, ctypes.c_int64]),
            "fo_step_var": (ctypes.c_int, [P, dp, dp, dp, dp, ctypes.c_int64]),
            "fo_step_sampled": (ctypes.c_int, [P, dp, dp, ip, ctypes.c_int64, dp]),
            "fo_threads": (ctypes.c_int, []),
            "fo_flush_subnormals": (ctypes.c_int, [ctypes.c_int]),
        }
        sig["fo_adjoint"] = (ctypes.c_int, [P, dp, dp, ctypes.c_int64, dp, dp, dp, dp, dp, dp])
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def make_problem(cfg: dict) -> Problem:
    """Build the C struct from a plain configuration dict (see ``synth``)."""
    P = Problem()
    d = int(cfg["dim"])
    P.dim = d
    for mu in range(3):
        P.n[mu] = int(cfg["n"][mu]) if mu < d else 1
    P.collision = {"BGK": 0, "MRT": 1}[cfg.get("collision", "MRT")]
    P.flux_form = {"rl": 0, "caputo": 1}[cfg.get("flux_form", "rl")]
    P.dx = float(cfg.get("dx", 1.0))
    P.dt = float(cfg.get("dt", 1.0))
    for mu in range(d):
        P.alpha[mu] = float(cfg["alpha"][mu])
        P.p[mu] = float(cfg["p"][mu])
        P.g[mu] = float(cfg.get("g", [1.0] * d)[mu])
        P.u[mu] = float(cfg.get("u", [0.0] * d)[mu])
    D = np.asarray(cfg["D"], dtype=np.float64).reshape(d, d)
    for a in range(d):
        for b in range(d):
            P.D[a * d + b] = float(D[a, b])
    tf = cfg.get("tau_free", [1.0] * 4)
    for k in range(4):
        P.tau_free[k] = float(tf[k]) if k < len(tf) else 1.0
    P.tau0 = float(cfg.get("tau0", 1.0))
    P.c_wall = float(cfg.get("c_wall", 0.0))
    return P


def shape_of(cfg: dict):
    """Array shape (slowest first) of a node field: (ny, nx) or (nz, ny, nx)."""
    return tuple(int(v) for v in reversed(cfg["n"][: cfg["dim"]]))


def Q_of(cfg: dict) -> int:
    return 2 * int(cfg["dim"]) + 1


def lattice(dim: int):
    Q = ctypes.c_int32()
    e = np.zeros(21, dtype=np.int32)
    w = np.zeros(7)
    e2 = ctypes.c_double()
    _check(lib().fo_lattice(dim, ctypes.byref(Q), e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                            ctypes.byref(e2)), "lattice")
    q = Q.value
    return e.reshape(7, 3)[:q, :dim].copy(), w[:q].copy(), e2.value


def cplus(l: int, n: int, gamma: float) -> float:
    return lib().fo_cplus(l, n, gamma)


def cminus(l: int, n: int, N: int, gamma: float) -> float:
    return lib().fo_cminus(l, n, N, gamma)


def phi(cfg: dict, C: np.ndarray) -> np.ndarray:
    """Fractional terms Phi_mu for every node: array (d, *shape)."""
    P = make_problem(cfg)
    C = np.ascontiguousarray(C, dtype=np.float64).reshape(shape_of(cfg))
    out = np.zeros((cfg["dim"],) + C.shape)
    _check(lib().fo_phi(ctypes.byref(P), _dp(C), _dp(out)), "phi")
    return out


def phi_at(cfg: dict, C: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    P = make_problem(cfg)
    C = np.ascontiguousarray(C, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((cfg["dim"], nodes.size))
    _check(lib().fo_phi_at(ctypes.byref(P), _dp(C), _ip(nodes), nodes.size, _dp(out)), "phi_at")
    return out


def collision_matrices(cfg: dict):
    P = make_problem(cfg)
    Q = Q_of(cfg)
    M = np.zeros((Q, Q))
    Mi = np.zeros((Q, Q))
    Lam = np.zeros((Q, Q))
    lam = ctypes.c_double()
    _check(lib().fo_collision_matrices(ctypes.byref(P), _dp(M), _dp(Mi), _dp(Lam), ctypes.byref(lam)),
           "collision_matrices")
    return M, Mi, Lam, lam.value


def equilibrium(cfg: dict, C: float, phi_node) -> np.ndarray:
    P = make_problem(cfg)
    ph = np.ascontiguousarray(phi_node, dtype=np.float64)
    out = np.zeros(Q_of(cfg))
    _check(lib().fo_equilibrium(ctypes.byref(P), float(C), _dp(ph), _dp(out)), "equilibrium")
    return out


def collide_node(cfg: dict, f_node, C: float, phi_node, S: float = 0.0) -> np.ndarray:
    P = make_problem(cfg)
    f = np.ascontiguousarray(f_node, dtype=np.float64)
    ph = np.ascontiguousarray(phi_node, dtype=np.float64)
    out = np.zeros(Q_of(cfg))
    _check(lib().fo_collide_node(ctypes.byref(P), _dp(f), float(C), _dp(ph), float(S), _dp(out)), "collide")
    return out


def moment(cfg: dict, f: np.ndarray) -> np.ndarray:
    P = make_problem(cfg)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(shape_of(cfg))
    _check(lib().fo_moment(ctypes.byref(P), _dp(f), _dp(out)), "moment")
    return out


def _field(cfg: dict, a, lead=()):
    """A node field (or stack of fields) as contiguous FP64, or None."""
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(tuple(lead) + shape_of(cfg))
    return a, _dp(a)


def init(cfg: dict, C0: np.ndarray, Cw: np.ndarray | None = None) -> np.ndarray:
    """Initial populations f = f^eq(C0 with walls := Dirichlet value): array (Q, *shape).

    Cw (optional) is a node field of Dirichlet values (its wall entries are
    used); without it every wall node takes cfg's c_wall.
    """
    P = make_problem(cfg)
    C0 = np.ascontiguousarray(C0, dtype=np.float64).reshape(shape_of(cfg))
    f = np.zeros((Q_of(cfg),) + C0.shape)
    if Cw is None:
        _check(lib().fo_init(ctypes.byref(P), _dp(C0), _dp(f)), "init")
    else:
        Cw, Cwp = _field(cfg, Cw)
        _check(lib().fo_init_var(ctypes.byref(P), _dp(C0), Cwp, _dp(f)), "init_var")
    return f


def step(cfg: dict, f: np.ndarray, nsteps: int, S: np.ndarray | None = None, D: np.ndarray | None = None,
         Cw: np.ndarray | None = None) -> np.ndarray:
    """Advance populations by nsteps time steps; returns a new array.

    Optional space-dependent coefficients (constant over the nsteps): S the
    source field, D the diffusion tensor of every node, shape (d, d, *shape)
    (MRT only), Cw the Dirichlet value of every node (wall entries used).
    """
    P = make_problem(cfg)
    d = int(cfg["dim"])
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    S, Sp = _field(cfg, S)
    if D is None and Cw is None:
        _check(lib().fo_step(ctypes.byref(P), _dp(f), Sp, int(nsteps)), "step")
        return f
    D, Dp = _field(cfg, D, (d, d))
    Cw, Cwp = _field(cfg, Cw)
    _check(lib().fo_step_var(ctypes.byref(P), _dp(f), Sp, Dp, Cwp, int(nsteps)), "step_var")
    return f


def step_sampled(cfg: dict, f: np.ndarray, nodes: np.ndarray, S: np.ndarray | None = None) -> np.ndarray:
    """One step from full state f, evaluated at the given flat node indices: (Q, count)."""
    P = make_problem(cfg)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    Sp = None
    if S is not None:
        S = np.ascontiguousarray(S, dtype=np.float64)
        Sp = _dp(S)
    out = np.zeros((Q_of(cfg), nodes.size))
    _check(lib().fo_step_sampled(ctypes.byref(P), _dp(f), Sp, _ip(nodes), nodes.size, _dp(out)), "step_sampled")
    return out


def threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP)."""
    return int(lib().fo_threads())


def flush_subnormals(on: bool = True) -> None:
    """Read and write subnormal FP64 values as zero in the oracle's threads (x86
    DAZ/FTZ; see fo_flush_subnormals).  For long golden runs only."""
    if int(lib().fo_flush_subnormals(1 if on else 0)) != 0:
        raise RuntimeError("subnormal flushing is not available on this CPU")


def run(cfg: dict, C0: np.ndarray, nsteps: int, S: np.ndarray | None = None) -> np.ndarray:
    """C after nsteps from the initial concentration C0."""
    f = init(cfg, C0)
    f = step(cfg, f, nsteps, S)
    return moment(cfg, f)


def adjoint(cfg: dict, C0: np.ndarray, nsteps: int, gC: np.ndarray, S: np.ndarray | None = None):
    """Gradients of L = <gC, C_n> (FP64): dict with dC0, dS (fields), D (d x d, symmetrised), u, p."""
    P = make_problem(cfg)
    shp = shape_of(cfg)
    d = int(cfg["dim"])
    C0 = np.ascontiguousarray(C0, dtype=np.float64).reshape(shp)
    gC = np.ascontiguousarray(gC, dtype=np.float64).reshape(shp)
    Sp = None
    if S is not None:
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(shp)
        Sp = _dp(S)
    dC0 = np.zeros(shp)
    dS = np.zeros(shp)
    dD = np.zeros(9)
    du = np.zeros(3)
    dpv = np.zeros(3)
    _check(lib().fo_adjoint(ctypes.byref(P), _dp(C0), Sp, int(nsteps), _dp(gC), _dp(dC0), _dp(dS), _dp(dD), _dp(du),
                            _dp(dpv)), "adjoint")
    return {"dC0": dC0, "dS": dS, "D": dD[: d * d].reshape(d, d), "u": du[:d], "p": dpv[:d]}


def loss(cfg: dict, C0: np.ndarray, nsteps: int, gC: np.ndarray, S: np.ndarray | None = None) -> float:
    """L = <gC, C_n> by the forward oracle."""
    return float(np.sum(np.asarray(gC, np.float64) * run(cfg, C0, nsteps, S=S)))


# ---------------------------------------------------------------------------
# Levy-stable random walk (random_walk.c)

class RWParams(ctypes.Structure):
    """Mirror of ``fo_rw_params`` in random_walk.c."""

    _fields_ = [
        ("dim", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("alpha", ctypes.c_double * 3),
        ("p", ctypes.c_double * 3),
        ("D", ctypes.c_double * 3),
        ("g", ctypes.c_double * 3),
        ("u", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


_rw_sig_done = False


def _rw_lib():
    global _rw_sig_done
    L = lib()
    if not _rw_sig_done:
        R = ctypes.POINTER(RWParams)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64, u32, u64 = ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "fo_philox4x32_10": (None, [u32p, u32p, u32p]),
            "fo_rw_uniforms": (None, [u64, i64, u32, u32, dp]),
            "fo_stable_from": (ctypes.c_double, [ctypes.c_double] * 4),
            "fo_stable_draw": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, u64, i64, u32, u32]),
            "fo_rw_init_gaussian": (ctypes.c_int, [R, dp, ctypes.c_double, i64, i64, dp, u8p]),
            "fo_rw_walk": (ctypes.c_int, [R, dp, u8p, i64, i64, i64, i64]),
            "fo_rw_histogram": (ctypes.c_int, [R, dp, u8p, i64, i32p, ctypes.c_double, u32p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _rw_sig_done = True
    return L


def rw_params(dim, lo, hi, alpha, p, D, g=None, u=None, dt=1e-3, seed=1) -> RWParams:
    P = RWParams()
    P.dim = int(dim)
    for mu in range(dim):
        P.lo[mu], P.hi[mu] = float(lo[mu]), float(hi[mu])
        P.alpha[mu], P.p[mu], P.D[mu] = float(alpha[mu]), float(p[mu]), float(D[mu])
        P.g[mu] = 1.0 if g is None else float(g[mu])
        P.u[mu] = 0.0 if u is None else float(u[mu])
    P.dt = float(dt)
    P.seed = int(seed)
    return P


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    _rw_lib().fo_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def rw_uniforms(seed: int, particle: int, step: int, purpose: int):
    u = np.zeros(2)
    _rw_lib().fo_rw_uniforms(int(seed), int(particle), int(step), int(purpose), _dp(u))
    return u


def stable_from(alpha, beta, V, W) -> float:
    return float(_rw_lib().fo_stable_from(float(alpha), float(beta), float(V), float(W)))


def stable_draws(alpha, beta, seed, count, step=1, purpose=0) -> np.ndarray:
    L = _rw_lib()
    return np.array([L.fo_stable_draw(float(alpha), float(beta), int(seed), k, int(step), int(purpose))
                     for k in range(int(count))])


def rw_init_gaussian(P: RWParams, center, sigma0: float, n: int, first: int = 0):
    """(x (dim, n), alive (n,)) of particles first .. first + n - 1."""
    x = np.zeros((P.dim, n))
    alive = np.zeros(n, np.uint8)
    c = np.zeros(3)
    c[: P.dim] = center
    rc = _rw_lib().fo_rw_init_gaussian(ctypes.byref(P), _dp(c), float(sigma0), int(n), int(first), _dp(x),
                                       alive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    _check(rc, "rw_init_gaussian")
    return x, alive


def rw_walk(P: RWParams, x, alive, nsteps: int, first: int = 0, step0: int = 0):
    """Steps step0 + 1 .. step0 + nsteps; returns new (x, alive)."""
    x = np.array(x, np.float64, order="C", copy=True)
    alive = np.array(alive, np.uint8, copy=True)
    n = alive.size
    rc = _rw_lib().fo_rw_walk(ctypes.byref(P), _dp(x), alive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), n,
                              int(first), int(step0), int(nsteps))
    _check(rc, "rw_walk")
    return x, alive


def rw_histogram(P: RWParams, x, alive, nodes, dx: float) -> np.ndarray:
    """Counts of living particles per node, array of shape reversed(nodes)."""
    x = np.ascontiguousarray(x, np.float64)
    alive = np.ascontiguousarray(alive, np.uint8)
    nn = np.zeros(3, np.int32)
    nn[: P.dim] = nodes
    counts = np.zeros(int(np.prod(nodes)), np.uint32)
    rc = _rw_lib().fo_rw_histogram(ctypes.byref(P), _dp(x), alive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   alive.size, nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(dx),
                                   counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    _check(rc, "rw_histogram")
    return counts.reshape(tuple(reversed(list(nodes))))
