"""GPU parity of the space-dependent coefficients: a diffusion tensor D(x)
(per-node flux block of Lambda, Sec. 2.3), per-node Dirichlet values and
time-dependent sources and walls (Sec. 2.5, Sec. 3.4), through the C ABI
(lbm_fade_set_diffusion, lbm_fade_set_wall, lbm_fade_set_source) against the
FP64 oracle (fo_step_var) on the same seeded inputs, and against the exact
power-law solution of Sec. 3.4.

Tolerances follow the constant-coefficient parity tests: one step from the
same FP32 populations within 2e-6 of the largest population, runs within
relative L2 1e-5 (FP32) or 1e-4 (split-BF16).  The per-node block reaches
the kernel as FP32 lambda-bar(x)^-1 - lambda-bar^-1 computed in FP64, an
extra rounding of 2^-24 relative on the flux block.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(cfg, precision="fp32", **kw):
    from paper_1706_09161_amd import LbmFade

    return LbmFade.from_config(cfg, precision=precision, **kw)


def _rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def _banner(msg):
    print(f"[gpu-variable] {msg}", flush=True)


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32)


STEP_CASES = [
    # (dim, n, precision, with_source): several 64-column strips and row chunks plus ragged tails
    (2, [150, 97], "fp32", True),
    (2, [37, 29], "fp32", False),
    (2, [3, 3], "fp32", True),
    (2, [130, 70], "bf16x3", True),
    (3, [70, 37, 23], "fp32", True),
    (3, [19, 14, 11], "fp32", False),
    (3, [33, 20, 9], "bf16x3", True),
]


@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}-{c[2]}-S{int(c[3])}")
def test_one_step_with_fields_matches_oracle(case):
    """One step from the same population state with a random D(x) (including
    nodes with D = 0) and random wall values: every population of every node."""
    dim, n, precision, with_source = case
    _banner(f"one-step var dim={dim} n={n} {precision} src={with_source}")
    cfg = synth.small(dim, n, seed=61, with_source=with_source, c_wall=0.2)
    S = synth.source(cfg)
    D = synth.random_tensor_field(cfg, seed=62)
    Cw = synth.random_wall_values(cfg, seed=63)
    f0 = oracle.init(cfg, synth.initial_C(cfg), Cw=Cw)
    f0 = oracle.step(cfg, f0, 2, S=S, D=D, Cw=Cw)
    f32 = f0.astype(np.float32)
    Sref = None if S is None else _f32(S).astype(np.float64)
    ref = oracle.step(cfg, f32.astype(np.float64), 1, S=Sref, D=D, Cw=Cw)
    with _solver(cfg, precision) as s:
        s.set_diffusion(_f32(D))
        s.set_wall(torch.from_numpy(_f32(Cw)).cuda())
        s.set_f(torch.from_numpy(f32).cuda())
        if S is not None:
            s.set_source(_f32(S))
        s.step(1)
        got = s.get_f(device=False).astype(np.float64)
        C = s.get_C(device=False).astype(np.float64)
    scale = np.abs(f0).max()
    tol = 2e-6 if precision == "fp32" else 2e-5
    err = np.abs(got - ref).max() / scale
    _banner(f"max err / max |f| = {err:.2e}")
    assert err <= tol
    assert np.abs(C - ref.sum(axis=0)).max() <= tol * scale


@pytest.mark.parametrize("dim,n", [(2, [75, 58]), (3, [24, 19, 21])])
def test_constant_fields_match_constant_path(dim, n):
    """A D field equal to the handle's tensor and a wall field equal to c_wall
    (FP32-exact values, so the per-node correction is exactly zero) run the
    space-dependent kernels and must reproduce the constant path."""
    _banner(f"constant fields dim={dim} n={n}")
    D = (np.diag([0.125, 0.0625, 0.25][:dim]) + 0.015625 * (np.ones((dim, dim)) - np.eye(dim))).tolist()
    cfg = synth.small(dim, n, seed=65, with_source=True, c_wall=0.375, D=D)
    C0 = synth.initial_C(cfg).astype(np.float32)
    S = synth.source(cfg).astype(np.float32)
    shp = synth.shape(cfg)
    Dfield = np.broadcast_to(np.asarray(D, np.float32).reshape((dim, dim) + (1,) * dim), (dim, dim) + shp).copy()
    out = []
    for var in (False, True):
        with _solver(cfg) as s:
            if var:
                s.set_diffusion(Dfield)
                s.set_wall(np.full(shp, 0.375, np.float32))
            s.set_C(C0)
            s.set_source(S)
            s.step(23)
            out.append(s.get_f(device=False))
    scale = np.abs(out[0]).max()
    assert np.abs(out[0].astype(np.float64) - out[1]).max() <= 1e-6 * scale


@pytest.mark.parametrize("dim,n,precision", [(2, [66, 45], "fp32"), (3, [21, 17, 19], "fp32"), (2, [66, 45], "bf16x3")])
def test_run_with_fields_matches_oracle(dim, n, precision):
    """40 steps with fixed fields; the step graph (10-step replays) is used."""
    _banner(f"run var dim={dim} n={n} {precision}")
    cfg = synth.small(dim, n, seed=67, with_source=True, c_wall=0.1)
    C0 = synth.initial_C(cfg).astype(np.float32)
    S = synth.source(cfg).astype(np.float32)
    D = synth.random_tensor_field(cfg, seed=68)
    Cw = synth.random_wall_values(cfg, seed=69)
    f = oracle.init(cfg, C0.astype(np.float64), Cw=Cw)
    ref = oracle.moment(cfg, oracle.step(cfg, f, 40, S=S.astype(np.float64), D=D, Cw=Cw))
    with _solver(cfg, precision) as s:
        s.set_diffusion(torch.from_numpy(_f32(D)).cuda())
        s.set_wall(_f32(Cw))
        s.set_C(C0)
        s.set_source(S)
        s.step(40)
        got = s.get_C(device=False)
    err = _rel_l2(got, ref)
    _banner(f"rel L2 {err:.2e}")
    assert err <= (1e-5 if precision == "fp32" else 1e-4)


def _gpu_power_law_run(P, steps, dt, precision="fp32", report=()):
    """GPU run of the power-law problem with source and walls updated before
    every step (S(t_m), C(t_{m+1})): the FP32 fields of P.schedule32, which
    the oracle runs below receive too."""
    base = P.base.astype(np.float32)
    out = {}
    with _solver(P.cfg, precision) as s:
        s.set_diffusion(_f32(P.D))
        s.set_wall(base)
        s.set_C(base)
        for m in range(steps):
            S, Cw = P.schedule32(m)
            s.set_source(S)
            s.set_wall(Cw)
            s.step(1)
            if m + 1 in report:
                out[m + 1] = s.get_C(device=False).astype(np.float64)
        out[steps] = s.get_C(device=False).astype(np.float64)
    return out


def _oracle_power_law_run(P, steps, dt):
    """The oracle on the same FP32 inputs as the GPU run above."""
    base = P.base.astype(np.float32).astype(np.float64)
    f = oracle.init(P.cfg, base, Cw=base)
    for m in range(steps):
        S, Cw = P.schedule32(m)
        f = oracle.step(P.cfg, f, 1, S=S.astype(np.float64), D=_f32(P.D).astype(np.float64),
                        Cw=Cw.astype(np.float64))
    return oracle.moment(P.cfg, f)


@pytest.mark.parametrize("dim,n,T,k,a,eps", [
    (2, 41, 0.5, 0.5, [2.0, 2.0], 0.0),
    (2, 41, 0.5, 0.5, [2.0, 2.0], 0.1),
    (2, 41, 0.5, 0.5, [0.4, 0.7], 0.0),
    (3, 21, 0.2, 0.4, [2.0, 2.0, 2.0], 0.0),
])
def test_time_dependent_power_law_matches_oracle_and_exact(dim, n, T, k, a, eps):
    """Time-dependent source and walls updated every step: GPU vs oracle on the
    same schedule, and both vs the exact solution."""
    dx = 1.0 / (n - 1)
    dt = k * dx * dx
    steps = int(round(T / dt))
    P = synth.PowerLawProblem(dim, n, dt, a=a, eps=eps)
    _banner(f"power law dim={dim} n={n} steps={steps} a={a} eps={eps}")
    got = _gpu_power_law_run(P, steps, dt)[steps]
    ref = _oracle_power_law_run(P, steps, dt)
    ex = P.exact(steps * dt)
    err = _rel_l2(got, ref)
    e_gpu = np.abs(got - ex).max()
    e_ora = np.abs(ref - ex).max()
    _banner(f"gpu vs oracle rel L2 {err:.2e}; max error vs exact gpu {e_gpu:.3e} oracle {e_ora:.3e}")
    assert err <= 1e-5
    assert e_gpu <= e_ora * 1.01 + 1e-5


def test_paper_exact_solution_setting():
    """The paper's validation (Sec. 3.4): 2D, alpha = (1.5, 1.7), a = (0.4, 0.7),
    dx = 0.01, dt = 5e-5, MRT, profiles at t = 0.05, 0.5 and 1 (20000 steps),
    against the stored oracle run of the same schedule
    (tests/golden/make_powerlaw_reference.py) and the exact solution: the GPU
    error to the exact solution must be the oracle's (discretisation) error.
    Both sides receive the same FP32 initial, wall, source and D(x) fields
    (PowerLawProblem.schedule32), so the comparison measures the step's own
    FP32 arithmetic: GPU-oracle parity is held to relative L2 1e-5 at every
    mark."""
    import os

    from conftest import GOLDEN

    dt = 5e-5
    ref = np.load(os.path.join(GOLDEN, "ref_powerlaw_2d_101sq_dt5e-5.npz"))
    P = synth.PowerLawProblem(2, 101, dt)
    _banner("paper exact-solution setting, 20000 steps")
    out = _gpu_power_law_run(P, 20000, dt, report=(1000, 10000))
    parity = {1000: 1e-5, 10000: 1e-5, 20000: 1e-5}
    for m in (1000, 10000, 20000):
        C, R, ex = out[m], ref[f"C{m}"], P.exact(m * dt)
        par = _rel_l2(C, R)
        e_gpu, e_ora = np.abs(C - ex).max(), np.abs(R - ex).max()
        _banner(f"t = {m * dt:.2f}: gpu vs oracle rel L2 {par:.2e}; max |C - exact| gpu {e_gpu:.3e} "
                f"oracle {e_ora:.3e}; rel L2 to exact {_rel_l2(C, ex):.2e}")
        assert par <= parity[m]
        assert e_gpu <= 1.01 * e_ora + 1e-5


def test_field_errors_and_resets():
    from paper_1706_09161_amd import LbmError, _lib

    cfg = synth.small(2, [20, 17], seed=71)
    shp = synth.shape(cfg)
    D = synth.random_tensor_field(cfg, seed=72)
    C0 = synth.initial_C(cfg).astype(np.float32)
    with _solver(cfg) as s:
        s.set_C(C0)
        s.step(3)
        a = s.get_f(device=False)
        bad = _f32(D)
        bad[0, 0, 4, 5] = -1e-3
        with pytest.raises(LbmError) as ei:
            s.set_diffusion(bad)
        assert ei.value.code == _lib.LBM_EINVAL
        bad = _f32(D)
        bad[0, 1, 4, 5] += 1e-2
        with pytest.raises(LbmError) as ei:
            s.set_diffusion(bad)
        assert ei.value.code == _lib.LBM_EINVAL
        with pytest.raises(ValueError):
            s.set_diffusion(np.zeros((2, 2, 3), np.float32))
        # the rejected calls left the constant path in place: same state as a fresh run
        s.set_C(C0)
        s.step(3)
        assert np.array_equal(s.get_f(device=False), a)
        # fields set, then reset: back to the constant path
        s.set_diffusion(_f32(D))
        s.set_wall(np.full(shp, 0.5, np.float32))
        with pytest.raises(LbmError) as ei:
            s.adjoint(2, 1, np.ones(shp, np.float32))
        assert ei.value.code == _lib.LBM_EINVAL
        s.set_diffusion(None)
        s.set_wall(None)
        s.set_C(C0)
        s.step(3)
        assert np.array_equal(s.get_f(device=False), a)
    bgk = synth.small(2, [20, 17], seed=71, collision="BGK")
    with _solver(bgk) as s:
        with pytest.raises(LbmError) as ei:
            s.set_diffusion(_f32(D))
        assert ei.value.code == _lib.LBM_EINVAL
        s.set_wall(np.full(shp, 0.5, np.float32))  # wall values are fine with BGK


def test_step_graph_follows_field_reallocation(monkeypatch):
    """Replayed step graphs (10-step runs) while the space-dependent fields are
    set, released and allocated again between runs: the populations equal
    those of the same sequence without graphs, bit for bit (a graph captured
    with freed field pointers would read stale memory)."""
    cfg = synth.small(2, [70, 45], seed=74, with_source=True)
    shp = synth.shape(cfg)
    C0 = synth.initial_C(cfg).astype(np.float32)
    S = synth.source(cfg).astype(np.float32)
    D = _f32(synth.random_tensor_field(cfg, seed=75))
    W1 = _f32(synth.random_wall_values(cfg, seed=76))
    W2 = _f32(synth.random_wall_values(cfg, seed=77))
    res = []
    for graphs in ("1", "0"):
        monkeypatch.setenv("LBM_STEP_GRAPH", graphs)
        with _solver(cfg) as s:
            s.set_C(C0)
            s.set_source(S)
            s.set_wall(W1)
            s.step(10)
            s.set_wall(None)       # both fields released
            s.step(10)
            s.set_diffusion(D)     # allocated again
            s.step(10)
            s.set_diffusion(None)
            s.set_wall(W2)         # and again, with only the wall values in use
            s.step(20)
            s.set_wall(None)
            s.step(10)
            res.append(s.get_f(device=False).copy())
    assert res[0].shape == (5,) + shp
    assert np.array_equal(res[0].view(np.uint32), res[1].view(np.uint32))
