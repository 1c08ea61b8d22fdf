"""Pins of the oracle's space-dependent coefficients against exact solutions.

The paper validates the scheme with a diffusion tensor that depends on x, a
time-dependent source and time-dependent non-homogeneous Dirichlet walls,
against the closed-form solution C = e^-t prod x_mu^a_mu (Sec. 3.4, equations
(Def_D_AS) and (exsolFADE_3D)).  Here the oracle's per-node relaxation blocks
and per-node wall values are checked against that solution and against a
variant with an off-diagonal D(x) whose source is derived in closed form (the
fields come from ``synth.PowerLawProblem``):

* with smooth exponents (a = 2) the error must fall by about 4 when dx halves
  at fixed dt / dx^2 (second order, the diffusive scaling of LB schemes), and
  be small in absolute terms; a dropped term, a wrong sign or a transposed
  index in the per-node block, the source or the wall values would leave an
  O(1) error that does not shrink;
* with the paper's exponents a = (0.4, 0.7) the error shrinks more slowly
  (x^0.4 is not differentiable at the wall) but still shrinks, and at the
  paper's own dx = 0.01, dt = 5e-5 stays within a few 1e-3 of the solution.

The Caputo-type flux of Sec. 3.5 (equations (Fg2), (CoeffA_FADE3DPS)) is
pinned the same way against its exact solution C = e^-t prod (x^beta + a)
(equation (SourceTerm_PS) for beta = alpha; ``synth.CaputoPowerLawProblem``),
against the closed form of its fractional term, and by its uniform equilibria.

Convention of every run: the source of step m is S(t_m) and the Dirichlet
value written by that step is C(t_{m+1}), the time the streamed populations
stand for.
"""
import math

import numpy as np
import pytest

import synth


def _march(oracle_lib, P, steps, dt):
    cfg = P.cfg
    f = oracle_lib.init(cfg, P.base, Cw=P.exact(0.0))
    for m in range(steps):
        f = oracle_lib.step(cfg, f, 1, S=P.source(m * dt), D=P.D, Cw=P.exact((m + 1) * dt))
    return oracle_lib.moment(cfg, f)


def _errors(oracle_lib, dim, n, T, k, **kw):
    """Max and relative-L2 error at time T on an n^dim grid with dt = k dx^2."""
    dx = 1.0 / (n - 1)
    dt = k * dx * dx
    steps = int(round(T / dt))
    P = synth.PowerLawProblem(dim, n, dt, **kw)
    C = _march(oracle_lib, P, steps, dt)
    ex = P.exact(steps * dt)
    err = C - ex
    return float(np.abs(err).max()), float(np.sqrt((err ** 2).mean() / (ex ** 2).mean()))


def test_constant_fields_reproduce_the_constant_path(oracle_lib):
    """A D field equal to the constant tensor everywhere and a wall field equal
    to c_wall give bit-identical populations to the constant-coefficient path."""
    for dim, n in ((2, (13, 9)), (3, (7, 6, 5))):
        cfg = synth.small(dim, n, seed=5, with_source=True, c_wall=0.25)
        shp = synth.shape(cfg)
        C0 = synth.initial_C(cfg)
        S = synth.source(cfg)
        D = np.asarray(cfg["D"], dtype=np.float64)
        Dfield = np.broadcast_to(D.reshape((dim, dim) + (1,) * dim), (dim, dim) + shp).copy()
        Cw = np.full(shp, 0.25)
        f0 = oracle_lib.init(cfg, C0)
        f0v = oracle_lib.init(cfg, C0, Cw=Cw)
        assert np.array_equal(f0, f0v)
        a = oracle_lib.step(cfg, f0, 4, S=S)
        b = oracle_lib.step(cfg, f0, 4, S=S, D=Dfield, Cw=Cw)
        assert np.array_equal(a, b)


def test_per_node_wall_values_are_held():
    """After a step every wall node carries its own Dirichlet value (Sec. 2.5)."""
    import oracle

    cfg = synth.small(2, (12, 10), seed=8)
    shp = synth.shape(cfg)
    rng = np.random.default_rng(3)
    Cw = rng.uniform(-1.0, 1.0, shp)
    f = oracle.init(cfg, synth.initial_C(cfg), Cw=Cw)
    C = oracle.moment(cfg, f)
    wall = np.zeros(shp, dtype=bool)
    wall[0, :] = wall[-1, :] = wall[:, 0] = wall[:, -1] = True
    assert np.allclose(C[wall], Cw[wall], rtol=0, atol=1e-14)
    f = oracle.step(cfg, f, 3, Cw=Cw)
    C = oracle.moment(cfg, f)
    assert np.allclose(C[wall], Cw[wall], rtol=0, atol=1e-14)


def test_powerlaw_exact_solution_second_order_2d(oracle_lib):
    e = [_errors(oracle_lib, 2, n, 0.5, 0.5, a=[2.0, 2.0])[0] for n in (11, 21, 41)]
    assert e[0] / e[1] > 3.6 and e[1] / e[2] > 3.6, e
    assert e[2] < 2.5e-4, e


@pytest.mark.parametrize("eps", [0.1, -0.1])
def test_offdiagonal_tensor_exact_solution_second_order(oracle_lib, eps):
    """D(x) with D_01 = eps x_0 x_1: the cross fluxes D_01 F_1 and D_10 F_0."""
    e = [_errors(oracle_lib, 2, n, 0.5, 0.5, a=[2.0, 2.0], eps=eps)[0] for n in (11, 21, 41)]
    assert e[0] / e[1] > 3.6 and e[1] / e[2] > 3.6, e
    assert e[2] < 4e-4, e


def test_powerlaw_exact_solution_second_order_3d(oracle_lib):
    e = [_errors(oracle_lib, 3, n, 0.2, 0.4, a=[2.0, 2.0, 2.0])[0] for n in (11, 21)]
    assert e[0] / e[1] > 3.5, e
    assert e[1] < 4e-4, e


def test_paper_exponents_converge(oracle_lib):
    """a = (0.4, 0.7), alpha = (1.5, 1.7), as in the paper's figure."""
    r = [_errors(oracle_lib, 2, n, 0.5, 0.5)[1] for n in (11, 21, 41)]
    assert r[0] > r[1] > r[2], r
    assert r[2] < 0.01, r


def test_paper_setting_short_time(oracle_lib):
    """The paper's dx = 0.01, dt = 5e-5 up to its first profile time t = 0.05."""
    mx, rel = _errors(oracle_lib, 2, 101, 0.05, 0.5)
    assert mx < 5e-3 and rel < 1.5e-3, (mx, rel)


def test_invalid_fields_rejected(oracle_lib):
    P = synth.PowerLawProblem(2, 11, 5e-3)
    f = oracle_lib.init(P.cfg, P.base, Cw=P.base)
    bad = P.D.copy()
    bad[0, 0, 3, 4] = -1e-3          # not positive semi-definite
    with pytest.raises(ValueError):
        oracle_lib.step(P.cfg, f, 1, D=bad)
    bad = P.D.copy()
    bad[0, 1, 3, 4] = 1e-3           # not symmetric
    with pytest.raises(ValueError):
        oracle_lib.step(P.cfg, f, 1, D=bad)
    bgk = dict(P.cfg, collision="BGK")
    with pytest.raises(ValueError):
        oracle_lib.step(bgk, f, 1, D=P.D)


# --------------------------------------------------------------------------
# Caputo-type flux variant (Sec. 3.5, equations (Fg2), (CoeffA_FADE3DPS))

@pytest.mark.parametrize("dim", [2, 3])
def test_variant_uniform_field_is_an_equilibrium(oracle_lib, dim):
    """The variant admits uniform equilibria (its flux is a fractional integral
    of the derivative): the fractional term of a constant field vanishes, and
    a constant initial field with the same wall value stays constant (u = 0);
    the form (Fg) does not."""
    n = [13, 11, 9][:dim]
    cfg = synth.small(dim, n, seed=9, u=[0.0] * dim, c_wall=0.7)
    cst = np.full(synth.shape(cfg), 0.7)
    var = dict(cfg, flux_form="caputo")
    assert np.abs(oracle_lib.phi(var, cst)).max() < 1e-13
    assert np.abs(oracle_lib.phi(cfg, cst)).max() > 1e-2
    C = oracle_lib.run(var, cst, 20)
    assert np.abs(C - 0.7).max() < 1e-13
    C = oracle_lib.run(cfg, cst, 20)
    assert np.abs(C - 0.7).max() > 1e-3


def test_variant_fractional_term_closed_form(oracle_lib):
    """On C = (x^beta + a) (y^beta' + a') the variant's term along x is
    Gamma(beta + 1) / Gamma(beta + 3 - alpha) x^(beta + 2 - alpha) (y^beta' + a'):
    second-order convergence of the quadrature for a smooth beta."""
    errs = []
    for n in (21, 41, 81):
        P = synth.CaputoPowerLawProblem(2, n, 1e-4, beta=[3.7, 3.2])
        x = np.arange(n) / (n - 1)
        al, b, a = P.alpha, P.beta, P.a
        g0 = 2 - al[0]
        expect = (math.gamma(b[0] + 1) / math.gamma(b[0] + 1 + g0) * x ** (b[0] + g0))[None, :] * \
            (x ** b[1] + a[1])[:, None]
        errs.append(np.abs(oracle_lib.phi(P.cfg, P.base)[0] - expect).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def _caputo_errors(oracle_lib, n, T, k, **kw):
    dx = 1.0 / (n - 1)
    dt = k * dx * dx
    steps = int(round(T / dt))
    P = synth.CaputoPowerLawProblem(2, n, dt, **kw)
    C = _march_caputo(oracle_lib, P, steps, dt)
    ex = P.exact(steps * dt)
    err = C - ex
    return float(np.abs(err).max()), float(np.sqrt((err ** 2).mean() / (ex ** 2).mean()))


def _march_caputo(oracle_lib, P, steps, dt):
    f = oracle_lib.init(P.cfg, P.base, Cw=P.exact(0.0))
    for m in range(steps):
        f = oracle_lib.step(P.cfg, f, 1, S=P.source(m * dt), Cw=P.exact((m + 1) * dt))
    return oracle_lib.moment(P.cfg, f)


def test_variant_exact_solution_second_order(oracle_lib):
    """C = e^-t prod (x^beta + a) with smooth beta = alpha + 2 (D = Id, p = 1)."""
    e = [_caputo_errors(oracle_lib, n, 0.2, 0.0625, beta=[3.7, 3.2])[0] for n in (11, 21, 41)]
    assert e[0] / e[1] > 3.6 and e[1] / e[2] > 3.6, e
    assert e[2] < 4e-4, e


def test_variant_paper_exact_solution(oracle_lib):
    """The paper's check of the variant: beta = alpha = (1.7, 1.2), a = (0.3, 1.2),
    equation (SourceTerm_PS); the error decreases under refinement, and at the
    paper's dx = 0.02, dt = 2.5e-5 the first profile time t = 0.025 is met within
    a few 1e-4."""
    r = [_caputo_errors(oracle_lib, n, 0.2, 0.0625)[1] for n in (11, 21, 41)]
    assert r[0] > r[1] > r[2] and r[2] < 2e-4, r
    mx, rel = _caputo_errors(oracle_lib, 51, 0.025, 0.0625)
    assert mx < 1e-3 and rel < 3e-4, (mx, rel)
