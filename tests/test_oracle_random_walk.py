"""Pins of the oracle's Levy-stable random walk (random_walk.c; the paper's
statistical check, Sec. 3.1 equations (RW_STABLE), (distri), killed at the
first exit; Weron's sampler; Philox-4x32-10 counters).

* the generator's uniforms are uniform and uncorrelated across counters;
* the stable draws have the characteristic function the paper prints,
  equations (stb), (stbb) (which fixes the sign convention of beta), and the
  skewness the paper describes (most probable value of sign -beta, heavier
  tail on the side of beta);
* alpha = 2 gives Brownian motion: mean and variance of the free walk in
  closed form, and the survival probability of the walk killed at the walls
  of a slab against the Fourier series of the Dirichlet heat equation
  (with the boundary shift 0.5826 sigma sqrt(dt) of discrete monitoring);
* stability of the law: n steps of dt equal one step of n dt in distribution
  (two-sample Kolmogorov-Smirnov);
* the walk killed in a square against the LB oracle (a method independent of
  it) for alpha = (1.5, 1.99): surviving mass and marginal profiles, as in the
  paper's comparisons of Sec. 3.2.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth


def test_uniforms_are_uniform_and_uncorrelated(oracle_lib):
    u = np.array([oracle_lib.rw_uniforms(5, k, 3, 1) for k in range(100000)])
    assert np.all((u > 0) & (u < 1))
    for col in (u[:, 0], u[:, 1]):
        counts, _ = np.histogram(col, bins=100, range=(0, 1))
        chi2 = float(((counts - 1000.0) ** 2 / 1000.0).sum())
        assert stats.chi2.sf(chi2, 99) > 1e-3
    lim = 5 / math.sqrt(len(u))
    assert abs(np.corrcoef(u[:, 0], u[:, 1])[0, 1]) < lim        # within one draw
    assert abs(np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]) < lim     # neighbouring particles
    v = np.array([oracle_lib.rw_uniforms(5, k, 4, 1) for k in range(20000)])
    assert abs(np.corrcoef(u[:20000, 0], v[:, 0])[0, 1]) < 5 / math.sqrt(20000)  # next step


@pytest.mark.parametrize("alpha,beta", [(1.5, 0.0), (1.5, 1.0), (1.2, -0.6), (1.8, 0.4), (2.0, 0.7)])
def test_stable_draws_have_the_printed_characteristic_function(oracle_lib, alpha, beta):
    N = 200000
    s = oracle_lib.stable_draws(alpha, beta, 13, N)
    for k in (-2.0, -0.7, 0.3, 1.0, 2.5):
        emp = np.mean(np.exp(1j * k * s))
        th = np.exp(-abs(k) ** alpha * (1 - 1j * beta * np.sign(k) * math.tan(math.pi * alpha / 2)))
        assert abs(emp - th) < 5 / math.sqrt(N), (k, emp, th)


def test_skewness_direction(oracle_lib):
    s = oracle_lib.stable_draws(1.5, 1.0, 17, 200000)
    assert np.median(s) < -0.1                       # most probable value has the sign of -beta
    assert np.mean(s > 4) > 10 * np.mean(s < -4)     # heavy tail on the side of beta
    assert abs(np.mean(s)) < 0.1                     # zero mean (alpha > 1)
    m = oracle_lib.stable_draws(1.5, -1.0, 19, 200000)
    assert stats.ks_2samp(-m, s).pvalue > 1e-3       # S(alpha, -beta) is the mirror image of S(alpha, beta)
    for V, W in ((0.3, 0.7), (-1.2, 2.5), (1.5, 0.01)):
        assert oracle_lib.stable_from(1.5, -0.4, V, W) == pytest.approx(-oracle_lib.stable_from(1.5, 0.4, -V, W),
                                                                        rel=1e-12)


def test_brownian_walk_moments(oracle_lib):
    """alpha = 2, no walls in reach: mean x_s + u t, variance sigma0^2 + 2 D g t."""
    D, g, u, t, dt, s0 = (0.3, 0.05), (1.0, 2.0), (0.4, -0.2), 0.5, 0.01, 0.05
    P = oracle_lib.rw_params(2, [-1e9, -1e9], [1e9, 1e9], [2.0, 2.0], [0.2, 0.9], D, g=g, u=u, dt=dt, seed=9)
    N = 100000
    x, al = oracle_lib.rw_init_gaussian(P, (0.1, 0.2), s0, N)
    x, al = oracle_lib.rw_walk(P, x, al, int(round(t / dt)))
    assert al.all()
    for mu in range(2):
        var = s0 ** 2 + 2 * D[mu] * g[mu] * t
        assert abs(x[mu].mean() - ((0.1, 0.2)[mu] + u[mu] * t)) < 5 * math.sqrt(var / N)
        assert abs(x[mu].var() / var - 1) < 5 * math.sqrt(2 / N)


def test_stable_law_is_stable_under_steps(oracle_lib):
    """n steps of dt and one step of n dt give the same law (equation (distri))."""
    a, p, D, n, dt = 1.6, 0.8, 0.7, 40, 1e-3
    P1 = oracle_lib.rw_params(1, [-1e12], [1e12], [a], [p], [D], dt=dt, seed=21)
    Pn = oracle_lib.rw_params(1, [-1e12], [1e12], [a], [p], [D], dt=n * dt, seed=22)
    N = 40000
    x1, al1 = oracle_lib.rw_init_gaussian(P1, (0.0,), 0.0, N)
    x1, al1 = oracle_lib.rw_walk(P1, x1, al1, n)
    xn, aln = oracle_lib.rw_init_gaussian(Pn, (0.0,), 0.0, N)
    xn, aln = oracle_lib.rw_walk(Pn, xn, aln, 1)
    assert stats.ks_2samp(x1[0], xn[0]).pvalue > 1e-3


def test_killed_brownian_survival(oracle_lib):
    """Walk killed at the walls of ]0, 1[ (no walls in reach along y): the
    surviving fraction against sum over odd m of 4/(m pi) sin(m pi x0 / L)
    exp(-D m^2 pi^2 t / L^2), with the walls moved out by 0.5826 sigma sqrt(dt)
    for the exits missed between steps (sigma^2 = 2 D)."""
    D, x0, t, dt = 0.1, 0.3, 0.3, 2e-4
    P = oracle_lib.rw_params(2, [0.0, -1e9], [1.0, 1e9], [2.0, 2.0], [0.5, 0.5], (D, D), dt=dt, seed=31)
    N = 20000
    x, al = oracle_lib.rw_init_gaussian(P, (x0, 0.0), 0.0, N)
    x, al = oracle_lib.rw_walk(P, x, al, int(round(t / dt)))
    shift = 0.5826 * math.sqrt(2 * D * dt)
    L, xe = 1.0 + 2 * shift, x0 + shift
    surv = sum(4 / (m * math.pi) * math.sin(m * math.pi * xe / L) * math.exp(-D * (m * math.pi / L) ** 2 * t)
               for m in range(1, 400, 2))
    sd = math.sqrt(surv * (1 - surv) / N)
    assert abs(al.mean() - surv) < 4 * sd + 2e-3, (al.mean(), surv)


def test_killed_stable_walk_against_lb(oracle_lib):
    """Omega = [0, 2]^2, D = 0.5 Id, alpha = (1.5, 1.99), p = 1/2, g = 1, u = 0,
    Gaussian of sigma0 = 0.1 at (1, 1), t = 0.05: LB (dx = 0.04, dt = 2e-4)
    against the walk (dt = 2.5e-4, 2e5 particles): surviving mass and the two
    marginal profiles."""
    n, dt, T, s0 = 51, 2e-4, 0.05, 0.1
    dx = 2.0 / (n - 1)
    cfg = dict(dim=2, n=[n, n], dx=dx, dt=dt, alpha=[1.5, 1.99], p=[0.5, 0.5], g=[1.0, 1.0],
               D=[[0.5, 0.0], [0.0, 0.5]], u=[0.0, 0.0], collision="MRT", tau_free=[1.0] * 4, tau0=1.0, c_wall=0.0)
    C0 = synth.paper_gaussian(cfg, (1.0, 1.0), sigma0=s0, C0=1.0)
    C = oracle_lib.run(cfg, C0, int(round(T / dt)))
    P = oracle_lib.rw_params(2, [0, 0], [2, 2], [1.5, 1.99], [0.5, 0.5], (0.5, 0.5), dt=2.5e-4, seed=3)
    N = 200000
    x, al = oracle_lib.rw_init_gaussian(P, (1.0, 1.0), s0, N)
    x, al = oracle_lib.rw_walk(P, x, al, int(round(T / 2.5e-4)))
    dens = oracle_lib.rw_histogram(P, x, al, [n, n], dx) / N / dx ** 2
    mass_lb = C.sum() * dx ** 2 / (C0.sum() * dx ** 2)
    assert abs(al.mean() - mass_lb) < 4 * math.sqrt(al.mean() * (1 - al.mean()) / N) + 1e-3
    for ax in (0, 1):
        m_lb, m_rw = C.sum(axis=ax) * dx, dens.sum(axis=ax) * dx
        assert np.linalg.norm(m_lb - m_rw) / np.linalg.norm(m_lb) < 0.02


def test_histogram_counts_every_living_particle_once(oracle_lib):
    P = oracle_lib.rw_params(2, [0, 0], [2, 1], [1.7, 1.7], [0.5, 0.5], (0.01, 0.01), dt=1e-3, seed=41)
    x, al = oracle_lib.rw_init_gaussian(P, (1.0, 0.5), 0.4, 50000)
    h = oracle_lib.rw_histogram(P, x, al, [201, 101], 0.01)
    assert h.sum() == al.sum() and h.shape == (101, 201)
    j = np.floor(x[0][al == 1] / 0.01 + 0.5).astype(int)
    assert np.array_equal(np.bincount(j, minlength=201), h.sum(axis=0))


def test_exits_mostly_through_the_super_diffusive_walls(oracle_lib):
    """The paper's validation 1 (Sec. 3.2): with alpha = (1.5, 1.99) most
    sample paths that leave [0, 2]^2 do so through the walls normal to x1."""
    P = oracle_lib.rw_params(2, [0, 0], [2, 2], [1.5, 1.99], [0.5, 0.5], (0.5, 0.5), dt=1e-3, seed=2024)
    x, al = oracle_lib.rw_init_gaussian(P, (1.0, 1.0), 0.05, 100000)
    x, al = oracle_lib.rw_walk(P, x, al, 100)
    dead = al == 0
    out1 = dead & ((x[0] <= 0.0) | (x[0] >= 2.0))
    out2 = dead & ~out1 & ((x[1] <= 0.0) | (x[1] >= 2.0))
    assert dead.sum() > 1000 and out1.sum() + out2.sum() == dead.sum()
    assert out1.sum() > 0.7 * dead.sum()
