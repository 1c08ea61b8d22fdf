"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself: values
printed in the paper (golden fixtures), closed forms, independent numerical
quadrature, exact invariants and special cases.  Sized to run in seconds on
the CPU.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import synth
from conftest import read_golden

GAMMAS = [0.0, 0.1, 0.3, 0.5, 0.8, 0.99]


# --------------------------------------------------------------------------
# Lattice tables (Sec. 2.1)

def test_lattice_matches_printed_weights(oracle_lib):
    for dim, Q, w0, wi, e2 in read_golden("lattice_weights.txt"):
        e, w, e2_o = oracle_lib.lattice(int(dim))
        assert e.shape == (int(Q), int(dim))
        assert w[0] == pytest.approx(float(w0), rel=1e-15)
        assert np.allclose(w[1:], float(wi), rtol=1e-15)
        assert e2_o == pytest.approx(float(e2), rel=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_weight_moment_conditions(oracle_lib, dim):
    """Equation (weights_c): <1|w> = 1, <e_mu|w> = 0, <e_mu e_nu|w> = e^2 delta."""
    e, w, e2 = oracle_lib.lattice(dim)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(e.T @ w, 0.0, atol=1e-15)
    second = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(second, e2 * np.eye(dim), atol=1e-15)
    # e_{2mu-1} = +b_mu, e_{2mu} = -b_mu, e_0 = 0
    assert np.all(e[0] == 0)
    for mu in range(dim):
        assert np.all(e[2 * mu + 1] == np.eye(dim, dtype=int)[mu])
        assert np.all(e[2 * mu + 2] == -np.eye(dim, dtype=int)[mu])


# --------------------------------------------------------------------------
# Fractional-integral coefficients (Sec. 2.4, equations (c+), (c-))

def _hat_quadrature(l, n, gamma):
    """Gamma(2+gamma)/Gamma(gamma) * int_0^n hat_l(s) (n-s)^(gamma-1) ds.

    The trapezoidal product rule integrates the piecewise-linear interpolant
    of f exactly against the kernel (x_n - s)^(gamma-1)/Gamma(gamma); in unit
    spacing the weight of node l is this integral of its hat function.
    Computed by adaptive quadrature with the algebraic end-point weight."""
    total = 0.0
    pieces = []
    if l >= 1:
        pieces.append((l - 1, l, lambda s: s - (l - 1)))
    if l + 1 <= n:
        pieces.append((l, l + 1, lambda s: (l + 1) - s))
    for a, b, hat in pieces:
        if b == n:
            val, _ = integrate.quad(hat, a, b, weight="alg", wvar=(0.0, gamma - 1.0), epsabs=1e-14, epsrel=1e-12)
        else:
            val, _ = integrate.quad(lambda s: hat(s) * (n - s) ** (gamma - 1.0), a, b, epsabs=1e-14, epsrel=1e-12)
        total += val
    return special.gamma(2 + gamma) / special.gamma(gamma) * total


@pytest.mark.parametrize("gamma", [0.1, 0.3, 0.5, 0.8, 0.99])
def test_cplus_equals_hat_function_quadrature(oracle_lib, gamma):
    for n in [1, 2, 3, 5, 8, 13]:
        for l in range(0, n + 1):
            ref = _hat_quadrature(l, n, gamma)
            got = oracle_lib.cplus(l, n, gamma)
            assert got == pytest.approx(ref, rel=1e-8, abs=1e-10), (l, n, gamma)


@pytest.mark.parametrize("gamma", GAMMAS)
def test_cplus_sum_and_first_moment_rules(oracle_lib, gamma):
    """Exactness on constants and on linear functions (power law of
    equation (derfracpuissce) with a = 0 and a = 1): sum_l c+_{ln} = (1+gamma) n^gamma
    and sum_l l c+_{ln} = n^(gamma+1), n >= 0 (at n = 0 the integral is over an
    empty interval: c+_{00} = 0^gamma, 1 only for gamma = 0)."""
    for n in range(0, 61):
        c = np.array([oracle_lib.cplus(l, n, gamma) for l in range(n + 1)])
        assert c.sum() == pytest.approx((1 + gamma) * float(n) ** gamma, rel=1e-12, abs=1e-300)
        assert (np.arange(n + 1) * c).sum() == pytest.approx(float(n) ** (gamma + 1), rel=1e-12)
    assert oracle_lib.cplus(0, 0, gamma) == (1.0 if gamma == 0.0 else 0.0)


@pytest.mark.parametrize("gamma", GAMMAS)
def test_cminus_is_mirror_of_cplus(oracle_lib, gamma):
    """c-_{ln}(gamma, N) = c+_{N-l, N-n}(gamma): the right integral is the left
    one seen from the other wall."""
    N = 17
    for n in range(N + 1):
        for l in range(N + 1):
            assert oracle_lib.cminus(l, n, N, gamma) == pytest.approx(oracle_lib.cplus(N - l, N - n, gamma),
                                                                      rel=1e-14, abs=1e-15)


def test_gamma_zero_is_identity(oracle_lib):
    """I^0 = Id (Sec. 1): gamma = 0 gives c_{ln} = delta_{ln}."""
    for n in range(0, 12):
        for l in range(0, 12):
            assert oracle_lib.cplus(l, n, 0.0) == pytest.approx(1.0 if l == n else 0.0, abs=1e-15)
            assert oracle_lib.cminus(l, n, 11, 0.0) == pytest.approx(1.0 if l == n else 0.0, abs=1e-15)


# --------------------------------------------------------------------------
# Discrete fractional integrals on grid lines (Sec. 2.4, (XXminus_discret))

def _line_cfg(dim, n, alpha, p, dx=1.0):
    cfg = synth.small(dim, n, alpha=alpha, p=p, u=[0.0] * dim, D=(0.1 * np.eye(dim)).tolist())
    cfg["dx"] = dx
    return cfg


@pytest.mark.parametrize("a", [0, 1])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_phi_power_law_exact_for_a_0_and_1(oracle_lib, a, axis):
    """Equation (derfracpuissce): I+^gamma x^a = Gamma(a+1)/Gamma(a+1+gamma) x^(a+gamma).
    The trapezoidal product rule is exact for a in {0, 1}.  p = 1 on the tested
    axis; the other coordinates carry an arbitrary factor, so the test also pins
    which nodes form a line in 3D."""
    n = [7, 9, 11]
    dx = 0.25
    alpha = [1.35, 1.6, 1.85]
    p = [0.4, 0.7, 0.2]
    p[axis] = 1.0
    cfg = _line_cfg(3, n, alpha, p, dx=dx)
    X = np.meshgrid(*[np.arange(v) * dx for v in reversed(n)], indexing="ij")[::-1]  # X[mu], shape (nz,ny,nx)
    rng = np.random.default_rng(3)
    other = rng.uniform(0.5, 1.5, size=X[0].shape)
    # make 'other' constant along the tested axis
    other = np.take(other, [0], axis=2 - axis).repeat(n[axis], axis=2 - axis)
    C = other * X[axis] ** a
    Phi = oracle_lib.phi(cfg, C)
    gamma = 2 - alpha[axis]
    exact = other * math.gamma(a + 1) / math.gamma(a + 1 + gamma) * X[axis] ** (a + gamma)
    interior = X[axis] > 0  # x = 0 carries the c+_{00} = 1 reading
    assert np.allclose(Phi[axis][interior], exact[interior], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("gamma", [0.2, 0.5, 0.8])
def test_phi_right_integral_power_law(oracle_lib, gamma):
    """Right integral (p = 0) of (L - x)^a, a in {0, 1}: mirror of the power law."""
    n = [13, 5]
    dx = 0.5
    L = (n[0] - 1) * dx
    cfg = _line_cfg(2, n, [2 - gamma, 1.5], [0.0, 0.5], dx=dx)
    x = np.arange(n[0]) * dx
    for a in (0, 1):
        C = np.tile((L - x) ** a, (n[1], 1))
        Phi = oracle_lib.phi(cfg, C)[0]
        exact = math.gamma(a + 1) / math.gamma(a + 1 + gamma) * (L - x) ** (a + gamma)
        assert np.allclose(Phi[:, :-1], exact[None, :-1], rtol=1e-12, atol=1e-14)


def test_phi_second_order_convergence(oracle_lib):
    """For a smooth non-polynomial function the product rule converges at
    order 2 (Sec. 2.4: errors of the order of dx^2).  f(x) = x^2 on [0, 1]:
    I+^gamma x^2 = 2/Gamma(3+gamma) x^(2+gamma)."""
    gamma = 0.5
    errs = []
    for N in (16, 32, 64, 128):
        dx = 1.0 / N
        cfg = _line_cfg(2, [N + 1, 3], [2 - gamma, 1.5], [1.0, 0.5], dx=dx)
        x = np.arange(N + 1) * dx
        C = np.tile(x**2, (3, 1))
        Phi = oracle_lib.phi(cfg, C)[0][1]
        exact = 2.0 / math.gamma(3 + gamma) * x ** (2 + gamma)
        errs.append(abs(Phi[-1] - exact[-1]))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(1.8 < r < 2.2 for r in rates), rates


def test_phi_alpha_two_is_identity_times_g(oracle_lib):
    cfg = synth.small(2, [9, 6], alpha=[2.0, 2.0], p=[0.3, 0.9])
    cfg["g"] = [1.7, 0.6]
    C = synth.initial_C(cfg)
    Phi = oracle_lib.phi(cfg, C)
    assert np.allclose(Phi[0], 1.7 * C, rtol=1e-15)
    assert np.allclose(Phi[1], 0.6 * C, rtol=1e-15)


def test_phi_p_mirror(oracle_lib):
    """Reversing the axis swaps the left and right integrals: Phi(p)(x) = Phi(1-p)(L-x) on the reversed field."""
    cfg = synth.small(2, [12, 7], alpha=[1.4, 1.7], p=[0.2, 0.6])
    C = synth.initial_C(cfg)
    mir = dict(cfg, p=[0.8, 0.6])
    P1 = oracle_lib.phi(cfg, C)
    P2 = oracle_lib.phi(mir, C[:, ::-1])
    assert np.allclose(P1[0], P2[0][:, ::-1], rtol=1e-13, atol=1e-15)
    assert np.allclose(P1[1], P2[1][:, ::-1], rtol=1e-13, atol=1e-15)


def test_phi_at_matches_full_phi(oracle_lib):
    """The node-by-node evaluation (used for sampled parity at large sizes)
    agrees with the line-by-line one."""
    cfg = synth.small(3, [6, 5, 7], seed=4)
    C = synth.initial_C(cfg)
    full = oracle_lib.phi(cfg, C).reshape(3, -1)
    nodes = np.array([0, 3, 17, 44, 101, 6 * 5 * 7 - 1])
    part = oracle_lib.phi_at(cfg, C, nodes)
    assert np.allclose(part, full[:, nodes], rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# Equilibrium (equations (M0)-(M2), (Feq), (CoeffA))

@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments(oracle_lib, dim):
    cfg = synth.small(dim, [5] * dim, seed=7)
    cfg["dt"], cfg["dx"] = 0.3, 0.7
    e, w, e2 = oracle_lib.lattice(dim)
    rng = np.random.default_rng(11)
    for _ in range(5):
        C = rng.uniform(-1, 2)
        phi = rng.uniform(-3, 3, dim)
        feq = oracle_lib.equilibrium(cfg, C, phi)
        assert feq.sum() == pytest.approx(C, abs=1e-14)
        assert np.allclose(e.T @ feq, C * np.array(cfg["u"]) * cfg["dt"] / cfg["dx"], atol=1e-14)
        second = np.einsum("i,ia,ib->ab", feq, e, e)
        assert np.allclose(second, e2 * np.diag(phi), atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_alpha_two_is_classical(oracle_lib, dim):
    """alpha = 2: the fractional part reduces to C|w> (Sec. 2.2)."""
    cfg = synth.small(dim, [5] * dim, seed=8, alpha=[2.0] * dim)
    e, w, e2 = oracle_lib.lattice(dim)
    C = 0.8
    feq = oracle_lib.equilibrium(cfg, C, np.full(dim, C))
    adv = (C / e2) * (e @ np.array(cfg["u"])) * w
    assert np.allclose(feq, C * w + adv, atol=1e-15)


# --------------------------------------------------------------------------
# Collision (Sec. 2.2, Sec. 2.3)

def test_moment_matrices_match_paper(oracle_lib):
    rows = read_golden("mrt_matrix_M.txt")
    blocks, cur = {}, None
    for r in rows:
        if r[0] in ("D2Q5", "D3Q7"):
            cur = r[0]
            blocks[cur] = []
        else:
            blocks[cur].append([float(v) for v in r])
    for dim, name in ((2, "D2Q5"), (3, "D3Q7")):
        cfg = synth.small(dim, [5] * dim, seed=1)
        M, Minv, Lam, _ = oracle_lib.collision_matrices(cfg)
        Mp = np.array(blocks[name])
        assert np.array_equal(M, Mp)
        # rows mutually orthogonal (Sec. 2.3), so M^-1 = M^T diag(1/|row|^2)
        G = Mp @ Mp.T
        assert np.allclose(G, np.diag(np.diag(G)))
        assert np.allclose(Minv, Mp.T @ np.diag(1.0 / np.diag(G)), atol=1e-14)


def test_bgk_relaxation_time_matches_printed_value(oracle_lib):
    """Sec. 3.3 prints lambda = 0.548 for D = 2e-3, dx = 1e-2, dt = 8e-4 (D2Q5)."""
    (D, dx, dt, lam, tol), = read_golden("bgk_relaxation.txt")
    cfg = synth.small(2, [5, 5], collision="BGK", D=[[float(D), 0], [0, float(D)]])
    cfg["dx"], cfg["dt"] = float(dx), float(dt)
    _, _, _, lam_o = oracle_lib.collision_matrices(cfg)
    assert abs(lam_o - float(lam)) < float(tol)


def test_mrt_flux_block_is_inverse_of_lambda_bar(oracle_lib):
    """Equation (D_ab): lambda-bar = D dt/(e^2 dx^2) + Id/2, and Lambda is the
    inverse of the block matrix (MatrixS), so its flux block is lambda-bar^-1."""
    cfg = synth.small(3, [5, 5, 5], seed=9)
    cfg["dx"], cfg["dt"] = 0.5, 0.2
    cfg["tau_free"] = [0.9, 1.3, 1.7, 1.0]
    cfg["tau0"] = 1.1
    _, _, Lam, _ = oracle_lib.collision_matrices(cfg)
    e2 = 0.25
    lam_bar = np.array(cfg["D"]) * cfg["dt"] / (e2 * cfg["dx"] ** 2) + 0.5 * np.eye(3)
    assert np.allclose(Lam[1:4, 1:4] @ lam_bar, np.eye(3), atol=1e-13)
    assert Lam[0, 0] == pytest.approx(1 / 1.1)
    assert np.allclose(np.diag(Lam)[4:], 1.0 / np.array([0.9, 1.3, 1.7]))
    off = Lam.copy()
    off[1:4, 1:4] = 0
    assert np.allclose(off - np.diag(np.diag(off)), 0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("collision", ["BGK", "MRT"])
def test_collision_conserves_mass(oracle_lib, dim, collision):
    cfg = synth.small(dim, [5] * dim, seed=12, collision=collision)
    rng = np.random.default_rng(5)
    f = rng.uniform(-1, 1, 2 * dim + 1)
    phi = rng.uniform(-2, 2, dim)
    S = 0.37
    fs = oracle_lib.collide_node(cfg, f, f.sum(), phi, S)
    assert fs.sum() == pytest.approx(f.sum() + S * cfg["dt"], abs=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_bgk_equals_mrt_with_equal_rates(oracle_lib, dim):
    """M^-1 (1/lambda) I M = (1/lambda) I: MRT with isotropic D and every free
    time equal to lambda is BGK."""
    D = 0.13
    mrt = synth.small(dim, [5] * dim, seed=13, D=(D * np.eye(dim)).tolist())
    e2 = 1 / 3 if dim == 2 else 1 / 4
    lam = D / e2 + 0.5
    mrt["tau_free"] = [lam] * 4
    mrt["tau0"] = lam
    bgk = dict(mrt, collision="BGK")
    rng = np.random.default_rng(6)
    for _ in range(4):
        f = rng.uniform(-1, 1, 2 * dim + 1)
        phi = rng.uniform(-2, 2, dim)
        a = oracle_lib.collide_node(mrt, f, f.sum(), phi, 0.01)
        b = oracle_lib.collide_node(bgk, f, f.sum(), phi, 0.01)
        assert np.allclose(a, b, atol=1e-14)


def test_tau0_has_no_effect(oracle_lib):
    """Sec. 2.3: lambda_0 acts on the conserved mass and has no effect."""
    cfg = synth.small(2, [5, 5], seed=14)
    rng = np.random.default_rng(7)
    f = rng.uniform(-1, 1, 5)
    phi = rng.uniform(-2, 2, 2)
    a = oracle_lib.collide_node(dict(cfg, tau0=0.7), f, f.sum(), phi)
    b = oracle_lib.collide_node(dict(cfg, tau0=3.0), f, f.sum(), phi)
    assert np.allclose(a, b, atol=1e-15)


# --------------------------------------------------------------------------
# Whole steps: streaming + Dirichlet rule + closed forms

def _rel_err_interior(C, ref, margin):
    sl = tuple(slice(margin, -margin) for _ in C.shape)
    return np.abs(C[sl] - ref[sl]).max() / np.abs(ref[sl]).max()


def _gauss_2d(n, sigma2, center, amp=1.0):
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return amp * np.exp(-0.5 * ((x - center[0]) ** 2 + (y - center[1]) ** 2) / sigma2)


def test_alpha_two_gaussian_closed_form_second_order(oracle_lib):
    """alpha = 2 turns the FADE into the classical ADE (Sec. 1).  A Gaussian of
    variance s0^2 under u = 0 and isotropic D has variance s0^2 + 2Dt and peak
    s0^2/(s0^2 + 2Dt).  Under diffusive refinement (dx/2, dt/4) the error
    drops by about 4 (second order)."""
    errs = []
    D = 0.1
    for k, (n, steps, s0) in enumerate([(33, 40, 2.0), (65, 160, 4.0), (129, 640, 8.0)]):
        cfg = synth.small(2, [n, n], alpha=[2.0, 2.0], p=[0.5, 0.5], u=[0.0, 0.0], D=[[D, 0], [0, D]])
        c = (n - 1) / 2
        C0 = _gauss_2d(n, s0**2, (c, c))
        C = oracle_lib.run(cfg, C0, steps)
        s2 = s0**2 + 2 * D * steps
        ref = _gauss_2d(n, s2, (c, c), amp=s0**2 / s2)
        errs.append(_rel_err_interior(C, ref, n // 4))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3
    assert all(1.7 < r < 2.4 for r in rates), (errs, rates)


@pytest.mark.parametrize("collision", ["MRT", "BGK"])
def test_alpha_two_mass_and_drift(oracle_lib, collision):
    """ADE limit with advection, plume far from the walls: mass is conserved
    and the centre of mass moves at u (equation (FADE_moreGeneral) with alpha = 2)."""
    n, steps = 64, 100
    u = [0.05, -0.03]
    D = [[0.08, 0.0], [0.0, 0.08]]
    cfg = synth.small(2, [n, n], collision=collision, alpha=[2.0, 2.0], p=[0.5, 0.5], u=u, D=D)
    C0 = _gauss_2d(n, 9.0, (28.0, 33.0))
    C = oracle_lib.run(cfg, C0, steps)
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    # the Gaussian tail that reaches the walls (about 5.6 sigma away) loses ~1e-7
    assert C.sum() == pytest.approx(C0.sum(), rel=1e-6)
    cx = (C * x).sum() / C.sum()
    cy = (C * y).sum() / C.sum()
    assert cx == pytest.approx(28.0 + u[0] * steps, abs=1e-4)
    assert cy == pytest.approx(33.0 + u[1] * steps, abs=1e-4)


def _lb_covariance_growth(lam_bar, e2, steps):
    """Exact covariance growth of the LB scheme in the ADE limit (alpha = 2, u = 0,
    free relaxation times 1, start from equilibrium, no wall losses).

    With A_k = sum_y y j(y)^T (position times flux moment, per unit mass) the
    streaming and the flux-block relaxation j* = (I - lambda-bar^-1) j give
        A_{k+1} = A_k R^T + e^2 I,   Sigma_{k+1} = Sigma_k + A_k R^T + R A_k^T + e^2 I,
    with R = I - lambda-bar^-1 and A_0 = 0.  Its limit increment is 2 e^2 (lambda-bar - I/2)
    = 2 D (equation (D_ab)); the start-up transient is what the recurrence adds."""
    d = lam_bar.shape[0]
    R = np.eye(d) - np.linalg.inv(lam_bar)
    A = np.zeros((d, d))
    growth = np.zeros((d, d))
    for _ in range(steps):
        growth += A @ R.T + R @ A.T + e2 * np.eye(d)
        A = A @ R.T + e2 * np.eye(d)
    return growth


def _covariance(C):
    m = C.sum()
    grids = np.meshgrid(*[np.arange(v) for v in C.shape], indexing="ij")[::-1]  # x first
    mean = [(C * g).sum() / m for g in grids]
    d = len(grids)
    return m, np.array([[(C * (grids[a] - mean[a]) * (grids[b] - mean[b])).sum() / m for b in range(d)]
                        for a in range(d)])


def test_alpha_two_anisotropic_covariance(oracle_lib):
    """ADE limit with a full SPD tensor (MRT, equation (D_ab)): the covariance of
    a centred Gaussian follows the exact LB recurrence, whose slope is 2 D,
    off-diagonal part included."""
    n, steps = 96, 150
    D = np.array([[0.0875, -0.0649519052838329], [-0.0649519052838329, 0.1625]])
    cfg = synth.small(2, [n, n], alpha=[2.0, 2.0], p=[0.5, 0.5], u=[0.0, 0.0], D=D.tolist())
    c = (n - 1) / 2
    C0 = _gauss_2d(n, 9.0, (c, c))
    C = oracle_lib.run(cfg, C0, steps)
    _, cov0 = _covariance(C0)
    _, cov = _covariance(C)
    e2 = 1.0 / 3.0
    lam_bar = D / e2 + 0.5 * np.eye(2)
    expect = cov0 + _lb_covariance_growth(lam_bar, e2, steps)
    assert np.allclose(cov, expect, rtol=0, atol=1e-5)  # tails beyond 5.7 sigma reach the walls
    assert np.abs(expect - cov0 - 2 * D * steps).max() < 0.1  # the transient is small


def test_alpha_two_gaussian_3d(oracle_lib):
    """D3Q7, alpha = 2, diagonal anisotropic D: mass is kept and the per-axis
    variance follows the exact LB recurrence (slope 2 D_mumu)."""
    n, steps = 48, 60
    Dd = [0.1, 0.06, 0.03]
    cfg = synth.small(3, [n, n, n], alpha=[2.0] * 3, p=[0.5] * 3, u=[0.0] * 3, D=np.diag(Dd).tolist())
    c = (n - 1) / 2
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    C0 = np.exp(-0.5 * ((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) / 4.0)
    C = oracle_lib.run(cfg, C0, steps)
    m, cov = _covariance(C)
    m0, cov0 = _covariance(C0)
    assert m == pytest.approx(m0, rel=1e-7)  # tails beyond ~6 sigma reach the walls
    e2 = 0.25
    expect = cov0 + _lb_covariance_growth(np.diag(Dd) / e2 + 0.5 * np.eye(3), e2, steps)
    assert np.allclose(cov, expect, rtol=0, atol=1e-5)


def test_walls_hold_dirichlet_value(oracle_lib):
    """Equation (Dirichlet_BC): after every step C = C_wall on every wall node,
    for a non-zero wall value too (3D: faces, edges and corners)."""
    for dim, n in ((2, [9, 7]), (3, [6, 5, 7])):
        cfg = synth.small(dim, n, seed=21, c_wall=0.37)
        C0 = synth.initial_C(cfg)
        f = oracle_lib.init(cfg, C0)
        for _ in range(3):
            f = oracle_lib.step(cfg, f, 1)
            C = oracle_lib.moment(cfg, f)
            wall = np.zeros(C.shape, bool)
            for ax in range(dim):
                idx = [slice(None)] * dim
                idx[ax] = 0
                wall[tuple(idx)] = True
                idx[ax] = -1
                wall[tuple(idx)] = True
            assert np.allclose(C[wall], 0.37, atol=1e-14)


def test_d4_symmetry_of_symmetric_workload(oracle_lib):
    """Equal orders, p = 1/2, isotropic D, u = 0, centred pulse: the solution
    keeps the square's symmetries."""
    cfg = synth.config("c1_64sq")
    C = oracle_lib.run(cfg, synth.initial_C(cfg), 40)
    assert np.allclose(C, C.T, atol=1e-14)
    assert np.allclose(C, C[::-1, :], atol=1e-14)
    assert np.allclose(C, C[:, ::-1], atol=1e-14)


def _symmetries(dim):
    """The box's symmetries as (map of a field, map of a population index):
    axis swaps and reflections of a field stored slowest axis first, with
    populations ordered 0, +x, -x, +y, -y (, +z, -z)."""
    out = []
    Q = 2 * dim + 1
    for a in range(dim):
        for b in range(a + 1, dim):  # swap axes a and b (array dims dim-1-a, dim-1-b)
            perm = list(range(Q))
            for s_ in (0, 1):
                perm[2 * a + 1 + s_], perm[2 * b + 1 + s_] = 2 * b + 1 + s_, 2 * a + 1 + s_
            out.append((lambda F, a=a, b=b: np.swapaxes(F, dim - 1 - a, dim - 1 - b), perm))
        perm = list(range(Q))  # reflect axis a
        perm[2 * a + 1], perm[2 * a + 2] = 2 * a + 2, 2 * a + 1
        out.append((lambda F, a=a: np.flip(F, axis=dim - 1 - a), perm))
    return out


@pytest.mark.parametrize("dim,n", [(2, 14), (3, 10)])
def test_box_symmetry_pins_corner_and_edge_shares(oracle_lib, dim, n):
    """Equal orders, p = 1/2, isotropic D, u = 0, a pulse centred in the box
    and a non-zero wall value: the populations keep the box's symmetries,
    f_i(x) = f_sigma(i)(sigma x) for every axis swap and reflection sigma.  At
    a 2D corner or 3D edge node a reflection exchanges the two unknown
    populations, and at a 3D corner the axis swaps permute the three, so
    only the equal 2-way and 3-way shares of the Dirichlet deficit (the
    reading used for Sec. 2.5's single-unknown rule) keep this symmetry.
    (C alone cannot pin the split: a zero-sum change of the unknown
    populations at a corner or edge leaves C unchanged at every node; the
    populations it changes only reach interior nodes in zero-mass pairs.)"""
    c = (n - 1) / 2.0
    iso = (0.1 * np.eye(dim)).tolist()
    cfg = synth.small(dim, [n] * dim, seed=27, alpha=[1.5] * dim, p=[0.5] * dim, u=[0.0] * dim, D=iso,
                      c_wall=0.3)
    X = np.meshgrid(*(np.arange(n, dtype=np.float64),) * dim, indexing="ij")
    C0 = np.exp(-sum((x - c) ** 2 for x in X) / (2 * 2.0 ** 2))
    f = oracle_lib.init(cfg, C0)
    f = oracle_lib.step(cfg, f, 30)
    scale = np.abs(f).max()
    for fmap, perm in _symmetries(dim):
        g = np.stack([fmap(f[i]) for i in range(2 * dim + 1)])
        assert np.abs(g[perm] - f).max() <= 1e-13 * scale, perm
    corner = (0,) * dim
    unknown = [f[2 * mu + 1][corner] for mu in range(dim)]  # +x, +y (, +z) come from outside
    assert np.ptp(unknown) <= 1e-13 * scale and abs(unknown[0]) > 1e-3 * scale


def test_one_sided_operator_skips_the_zero_weighted_integral(oracle_lib):
    """p = 1 or p = 0 weighs one integral by exactly zero: the full-field
    term, which then forms only the other sum, equals the node-by-node term,
    which forms both, bit for bit."""
    cfg = synth.small(2, [19, 23], seed=28, alpha=[1.3, 1.8], p=[1.0, 0.0])
    C = np.random.default_rng(3).uniform(-1, 1, (23, 19))
    full = oracle_lib.phi(cfg, C)
    nodes = np.arange(19 * 23)
    at = oracle_lib.phi_at(cfg, C, nodes)
    assert np.array_equal(full.reshape(2, -1), at.reshape(2, -1))


def test_mirror_p_and_u(oracle_lib):
    """Mirroring x maps p_x -> 1 - p_x and u_x -> -u_x (D diagonal)."""
    cfg = synth.small(2, [21, 17], seed=22, alpha=[1.4, 1.7], p=[0.2, 0.65], u=[0.03, 0.01],
                      D=[[0.09, 0.0], [0.0, 0.12]])
    C0 = synth.initial_C(cfg)
    a = oracle_lib.run(cfg, C0, 15)
    mir = dict(cfg, p=[0.8, 0.65], u=[-0.03, 0.01])
    b = oracle_lib.run(mir, C0[:, ::-1], 15)
    assert np.allclose(a, b[:, ::-1], rtol=1e-12, atol=1e-14)


def test_linearity(oracle_lib):
    """With C_wall = 0 and S = 0 the step is linear in the state."""
    cfg = synth.small(2, [15, 12], seed=23)
    rng = np.random.default_rng(1)
    A = rng.uniform(0, 1, (12, 15))
    B = rng.uniform(0, 1, (12, 15))
    ra = oracle_lib.run(cfg, A, 6)
    rb = oracle_lib.run(cfg, B, 6)
    rab = oracle_lib.run(cfg, 2.0 * A - 0.5 * B, 6)
    assert np.allclose(rab, 2.0 * ra - 0.5 * rb, rtol=1e-11, atol=1e-13)


def test_source_adds_w_S_dt(oracle_lib):
    """A constant source adds S dt of mass per step at its node before streaming
    (equation (LBE_FADE)); far from walls total mass grows by S dt per step."""
    cfg = synth.small(2, [31, 31], seed=24, alpha=[2.0, 2.0], u=[0.0, 0.0])
    S = np.zeros((31, 31))
    S[15, 15] = 0.01
    C = oracle_lib.run(cfg, np.zeros((31, 31)), 5, S=S)
    assert C.sum() == pytest.approx(5 * 0.01, rel=1e-12)


def test_step_sampled_matches_full_step(oracle_lib):
    """Consistency of the node-by-node step (used at full size) with the full step."""
    for dim, n in ((2, [11, 9]), (3, [5, 6, 4])):
        cfg = synth.small(dim, n, seed=25, with_source=True)
        S = synth.source(cfg)
        f0 = oracle_lib.init(cfg, synth.initial_C(cfg))
        f0 = oracle_lib.step(cfg, f0, 2, S=S)
        f1 = oracle_lib.step(cfg, f0, 1, S=S)
        nodes = np.arange(0, int(np.prod(n)), 7)
        part = oracle_lib.step_sampled(cfg, f0, nodes, S=S)
        Q = 2 * dim + 1
        assert np.allclose(part, f1.reshape(Q, -1)[:, nodes], rtol=1e-13, atol=1e-14)


def test_invalid_parameters_rejected(oracle_lib):
    base = synth.small(2, [6, 6], seed=26)
    bad = [dict(base, alpha=[1.0, 1.5]), dict(base, alpha=[2.1, 1.5]), dict(base, p=[1.2, 0.5]),
           dict(base, n=[2, 6]), dict(base, D=[[0.1, 0.2], [0.2, 0.1]]), dict(base, tau_free=[0.5, 1, 1, 1])]
    for cfg in bad:
        with pytest.raises(ValueError):
            oracle_lib.run(cfg, np.zeros((6, 6)) if cfg["n"][0] == 6 else np.zeros((6, 2)), 1)


def test_subnormal_flush_changes_nothing_in_the_normal_range(oracle_lib):
    """The golden generator's opt-in subnormal flush (x86 DAZ/FTZ in the oracle's
    threads) may only alter values below the FP64 normal range: a run whose
    tails stay normal is bit-identical with and without it, and a run seeded
    with subnormal concentrations differs from the unflushed run by less than
    1e-300 anywhere."""
    cfg = synth.small(2, [40, 33], alpha=[1.3, 1.7], p=[1.0, 0.0], seed=21)
    C0 = synth.initial_C(cfg)
    a = oracle_lib.run(cfg, C0, 15)
    tiny = np.finfo(np.float64).tiny
    C1 = C0.copy()
    C1[5:9, 5:30] = 0.25 * tiny  # subnormal
    b = oracle_lib.run(cfg, C1, 15)
    try:
        oracle_lib.flush_subnormals(True)
        af = oracle_lib.run(cfg, C0, 15)
        bf = oracle_lib.run(cfg, C1, 15)
    finally:
        oracle_lib.flush_subnormals(False)
    if np.any((np.abs(a) > 0) & (np.abs(a) < tiny)):
        assert np.max(np.abs(af - a)) < 1e-300
    else:
        assert np.array_equal(af, a)
    assert np.max(np.abs(bf - b)) < 1e-300
    assert np.array_equal(oracle_lib.run(cfg, C0, 15), a)  # flush is off again
