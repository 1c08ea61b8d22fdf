"""Von Neumann (Fourier) amplification of the D2Q5 scheme, for the stability
pins of Sec. 3.3.  Test infrastructure, independent of the oracle and of the
GPU library: on an infinite periodic lattice one step maps the Fourier
amplitudes of the five populations by G(k) = S(k) (I - R + R E(k)), with the
streaming shifts S(k) = diag(exp(-i k.e_i)), the collision matrix
R = M^-1 Lambda M (M as printed in equation (MatrixD2); BGK: I / lambda), and
the equilibrium map E(k) (equations (Feq), (CoeffA_FADE3D)) with the symbol of
the discrete fractional integral, s [p (1 + sum_k a_k e^-ik.theta) + (1 - p)
(1 + sum_k a_k e^ik.theta)], a_k = (k+1)^(g+1) - 2 k^(g+1) + (k-1)^(g+1)
(the interior product-rule weights of Sec. 2.4), truncated at K terms.  The
scheme is linearly unstable when the spectral radius of G exceeds 1.
"""
import math

import numpy as np

M = np.array([[1, 1, 1, 1, 1], [0, 1, -1, 0, 0], [0, 0, 0, 1, -1], [4, -1, -1, -1, -1], [0, 1, 1, -1, -1]], float)
E_VEC = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1]])
W = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])
E2 = 1.0 / 3.0


def symbol(theta: float, alpha: float, p: float, dx: float, K: int = 4000) -> complex:
    gam = 2.0 - alpha
    if gam == 0.0:
        return 1.0 + 0j
    k = np.arange(1, K, dtype=np.float64)
    a = (k + 1.0) ** (gam + 1) - 2.0 * k ** (gam + 1) + (k - 1.0) ** (gam + 1)
    s = dx ** gam / math.gamma(2.0 + gam)
    lower = 1.0 + np.sum(a * np.exp(-1j * k * theta))
    upper = 1.0 + np.sum(a * np.exp(1j * k * theta))
    return s * (p * lower + (1.0 - p) * upper)


def spectral_radius(u_lat: float, lam: float, tau_free: float, alpha: float, p: float, dx: float, bgk: bool,
                    nk: int = 181, tau4: float | None = None, free_as_rates: bool = False,
                    velocity_squared: bool = False, ky_step: int | None = None) -> float:
    """Largest |eigenvalue| of G over a grid of wave vectors (k_x, k_y) in
    [-pi, pi]^2, velocity (u_lat, 0) in lattice units, isotropic
    relaxation time lam of the fluxes (BGK: of every moment).

    Alternative readings of Sec. 3.3, for comparison with the printed scheme
    (the defaults): tau4 gives row 4 of M (0, 1, 1, -1, -1) its own value
    (tau_free then belongs to row 3 only); free_as_rates takes the free values
    as relaxation rates (Lambda's entries) instead of times; velocity_squared
    adds the second-order velocity terms of the usual advection-diffusion
    equilibrium, w_i C [(e_i.u)^2 / (2 e^4) - u^2 / (2 e^2)], which equation
    (Feq) does not have."""
    t3 = tau_free
    t4 = tau_free if tau4 is None else tau4
    if bgk:
        R = np.eye(5) / lam
    elif free_as_rates:
        R = np.linalg.inv(M) @ np.diag([1.0, 1 / lam, 1 / lam, t3, t4]) @ M
    else:
        R = np.linalg.inv(M) @ np.diag([1.0, 1 / lam, 1 / lam, 1 / t3, 1 / t4]) @ M
    ks = np.linspace(-math.pi, math.pi, nk)
    sym = {k: symbol(k, alpha, p, dx) for k in ks}
    u2 = W * ((E_VEC[:, 0] * u_lat) ** 2 / (2 * E2 * E2) - u_lat ** 2 / (2 * E2)) if velocity_squared else 0.0
    best = 0.0
    for kx in ks:
        for ky in ks[:: (ky_step or max(1, nk // 30))]:
            px, py = sym[kx], sym[ky]
            feq = np.array([1 - W[0] * (px + py), W[1] * (px + u_lat / E2), W[2] * (px - u_lat / E2), W[3] * py,
                            W[4] * py]) + u2
            A = np.eye(5) - R + R @ np.outer(feq, np.ones(5))
            S = np.diag(np.exp(-1j * (E_VEC[:, 0] * kx + E_VEC[:, 1] * ky)))
            best = max(best, float(np.abs(np.linalg.eigvals(S @ A)).max()))
    return best


def measured_rate(maxes, every: int) -> float:
    """Per-step growth of max |C| over the last third of a history sampled
    every `every` steps (the unstable mode dominates there)."""
    m = np.asarray(maxes, np.float64)
    a = len(m) - 1 - (len(m) - 1) // 3
    return float((m[-1] / m[a]) ** (1.0 / ((len(m) - 1 - a) * every)))
