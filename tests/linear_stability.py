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
                    nk: int = 181) -> float:
    """Largest |eigenvalue| of G over a grid of wave vectors (k_x, k_y) in
    [-pi, pi]^2, velocity (u_lat, 0) in lattice units, isotropic
    relaxation time lam of the fluxes (BGK: of every moment)."""
    if bgk:
        R = np.eye(5) / lam
    else:
        R = np.linalg.inv(M) @ np.diag([1.0, 1 / lam, 1 / lam, 1 / tau_free, 1 / tau_free]) @ M
    ks = np.linspace(-math.pi, math.pi, nk)
    sym = {k: symbol(k, alpha, p, dx) for k in ks}
    best = 0.0
    for kx in ks:
        for ky in ks[:: max(1, nk // 30)]:
            px, py = sym[kx], sym[ky]
            feq = np.array([1 - W[0] * (px + py), W[1] * (px + u_lat / E2), W[2] * (px - u_lat / E2), W[3] * py,
                            W[4] * py])
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
