"""Stability of the oracle at high Peclet number (Sec. 3.3), pinned to a
linear stability analysis of the printed scheme (``linear_stability``): in a
linearly unstable case the oracle's max |C| must grow per step at the
spectral radius of the von Neumann amplification matrix (within 1.5 %: the
bounded domain with walls, and the sampled wave vectors), and in a stable
case it must stay bounded.  This checks the collision (BGK and MRT with the
free relaxation times), the advective part of the equilibrium and the
fractional symbol in a regime the other pins do not reach.

What of the paper's statements the scheme as read reproduces (the growth
rates below hold for the paper's own mesh, dx = 0.01, dt = 8e-4, D = 2e-3):
BGK is unstable for the advection-diffusion equation at u1 = 5 and for
alpha = 1.7 at u1 = 1, MRT grows far more slowly than BGK and the more so the
larger lambda_3 = lambda_4, and BGK at u1 = 0.7 does not blow up.  MRT with
lambda_3 = lambda_4 = 2.1277 at u1 = 1 is still weakly unstable (spectral
radius 1.010), so with the paper's needle-like initial condition
(sigma_0 = 0.002 < dx) its growth is visible before t = 1.
"""
import numpy as np
import pytest

import synth
from linear_stability import measured_rate, spectral_radius


def _history(oracle_lib, alpha, u1, collision, tau, steps, every=10, cap=1e200):
    cfg = synth.stability_config(alpha, u1, collision, tau)
    C0 = synth.paper_gaussian(cfg, (0.5, 0.5))
    f = oracle_lib.init(cfg, C0)
    maxes = [float(np.abs(C0).max())]
    for _ in range(steps // every):
        f = oracle_lib.step(cfg, f, every)
        maxes.append(float(np.abs(oracle_lib.moment(cfg, f)).max()))
        if maxes[-1] > cap:
            break
    return cfg, maxes


@pytest.mark.parametrize("alpha,u1,collision,tau,steps", [
    (2.0, 5.0, "BGK", 1.0, 300),
    (2.0, 5.0, "MRT", 2.1277, 400),
    (1.7, 1.0, "BGK", 1.0, 400),
    (1.7, 1.0, "MRT", 2.1277, 1250),
])
def test_growth_rate_is_the_von_neumann_spectral_radius(oracle_lib, alpha, u1, collision, tau, steps):
    cfg, maxes = _history(oracle_lib, alpha, u1, collision, tau, steps)
    u_lat = u1 * cfg["dt"] / cfg["dx"]
    lam = 0.5 + cfg["D"][0][0] * cfg["dt"] / (cfg["dx"] ** 2 / 3.0)
    rho = spectral_radius(u_lat, lam, tau, alpha, 0.5, cfg["dx"], collision == "BGK")
    rate = measured_rate(maxes, 10)
    print(f"alpha={alpha} u1={u1} {collision} tau={tau}: measured {rate:.4f}, von Neumann {rho:.4f}")
    assert rho > 1.0
    assert rho - 0.015 <= rate <= rho + 0.003


def test_stable_case_stays_bounded(oracle_lib):
    """BGK at u1 = 0.7, alpha = 1.7 (spectral radius 1): no growth to t = 1."""
    cfg, maxes = _history(oracle_lib, 1.7, 0.7, "BGK", 1.0, 1250, every=50)
    rho = spectral_radius(0.7 * cfg["dt"] / cfg["dx"], 0.548, 1.0, 1.7, 0.5, cfg["dx"], True)
    assert rho < 1.0 + 1e-9
    assert max(maxes[1:]) <= maxes[0]


def test_larger_free_times_grow_more_slowly():
    """MRT against BGK in the paper's unstable cases: the spectral radius falls
    as lambda_3 = lambda_4 grows (u1 = 5 ADE; u1 = 1 and 1.3 at alpha = 1.7)."""
    dx, dt = 0.01, 8e-4
    for alpha, u1 in ((2.0, 5.0), (1.7, 1.0), (1.7, 1.3)):
        r_bgk = spectral_radius(u1 * dt / dx, 0.548, 1.0, alpha, 0.5, dx, True, nk=91)
        r = [spectral_radius(u1 * dt / dx, 0.548, t, alpha, 0.5, dx, False, nk=91) for t in (1.0, 2.1277, 2.6316)]
        assert r_bgk > r[0] > r[1] > r[2] >= 1.0, (alpha, u1, r_bgk, r)


def test_alternative_readings_of_section_3_3():
    """Sec. 3.3 states that free relaxation times lambda_3 = lambda_4 > 0.833
    re-stabilise the advection-diffusion case at u1 = 5, and that 2.1277 and
    2.6316 keep alpha = 1.7 stable at u1 = 1 and 1.3.  No reading of the
    scheme tried here reproduces all of these (von Neumann radii; the scheme
    as printed is the default reading):
      * as printed: 0.833 grows (radius 1.125), 2.1277 / 2.6316 grow by ~1 %;
      * one free time on row 3 or row 4 of M only (the other 1): still grows,
        so the garbled D2Q5 mapping of lambda_3 / lambda_4 does not matter;
      * free values as rates (Lambda's entries): rates above 2 diverge;
      * the usual second-order velocity terms in f^eq (not in eq. (Feq)): 0.833
        becomes stable for the advection-diffusion case but 1.0 and 2.1277
        do not (the opposite of '> 0.833'), and alpha = 1.7 still grows."""
    dx, dt, lam = 0.01, 8e-4, 0.548
    kw = dict(nk=61, ky_step=1)
    u5, u1 = 5.0 * dt / dx, 1.0 * dt / dx
    printed = spectral_radius(u5, lam, 0.833, 2.0, 0.5, dx, False, **kw)
    assert printed > 1.1
    assert spectral_radius(u5, lam, 10.0, 2.0, 0.5, dx, False, **kw) <= 1.0 + 1e-9
    assert spectral_radius(u5, lam, 0.833, 2.0, 0.5, dx, False, tau4=1.0, **kw) > 1.1
    assert spectral_radius(u5, lam, 1.0, 2.0, 0.5, dx, False, tau4=0.833, **kw) > 1.1
    assert spectral_radius(u1, lam, 2.1277, 1.7, 0.5, dx, False, free_as_rates=True, **kw) > 1.2
    assert spectral_radius(u5, lam, 0.833, 2.0, 0.5, dx, False, velocity_squared=True, **kw) <= 1.0 + 1e-9
    assert spectral_radius(u5, lam, 1.0, 2.0, 0.5, dx, False, velocity_squared=True, **kw) > 1.002
    assert spectral_radius(u1, lam, 2.1277, 1.7, 0.5, dx, False, velocity_squared=True, **kw) > 1.005
    assert spectral_radius(u1, lam, 2.1277, 1.7, 0.5, dx, False, **kw) > 1.005
