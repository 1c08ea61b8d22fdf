"""GPU random walk (lbm_rw_* of the C ABI) against the oracle's walk and
against the GPU LB solver.

Both sides draw the same counter-based numbers and evaluate the same FP64
formulas with the same operation order (no contraction into FMA), so a
particle's path agrees up to the last-ulp differences of the device and host
sin / cos / log / pow: positions within 1e-12 relative after hundreds of
steps, and the exit and binning decisions, taken in FP64 on both sides,
identical (a particle would have to sit within ~1e-13 of a wall or a bin edge
for them to differ).  Runs are independent of how particles and steps are
split across calls.  At scale the density of the surviving particles is
compared with the LB solution, as in the paper's comparisons (Sec. 3.2).
"""
import math
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rw(dim, lo, hi, alpha, p, D, **kw):
    from paper_1706_09161_amd.random_walk import RandomWalk

    return RandomWalk(dim, lo, hi, alpha=alpha, p=p, D=D, **kw)


CASES = [
    # dim, box, alpha, p, D, u, dt, center, sigma0
    (2, ([0, 0], [2, 2]), [1.5, 1.99], [0.5, 0.5], [0.5, 0.5], [0.0, 0.0], 1e-3, [1.0, 1.0], 0.1),
    (2, ([0, 0], [2, 1]), [1.7, 1.2], [0.9, 0.2], [0.02, 0.05], [0.5, -0.1], 1e-3, [0.5, 0.5], 0.05),
    (1, ([-1], [3]), [1.3], [0.0], [0.1], [0.2], 5e-4, [0.0], 0.2),
    (3, ([0, 0, 0], [1, 1, 1]), [1.5, 1.8, 2.0], [0.7, 0.5, 0.3], [0.01, 0.02, 0.03], [0.0, 0.1, 0.0], 1e-3,
     [0.5, 0.5, 0.5], 0.1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-a{c[2][0]}")
def test_paths_match_the_oracle(case):
    dim, (lo, hi), alpha, p, D, u, dt, center, s0 = case
    n, steps, seed = 20000, 200, 77
    print(f"[gpu-rw] paths dim={dim} alpha={alpha}", flush=True)
    P = oracle.rw_params(dim, lo, hi, alpha, p, D, u=u, dt=dt, seed=seed)
    x0, a0 = oracle.rw_init_gaussian(P, center, s0, n)
    xr, ar = oracle.rw_walk(P, x0, a0, steps)
    W = _rw(dim, lo, hi, alpha, p, D, u=u, dt=dt, seed=seed)
    x, alive = W.init_gaussian(center, s0, n)
    xi = x.cpu().numpy()
    assert np.array_equal(alive.cpu().numpy(), a0)
    assert np.abs(xi - x0).max() <= 1e-14 * np.abs(x0).max()
    W.walk(x, alive, steps)
    xg, ag = x.cpu().numpy(), alive.cpu().numpy()
    assert np.array_equal(ag, ar), int((ag != ar).sum())
    live = ar == 1
    rel = np.abs(xg[:, live] - xr[:, live]).max() / np.abs(xr[:, live]).max()
    print(f"[gpu-rw] survivors {live.mean():.4f}, max rel position difference {rel:.2e}", flush=True)
    assert rel <= 1e-12
    nodes = [41] * dim
    dx = (hi[0] - lo[0]) / 40
    if all(abs((hi[mu] - lo[mu]) / dx - round((hi[mu] - lo[mu]) / dx)) < 1e-9 for mu in range(dim)):
        nodes = [int(round((hi[mu] - lo[mu]) / dx)) + 1 for mu in range(dim)]
    hg = W.histogram(x, alive, nodes, dx).cpu().numpy().astype(np.int64)
    hr = oracle.rw_histogram(P, xr, ar, nodes, dx).astype(np.int64)
    assert np.array_equal(hg, hr)


def test_runs_do_not_depend_on_the_split():
    """Particles split across two calls and steps split into two runs give the
    same paths bit for bit (counters carry the particle index and step)."""
    dim, lo, hi = 2, [0, 0], [2, 2]
    W = _rw(dim, lo, hi, alpha=[1.6, 1.4], p=[0.3, 0.8], D=[0.1, 0.2], dt=1e-3, seed=5)
    n, half = 30000, 12345
    x, a = W.init_gaussian([1, 1], 0.2, n)
    W.walk(x, a, 150)
    x1, a1 = W.init_gaussian([1, 1], 0.2, half, first=0)
    x2, a2 = W.init_gaussian([1, 1], 0.2, n - half, first=half)
    W.walk(x1, a1, 60)
    W.walk(x1, a1, 90, step0=60)
    W.walk(x2, a2, 150, first=half)
    assert torch.equal(torch.cat([x1, x2], dim=1), x) and torch.equal(torch.cat([a1, a2]), a)


def test_brownian_limit_on_gpu():
    """alpha = 2 far from walls: mean and variance in closed form (1e6 particles)."""
    W = _rw(2, [-1e9, -1e9], [1e9, 1e9], alpha=[2.0, 2.0], p=[0.1, 0.9], D=[0.3, 0.05], g=[1.0, 2.0],
            u=[0.4, -0.2], dt=0.01, seed=9)
    N, t, s0 = 1_000_000, 0.5, 0.05
    x, a = W.init_gaussian([0.1, 0.2], s0, N)
    W.walk(x, a, int(round(t / 0.01)))
    xs = x.cpu().numpy()
    for mu, (D, g, u, c) in enumerate(((0.3, 1.0, 0.4, 0.1), (0.05, 2.0, -0.2, 0.2))):
        var = s0 ** 2 + 2 * D * g * t
        assert abs(xs[mu].mean() - (c + u * t)) < 5 * math.sqrt(var / N)
        assert abs(xs[mu].var() / var - 1) < 5 * math.sqrt(2 / N)


def test_walk_against_lb_validation_1():
    """The paper's validation 1 (Sec. 3.2): Omega = [0, 2]^2, x_s = (1, 1),
    D = 0.5 Id, g = 1, alpha = (1.5, 1.99), p = 1/2, u = 0, dx = 0.02 (101
    nodes), LB dt = 1e-4 to t = 0.1; walk dt = 1e-3 (the paper's bound), 4e6
    particles, sigma0 = 0.05 (resolved by the grid, so both start from the same
    mass).  The surviving mass and the marginal profiles of the walk's density
    against the LB solution, and the 2D density where it is well sampled."""
    from paper_1706_09161_amd import LbmFade

    n, dx, dt, T, s0 = 101, 0.02, 1e-4, 0.1, 0.05
    cfg = dict(dim=2, n=[n, n], dx=dx, dt=dt, alpha=[1.5, 1.99], p=[0.5, 0.5], g=[1.0, 1.0],
               D=[[0.5, 0.0], [0.0, 0.5]], u=[0.0, 0.0], collision="MRT", tau_free=[1.0] * 4, tau0=1.0, c_wall=0.0)
    C0 = synth.paper_gaussian(cfg, (1.0, 1.0), sigma0=s0, C0=1.0)
    with LbmFade.from_config(cfg) as s:
        s.set_C(C0.astype(np.float32))
        s.step(int(round(T / dt)))
        C = s.get_C(device=False).astype(np.float64)
    mass0 = C0.sum() * dx * dx
    W = _rw(2, [0, 0], [2, 2], alpha=[1.5, 1.99], p=[0.5, 0.5], D=[0.5, 0.5], dt=1e-3, seed=2024)
    N = 4_000_000
    x, a = W.init_gaussian([1.0, 1.0], s0, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W.walk(x, a, int(round(T / 1e-3)))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    dens = W.histogram(x, a, [n, n], dx).cpu().numpy().astype(np.float64) / N / dx ** 2
    surv = float(a.float().mean())
    print(f"[gpu-rw] validation 1: {N} particles x 100 steps in {secs * 1e3:.1f} ms "
          f"({N * 100 * 2 / secs / 1e9:.2f} G stable draws/s); survival {surv:.5f}, "
          f"LB mass {C.sum() * dx * dx / mass0:.5f}", flush=True)
    assert abs(surv - C.sum() * dx * dx / mass0) < 4 * math.sqrt(surv * (1 - surv) / N) + 2e-3
    Cn = C / mass0
    for ax in (0, 1):
        m_lb, m_rw = Cn.sum(axis=ax) * dx, dens.sum(axis=ax) * dx
        err = np.linalg.norm(m_lb - m_rw) / np.linalg.norm(m_lb)
        print(f"[gpu-rw] marginal along axis {1 - ax}: rel L2 {err:.2e}", flush=True)
        assert err < 0.01
    well = Cn > 0.2 * Cn.max()
    rel2d = np.abs(dens[well] - Cn[well]) / Cn[well]
    print(f"[gpu-rw] 2D density where C > 20% of max: median rel diff {np.median(rel2d):.3f}", flush=True)
    assert np.median(rel2d) < 0.03
    # most paths leave through the walls normal to x1, where alpha_1 = 1.5
    # makes long jumps likely (a dead particle keeps its first position outside)
    xs, dead = x.cpu().numpy(), a.cpu().numpy() == 0
    out1 = dead & ((xs[0] <= 0.0) | (xs[0] >= 2.0))
    print(f"[gpu-rw] exits through the x1 walls: {out1.sum()} of {dead.sum()}", flush=True)
    assert out1.sum() > 0.7 * dead.sum()


def _lb_vs_walk(dim, n, L, dx, dt, T, alpha, p, center, s0, seed, N=4_000_000, dt_rw=1e-3):
    """GPU LB (BGK, D = 0.5 Id, g = 1, u = 0, walls 0) and GPU walk from the
    same resolved Gaussian hill: the LB field normalised by its initial mass,
    the walk's density per node, their surviving masses."""
    from paper_1706_09161_amd import LbmFade

    cfg = dict(dim=dim, n=[n] * dim, dx=dx, dt=dt, alpha=list(alpha), p=list(p), g=[1.0] * dim,
               D=(0.5 * np.eye(dim)).tolist(), u=[0.0] * dim, collision="BGK", tau_free=[1.0] * 4, tau0=1.0,
               c_wall=0.0)
    C0 = synth.paper_gaussian(cfg, center, sigma0=s0, C0=1.0)
    with LbmFade.from_config(cfg) as s:
        s.set_C(C0.astype(np.float32))
        s.step(int(round(T / dt)))
        C = s.get_C(device=False).astype(np.float64)
    mass0 = C0.sum() * dx ** dim
    W = _rw(dim, [0.0] * dim, [L] * dim, alpha=list(alpha), p=list(p), D=[0.5] * dim, dt=dt_rw, seed=seed)
    x, a = W.init_gaussian(center, s0, N)
    W.walk(x, a, int(round(T / dt_rw)))
    dens = W.histogram(x, a, [n] * dim, dx).cpu().numpy().astype(np.float64) / N / dx ** dim
    surv = float(a.float().mean())
    return C / mass0, dens, C.sum() * dx ** dim / mass0, surv


def test_walk_against_lb_validation_2():
    """The paper's validation 2 (Sec. 3.2): Omega = [0, 2]^2, alpha = 1.2,
    p = (0.35, 0.5) (skewed along x1 only), D = 0.5 Id, BGK, dx = 0.01 (201
    nodes), dt = 5e-5, to t = 0.6.  LB and walk agree on the surviving mass
    and both marginals, and both show what the paper describes: with p1 < 1/2
    the maximum moves to larger x1 although u = 0, and the x1-profile decays
    more slowly to the left of its maximum than to the right."""
    n, dx = 201, 0.01
    Cn, dens, mass_lb, surv = _lb_vs_walk(2, n, 2.0, dx, 5e-5, 0.6, (1.2, 1.2), (0.35, 0.5), (1.0, 1.0), 0.05,
                                          seed=2025)
    N = 4_000_000
    print(f"[gpu-rw] validation 2: survival {surv:.5f}, LB mass {mass_lb:.5f}", flush=True)
    assert abs(surv - mass_lb) < 4 * math.sqrt(surv * (1 - surv) / N) + 2e-3
    xs = np.arange(n) * dx
    prof = {}
    for ax, name in ((0, "x1"), (1, "x2")):
        m_lb, m_rw = Cn.sum(axis=ax) * dx, dens.sum(axis=ax) * dx
        err = np.linalg.norm(m_lb - m_rw) / np.linalg.norm(m_lb)
        print(f"[gpu-rw] marginal along {name}: rel L2 {err:.2e}", flush=True)
        assert err < 0.02
        prof[name] = (m_lb, m_rw)
    for m in prof["x1"]:
        k = int(np.argmax(m))
        print(f"[gpu-rw] x1 marginal: peak at {xs[k]:.2f}; 0.3 and 0.5 either side of it: "
              f"{m[k - 30]:.3f} / {m[k + 30]:.3f}, {m[k - 50]:.3f} / {m[k + 50]:.3f}", flush=True)
        assert xs[k] > 1.0 + 2 * dx
        assert m[k - 30] > m[k + 30] and m[k - 50] > m[k + 50]
    m2 = prof["x2"][0]
    assert abs(xs[int(np.argmax(m2))] - 1.0) <= dx  # p2 = 1/2: no shift along x2


def test_walk_against_lb_validation_3():
    """The paper's validation 3 (Sec. 3.2): Omega = [0, 1]^3, alpha = 1.2,
    p = (0.35, 0.5, 0.5), D = 0.5 Id, BGK, dx = 0.0125 (81 nodes per axis),
    dt = 3e-5, to t = 0.21: surviving mass, the x1-marginal, and its maximum
    moved to larger x1."""
    n, dx = 81, 0.0125
    Cn, dens, mass_lb, surv = _lb_vs_walk(3, n, 1.0, dx, 3e-5, 0.21, (1.2, 1.2, 1.2), (0.35, 0.5, 0.5),
                                          (0.5, 0.5, 0.5), 0.05, seed=2026)
    N = 4_000_000
    print(f"[gpu-rw] validation 3: survival {surv:.5f}, LB mass {mass_lb:.5f}", flush=True)
    assert abs(surv - mass_lb) < 4 * math.sqrt(surv * (1 - surv) / N) + 3e-3
    xs = np.arange(n) * dx
    for axes, name in (((0, 1), "x1"), ((0, 2), "x2")):
        m_lb, m_rw = Cn.sum(axis=axes) * dx * dx, dens.sum(axis=axes) * dx * dx
        err = np.linalg.norm(m_lb - m_rw) / np.linalg.norm(m_lb)
        print(f"[gpu-rw] 3D marginal along {name}: rel L2 {err:.2e}", flush=True)
        assert err < 0.03
        if name == "x1":
            for m in (m_lb, m_rw):
                assert xs[int(np.argmax(m))] > 0.5 + dx


def test_empty_and_degenerate_inputs():
    """No particles, no steps, sigma0 = 0 (every particle starts at the
    centre), and a particle that starts on a wall (dead from the start, never
    moved)."""
    W = _rw(2, [0, 0], [1, 1], alpha=[1.5, 1.5], p=[0.5, 0.5], D=[0.1, 0.1], dt=1e-3, seed=3)
    x, a = W.init_gaussian([0.5, 0.5], 0.1, 0)
    W.walk(x, a, 10)
    h = W.histogram(x, a, [11, 11], 0.1)
    assert x.shape == (2, 0) and a.numel() == 0 and int(h.sum()) == 0
    x, a = W.init_gaussian([0.5, 0.5], 0.0, 1000)
    assert torch.all(x == 0.5) and torch.all(a == 1)
    before = x.clone()
    W.walk(x, a, 0)
    assert torch.equal(x, before)
    x, a = W.init_gaussian([0.0, 0.5], 0.0, 10)  # on the wall x1 = 0: outside the open box
    assert torch.all(a == 0)
    W.walk(x, a, 5)
    assert torch.all(x[0] == 0.0) and torch.all(a == 0)
    assert int(W.histogram(x, a, [11, 11], 0.1).sum()) == 0
