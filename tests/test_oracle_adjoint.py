"""Pins of the oracle's hand-written FP64 adjoint.

With a zero wall value the map (C0, S) -> C_n is linear, so L = <gC, C_n>
equals <dL/dC0, C0> + <dL/dS, S> exactly: a dot-product identity that any
error in the transposed streaming, boundary rule, collision, equilibrium or
fractional term breaks.  The parameter gradients (D, u, p) are checked
against FP64 central differences of the forward oracle.
"""
import numpy as np
import pytest

import synth


def _problem(dim, n, collision="MRT", seed=61, c_wall=0.0):
    cfg = synth.small(dim, n, seed=seed, collision=collision, with_source=True, c_wall=c_wall)
    rng = np.random.default_rng(seed + 7)
    C0 = synth.initial_C(cfg)
    S = synth.source(cfg)
    gC = rng.standard_normal(synth.shape(cfg))
    return cfg, C0, S, gC


@pytest.mark.parametrize("dim,n,collision", [(2, [13, 11], "MRT"), (2, [9, 12], "BGK"), (3, [7, 6, 5], "MRT"),
                                             (3, [6, 5, 7], "BGK")])
def test_linear_identity(oracle_lib, dim, n, collision):
    cfg, C0, S, gC = _problem(dim, n, collision)
    steps = 7
    g = oracle_lib.adjoint(cfg, C0, steps, gC, S=S)
    Lf = oracle_lib.loss(cfg, C0, steps, gC, S=S)
    Ladj = float(np.sum(g["dC0"] * C0) + np.sum(g["dS"] * S))
    assert Ladj == pytest.approx(Lf, rel=1e-12, abs=1e-14)


def test_affine_with_wall_value(oracle_lib):
    """Non-zero wall value: L(C0 + delta) - L(C0) = <dL/dC0, delta> exactly, and
    dL/dC0 vanishes on the wall nodes (they are overwritten)."""
    cfg, C0, S, gC = _problem(2, [12, 10], c_wall=0.4)
    steps = 6
    g = oracle_lib.adjoint(cfg, C0, steps, gC, S=S)
    rng = np.random.default_rng(3)
    delta = rng.standard_normal(C0.shape)
    dL = oracle_lib.loss(cfg, C0 + delta, steps, gC, S=S) - oracle_lib.loss(cfg, C0, steps, gC, S=S)
    assert float(np.sum(g["dC0"] * delta)) == pytest.approx(dL, rel=1e-11)
    wall = np.ones_like(C0, bool)
    wall[1:-1, 1:-1] = False
    assert np.all(g["dC0"][wall] == 0.0)


def _fd(oracle_lib, cfg, C0, S, gC, steps, mutate, h):
    a, b = dict(cfg), dict(cfg)
    mutate(a, +h)
    mutate(b, -h)
    return (oracle_lib.loss(a, C0, steps, gC, S=S) - oracle_lib.loss(b, C0, steps, gC, S=S)) / (2 * h)


@pytest.mark.parametrize("dim,n,collision", [(2, [11, 10], "MRT"), (3, [6, 6, 5], "MRT"), (2, [10, 9], "BGK")])
def test_parameter_gradients_match_central_differences(oracle_lib, dim, n, collision):
    cfg, C0, S, gC = _problem(dim, n, collision, seed=71)
    steps = 6
    g = oracle_lib.adjoint(cfg, C0, steps, gC, S=S)
    h = 1e-5

    def set_vec(key, k):
        def f(c, dh):
            v = list(c[key])
            v[k] = v[k] + dh
            c[key] = v
        return f

    for k in range(dim):
        fd_u = _fd(oracle_lib, cfg, C0, S, gC, steps, set_vec("u", k), h)
        assert g["u"][k] == pytest.approx(fd_u, rel=1e-7, abs=1e-10)
        fd_p = _fd(oracle_lib, cfg, C0, S, gC, steps, set_vec("p", k), h)
        assert g["p"][k] == pytest.approx(fd_p, rel=1e-7, abs=1e-10)
    D0 = np.array(cfg["D"])
    if collision == "BGK":
        def scale_D(c, dh):
            c["D"] = ((D0[0, 0] + dh) * np.eye(dim)).tolist()
        fd = _fd(oracle_lib, cfg, C0, S, gC, steps, scale_D, h)
        assert np.trace(g["D"]) == pytest.approx(fd, rel=1e-7)
        return
    for a in range(dim):
        for b in range(a, dim):
            def pert(c, dh, a=a, b=b):
                D = D0.copy()
                D[a, b] += dh
                if a != b:
                    D[b, a] += dh
                c["D"] = D.tolist()
            fd = _fd(oracle_lib, cfg, C0, S, gC, steps, pert, h)
            expect = g["D"][a, b] * (1 if a == b else 2)
            assert expect == pytest.approx(fd, rel=1e-6, abs=1e-10), (a, b)


@pytest.mark.parametrize("dim,n", [(2, [11, 10]), (3, [6, 7, 5])])
def test_caputo_variant_adjoint(oracle_lib, dim, n):
    """The Caputo-type flux (Sec. 3.5) adds boundary terms to the fractional
    term that reach the wall values of each line: with a non-zero wall value
    the affine identity for C0 and the D, u, p gradients against central
    differences."""
    cfg, C0, S, gC = _problem(dim, n, seed=73, c_wall=0.3)
    cfg["flux_form"] = "caputo"
    steps = 5
    g = oracle_lib.adjoint(cfg, C0, steps, gC, S=S)
    rng = np.random.default_rng(4)
    delta = rng.standard_normal(C0.shape)
    dL = oracle_lib.loss(cfg, C0 + delta, steps, gC, S=S) - oracle_lib.loss(cfg, C0, steps, gC, S=S)
    assert float(np.sum(g["dC0"] * delta)) == pytest.approx(dL, rel=1e-11)
    h = 1e-5
    for k in range(dim):
        for key in ("u", "p"):
            def f(c, dh, key=key, k=k):
                v = list(c[key])
                v[k] = v[k] + dh
                c[key] = v
            fd = _fd(oracle_lib, cfg, C0, S, gC, steps, f, h)
            assert g[key][k] == pytest.approx(fd, rel=1e-7, abs=1e-10), (key, k)
    D0 = np.array(cfg["D"])

    def pert(c, dh):
        c["D"] = (D0 + dh * np.eye(dim)).tolist()
    fd = _fd(oracle_lib, cfg, C0, S, gC, steps, pert, h)
    assert np.trace(g["D"]) == pytest.approx(fd, rel=1e-6)
