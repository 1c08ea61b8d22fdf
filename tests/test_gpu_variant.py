"""GPU parity of the Caputo-type flux variant (Sec. 3.5, equations (Fg2),
(CoeffA_FADE3DPS); flux_form = LBM_FLUX_CAPUTO), and of the fractional term's
values on wall nodes with non-zero wall values (the empty-interval
coefficients c+_00 = c-_NN = 0^gamma), through the C ABI against the FP64
oracle.

The variant changes only the two boundary columns of every axis operator, so
the GEMM kernels run unchanged; the tolerances of the constant-coefficient
tests apply, with the bound of a fractional-term value taken on the sum of the
magnitudes it is formed from: for C >= 0, Phi(C) and the boundary terms
Phi(C) - Phi~(C) are both non-negative, and 2 Phi(C) - Phi~(C) bounds their sum
(the kernels add each boundary column whole, so nothing else is added and
cancelled).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import GOLDEN

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(cfg, precision="fp32", **kw):
    from paper_1706_09161_amd import LbmFade

    return LbmFade.from_config(cfg, precision=precision, **kw)


def _rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def _banner(msg):
    print(f"[gpu-variant] {msg}", flush=True)


PHI_CASES = [
    (2, [67, 45], [1.3, 1.8], [0.3, 0.8]),
    (2, [130, 97], [1.5, 1.2], [1.0, 0.0]),
    (2, [3, 5], [1.7, 2.0], [0.2, 0.9]),
    (3, [21, 18, 13], [1.5, 1.6, 1.8], [0.5, 0.2, 0.9]),
]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp32_simt"])
@pytest.mark.parametrize("flux_form", ["rl", "caputo"])
@pytest.mark.parametrize("case", PHI_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_fractional_term_with_wall_values(case, flux_form, precision):
    """Random C >= 0 (wall nodes included): every value of every axis."""
    dim, n, alpha, p = case
    _banner(f"phi {flux_form} {precision} dim={dim} n={n}")
    cfg = synth.small(dim, n, alpha=alpha, p=p, seed=37, flux_form=flux_form)
    cfg["g"] = [1.3, 0.7, 1.1][:dim]
    cfg["dx"] = 0.5
    rng = np.random.default_rng(23)
    C = rng.uniform(0.0, 1.0, synth.shape(cfg)).astype(np.float32)
    ref = oracle.phi(cfg, C.astype(np.float64))
    rl = oracle.phi(dict(cfg, flux_form="rl"), C.astype(np.float64))
    scale = 2 * rl - ref if flux_form == "caputo" else rl.copy()
    with _solver(cfg, precision) as s:
        got = s.apply_phi(torch.from_numpy(C).cuda()).cpu().numpy().astype(np.float64)
    rel = 4 * max(n) * 2.0**-24 if precision != "bf16x3" else 2.0**-14
    err = np.abs(got - ref) / (scale + 1e-30)
    _banner(f"max err / scale {err.max():.2e}")
    assert np.all(np.abs(got - ref) <= rel * scale + 1e-30), err.max()


@pytest.mark.parametrize("dim,n,collision,precision", [(2, [70, 66], "MRT", "fp32"), (2, [33, 40], "BGK", "fp32"),
                                                       (3, [19, 14, 11], "MRT", "fp32"),
                                                       (2, [70, 66], "MRT", "bf16x3")])
def test_one_step_variant_matches_oracle(dim, n, collision, precision):
    _banner(f"one-step caputo dim={dim} n={n} {collision} {precision}")
    cfg = synth.small(dim, n, seed=43, collision=collision, with_source=True, c_wall=0.35, flux_form="caputo")
    S = synth.source(cfg)
    f0 = oracle.init(cfg, synth.initial_C(cfg))
    f0 = oracle.step(cfg, f0, 3, S=S)
    f32 = f0.astype(np.float32)
    ref = oracle.step(cfg, f32.astype(np.float64), 1, S=S.astype(np.float32).astype(np.float64))
    with _solver(cfg, precision) as s:
        s.set_f(torch.from_numpy(f32).cuda())
        s.set_source(S.astype(np.float32))
        s.step(1)
        got = s.get_f(device=False).astype(np.float64)
    scale = np.abs(f0).max()
    tol = 2e-6 if precision == "fp32" else 2e-5
    assert np.abs(got - ref).max() <= tol * scale


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_variant_keeps_uniform_field(precision):
    """u = 0, C0 = wall value = 0.7: the variant keeps C uniform (to FP32
    rounding), the form (Fg) does not."""
    cfg = synth.small(2, [96, 80], seed=12, u=[0.0, 0.0], c_wall=0.7)
    C0 = np.full(synth.shape(cfg), 0.7, np.float32)
    drift = {}
    for form in ("caputo", "rl"):
        with _solver(dict(cfg, flux_form=form), precision) as s:
            s.set_C(C0)
            s.step(100)
            drift[form] = float(np.abs(s.get_C(device=False).astype(np.float64) - 0.7).max())
    _banner(f"uniform drift after 100 steps: {drift}")
    assert drift["caputo"] <= 1e-5
    assert drift["rl"] > 1e-3


def test_variant_paper_exact_solution_setting():
    """The paper's check of the variant (Sec. 3.5): alpha = (1.7, 1.2),
    a = (0.3, 1.2), p = 1, D = Id, dx = 0.02, dt = 2.5e-5, profiles at
    t = 0.025 and 0.425 (17000 steps), source (SourceTerm_PS) and walls set
    every step, against the stored oracle run
    (tests/golden/make_caputo_reference.py) and the exact solution."""
    dt = 2.5e-5
    ref = np.load(os.path.join(GOLDEN, "ref_caputo_2d_51sq_dt2.5e-5.npz"))
    P = synth.CaputoPowerLawProblem(2, 51, dt)
    base = P.base.astype(np.float32)
    out = {}
    with _solver(P.cfg) as s:
        s.set_wall(base)
        s.set_C(base)
        for m in range(17000):
            S, Cw = P.schedule32(m)  # the FP32 fields the stored oracle run received
            s.set_source(S)
            s.set_wall(Cw)
            s.step(1)
            if m + 1 in (1000, 17000):
                out[m + 1] = s.get_C(device=False).astype(np.float64)
    for m, bound in ((1000, 1e-5), (17000, 1e-5)):
        C, R, ex = out[m], ref[f"C{m}"], P.exact(m * dt)
        par = _rel_l2(C, R)
        e_gpu, e_ora = np.abs(C - ex).max(), np.abs(R - ex).max()
        _banner(f"t = {m * dt:.3f}: gpu vs oracle rel L2 {par:.2e}; max |C - exact| gpu {e_gpu:.3e} oracle {e_ora:.3e}")
        assert par <= bound
        assert e_gpu <= 1.01 * e_ora + 2e-5


def test_flux_form_rejected_when_unknown():
    from paper_1706_09161_amd import LbmError, _lib

    cfg = synth.small(2, [16, 16], seed=3)
    with pytest.raises(KeyError):
        _solver(dict(cfg, flux_form="other"))
    import ctypes

    grid = _lib.lbm_grid()
    grid.dim = 2
    grid.n[0] = grid.n[1] = 16
    grid.n[2] = 1
    grid.dx = grid.dt = 1.0
    P = _lib.lbm_params()
    for mu in range(2):
        P.alpha[mu], P.p[mu], P.g[mu] = 1.5, 0.5, 1.0
    P.D[0] = P.D[3] = 0.1
    P.tau_free[0] = P.tau_free[1] = 1.0
    P.tau0 = 1.0
    P.collision = _lib.LBM_MRT
    P.flux_form = 2
    h = ctypes.c_void_p()
    rc = _lib.lib().lbm_fade_create(ctypes.byref(grid), 5, ctypes.byref(P), ctypes.byref(h))
    assert rc == _lib.LBM_EINVAL and not h.value
    with pytest.raises(LbmError):
        _lib.check(rc)
