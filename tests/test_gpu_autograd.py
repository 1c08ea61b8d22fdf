"""The torch.autograd.Function over the library (paper_1706_09161_amd.autograd):
forward = lbm_fade_step, backward = lbm_fade_adjoint, both through the C ABI.

Gradients of a misfit loss taken with loss.backward() are compared with the
FP64 oracle adjoint fed the same output gradient gC = C_n - C_obs, at the
bounds of the adjoint's own oracle test (field gradients 1e-5 relative L2;
scalar gradients 1e-5 of the largest scalar gradient).  D, u and p are
float64 CUDA tensors that require grad; their gradients must come back with
the dtype and device of the inputs.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _opts(cfg):
    return dict(g=cfg["g"], dx=cfg["dx"], dt=cfg["dt"], tau_free=cfg["tau_free"], tau0=cfg["tau0"],
                c_wall=cfg["c_wall"], collision=cfg["collision"], flux_form=cfg.get("flux_form", "rl"))


CASES = [
    (2, [26, 21], "MRT", 0.0, "rl", 12, 5),
    (3, [11, 10, 9], "MRT", 0.0, "rl", 8, 3),
    (2, [24, 19], "MRT", 0.2, "caputo", 10, 4),   # Caputo-type flux (Sec. 3.5), non-zero walls
    (2, [23, 20], "BGK", 0.0, "rl", 9, 9),
]


@pytest.mark.parametrize("dim,n,collision,c_wall,flux_form,steps,K", CASES)
def test_fade_solve_backward_matches_oracle_adjoint(dim, n, collision, c_wall, flux_form, steps, K):
    from paper_1706_09161_amd.autograd import fade_solve

    print(f"[gpu-autograd] dim={dim} n={n} {collision} c_wall={c_wall} {flux_form} steps={steps} K={K}",
          flush=True)
    cfg = synth.small(dim, n, seed=91, collision=collision, with_source=True, c_wall=c_wall, flux_form=flux_form)
    C0 = synth.initial_C(cfg).astype(np.float32)
    S = synth.source(cfg).astype(np.float32)
    C_obs = np.random.default_rng(12).uniform(0.0, 0.5, synth.shape(cfg))
    dev = "cuda"
    C0t = torch.tensor(C0, dtype=torch.float64, device=dev, requires_grad=True)
    St = torch.tensor(S, dtype=torch.float64, device=dev, requires_grad=True)
    Dt = torch.tensor(cfg["D"], dtype=torch.float64, device=dev, requires_grad=True)
    ut = torch.tensor(cfg["u"], dtype=torch.float64, device=dev, requires_grad=True)
    pt = torch.tensor(cfg["p"], dtype=torch.float64, device=dev, requires_grad=True)
    Cn = fade_solve(C0t, St, Dt, ut, pt, alpha=cfg["alpha"], steps=steps, ckpt_every=K, **_opts(cfg))
    assert Cn.dtype == torch.float32 and Cn.is_cuda and tuple(Cn.shape) == synth.shape(cfg)
    obs = torch.tensor(C_obs, device=dev)
    loss = 0.5 * ((Cn.double() - obs) ** 2).sum()
    loss.backward()

    for t in (C0t, St, Dt, ut, pt):
        assert t.grad is not None and t.grad.dtype == torch.float64 and t.grad.is_cuda
        assert t.grad.shape == t.shape

    gC = (Cn.detach().double() - obs).cpu().numpy()
    ref = oracle.adjoint(cfg, C0.astype(np.float64), steps, gC.astype(np.float32).astype(np.float64),
                         S=S.astype(np.float64))
    ref_Cn = oracle.run(cfg, C0.astype(np.float64), steps, S=S.astype(np.float64))
    assert _rel(Cn.detach().cpu().numpy(), ref_Cn) < 1e-5
    assert _rel(C0t.grad.cpu().numpy(), ref["dC0"]) < 1e-5
    assert _rel(St.grad.cpu().numpy(), ref["dS"]) < 1e-5
    scale = max(np.abs(ref["D"]).max(), np.abs(ref["u"]).max(), np.abs(ref["p"]).max())
    got = {"D": Dt.grad.cpu().numpy(), "u": ut.grad.cpu().numpy(), "p": pt.grad.cpu().numpy()}
    for key in ("D", "u", "p"):
        assert np.abs(got[key] - ref[key]).max() <= 1e-5 * scale, (key, got[key], ref[key])


def test_tied_offdiagonal_parameter_gets_both_entries():
    """D built from three parameters (D_01 = D_10 tied): the parameter's
    gradient is the sum of both entries' derivatives, 2 x the symmetrised
    gradient the library reports."""
    from paper_1706_09161_amd.autograd import fade_solve

    cfg = synth.small(2, [22, 25], seed=92, with_source=False)
    steps = 7
    C0 = synth.initial_C(cfg).astype(np.float32)
    D = np.array(cfg["D"])
    prm = torch.tensor([D[0, 0], D[0, 1], D[1, 1]], dtype=torch.float64, device="cuda", requires_grad=True)
    Dt = torch.stack([torch.stack([prm[0], prm[1]]), torch.stack([prm[1], prm[2]])])
    C0t = torch.tensor(C0, device="cuda")
    gCn = np.random.default_rng(13).standard_normal(synth.shape(cfg))
    Cn = fade_solve(C0t, None, Dt, cfg["u"], cfg["p"], alpha=cfg["alpha"], steps=steps, ckpt_every=3,
                    **_opts(cfg))
    (Cn.double() * torch.tensor(gCn, device="cuda")).sum().backward()
    ref = oracle.adjoint(cfg, C0.astype(np.float64), steps, gCn.astype(np.float32).astype(np.float64))
    want = np.array([ref["D"][0, 0], 2 * ref["D"][0, 1], ref["D"][1, 1]])
    scale = np.abs(want).max()
    assert np.abs(prm.grad.cpu().numpy() - want).max() <= 1e-5 * scale, (prm.grad, want)


def test_inplace_change_of_an_input_is_caught():
    """C0 and S are saved with save_for_backward: changing one in place
    between forward and backward raises instead of replaying a wrong state."""
    from paper_1706_09161_amd.autograd import fade_solve

    cfg = synth.small(2, [20, 18], seed=93)
    leaf = torch.tensor(synth.initial_C(cfg).astype(np.float32), device="cuda", requires_grad=True)
    C0 = leaf * 1.0
    Cn = fade_solve(C0, None, cfg["D"], cfg["u"], cfg["p"], alpha=cfg["alpha"], steps=3, ckpt_every=2,
                    **_opts(cfg))
    with torch.no_grad():
        C0.add_(1.0)
    with pytest.raises(RuntimeError):
        Cn.sum().backward()
