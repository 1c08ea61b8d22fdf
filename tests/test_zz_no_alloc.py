"""lbm_fade_apply_phi_noalloc (the handle-free, allocation-free fractional
operator) through the C ABI, against lbm_fade_apply_phi of a handle created
with the same grid and parameters: same weights, same kernels, so the two
agree bit for bit; and against the FP64 oracle at the FP32 / split-BF16
bounds of the other parity tests.  Two calls in a row (the second on a
smaller grid) reuse the library's one device scratch array."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _handle_phi(cfg, precision, C):
    from paper_1706_09161_amd import LbmFade

    with LbmFade.from_config(cfg, precision=precision) as s:
        out = s.apply_phi(C)
        torch.cuda.synchronize()
        return out.cpu().numpy()


PAIRS = [
    # (first grid, second smaller grid): several tiles plus ragged tails, then fewer
    ((2, [150, 97]), (2, [61, 40])),
    ((3, [33, 20, 17]), (3, [19, 14, 11])),
    ((2, [257, 129]), (3, [9, 8, 7])),
]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp32_simt"])
@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: f"{p[0][0]}d{p[0][1]}-then-{p[1][0]}d{p[1][1]}")
def test_noalloc_matches_handle_twice_in_a_row(precision, pair):
    from paper_1706_09161_amd import apply_phi_noalloc
    from paper_1706_09161_amd.solver import config_kwargs

    print(f"[gpu-noalloc] {precision} {pair}", flush=True)
    for k, (dim, n) in enumerate(pair):
        cfg = synth.small(dim, n, seed=120 + k, c_wall=0.1 * k, flux_form="caputo" if k else "rl")
        C = np.random.default_rng(7 + k).uniform(0.0, 1.0, synth.shape(cfg)).astype(np.float32)
        Ct = torch.from_numpy(C).cuda()
        got = apply_phi_noalloc(dim, n, Ct, precision=precision, **config_kwargs(cfg))
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        want = _handle_phi(cfg, precision, Ct)
        assert got.shape == want.shape == (dim,) + synth.shape(cfg)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (k, np.abs(got - want).max())
        ref = oracle.phi(cfg, C.astype(np.float64))
        bound = 1e-4 if precision == "bf16x3" else 1e-5
        for mu in range(dim):
            assert _rel(got[mu], ref[mu]) <= bound, (k, mu, _rel(got[mu], ref[mu]))


def test_noalloc_calls_queued_on_one_stream():
    """Three calls queued on one stream without waiting for the kernels: each
    call's upload is ordered after the previous call's kernels, so every
    result is right."""
    from paper_1706_09161_amd import apply_phi_noalloc
    from paper_1706_09161_amd.solver import config_kwargs

    cases = [(2, [130, 70]), (2, [64, 33]), (3, [21, 17, 12])]
    outs, want = [], []
    for k, (dim, n) in enumerate(cases):
        cfg = synth.small(dim, n, seed=130 + k)
        Ct = torch.from_numpy(np.random.default_rng(30 + k).uniform(0, 1, synth.shape(cfg)).astype(np.float32)).cuda()
        outs.append(apply_phi_noalloc(dim, n, Ct, **config_kwargs(cfg)))
        want.append((cfg, Ct))
    torch.cuda.synchronize()
    for out, (cfg, Ct) in zip(outs, want):
        ref = _handle_phi(cfg, "fp32", Ct)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_noalloc_rejects_grids_beyond_its_scratch():
    """A grid whose operator data exceed the fixed scratch (about 40 bytes per
    node of each axis) is refused with LBM_EINVAL before any device work
    (host-side check), naming the sizes; a large grid within it runs."""
    from paper_1706_09161_amd import LbmError, _lib, apply_phi_noalloc
    from paper_1706_09161_amd.solver import config_kwargs

    cfg = synth.small(2, [450000, 3], seed=140)  # ~18 MB of operator data along x
    Ct = torch.zeros((3, 450000), device="cuda")
    with pytest.raises(LbmError) as ei:
        apply_phi_noalloc(2, [450000, 3], Ct, **config_kwargs(cfg))
    assert ei.value.code == _lib.LBM_EINVAL and "scratch" in str(ei.value)
    cfg = synth.small(2, [2100, 2100], seed=141)
    Ct = torch.zeros((2100, 2100), device="cuda")
    for precision in ("fp32", "bf16x3"):
        out = apply_phi_noalloc(2, [2100, 2100], Ct, precision=precision, **config_kwargs(cfg))
        torch.cuda.synchronize()
        assert not torch.any(out).item()
