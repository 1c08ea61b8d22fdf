"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element on the same seeded inputs.

Tolerances (FP32 path): the fractional term accumulates n products in FP32,
so each value carries a relative error of order n * 2^-24 of
sum_k |K_jk| |C_k| at worst (sqrt(n) * 2^-24 typical); a full time step adds
FP32 rounding of order 2^-24 times the largest population magnitude; a run of
steps is held to the relative L2 bound 1e-5 of the FP32 target.

Split-BF16 path: every product K_jk C_k is formed from 2-term BF16 splits of
both operands with the lo*lo term dropped, a relative error of at most about
3 * 2^-17 per product (two representation remainders of 2^-17 and the dropped
term of 2^-16 * 2^-16), plus the FP32 accumulation; the bound used per value
is 2^-14 of sum_k |K_jk| |C_k|, and runs are held to relative L2 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(cfg, precision="fp32", **kw):
    from paper_1706_09161_amd import LbmFade

    return LbmFade.from_config(cfg, precision=precision, **kw)


def _rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def _banner(msg):
    print(f"[gpu-parity] {msg}", flush=True)


def _phi_scale(cfg, C, ref):
    """Magnitude a fractional-term value is formed from, sum_k |K_jk| |C_k|: for
    C >= 0 the value itself, since every product-rule weight is >= 0.  (The
    kernels sum the Toeplitz part over the interior columns and add the two
    boundary columns K[j][0] C(x_0) and K[j][N] C(x_N) whole, so no product is
    added and then cancelled.)"""
    return np.abs(ref)


PHI_CASES = [
    # (dim, n, alpha, p) -- several tiles plus ragged tails, one-sided and two-sided operators
    (2, [67, 45], [1.3, 1.8], [0.3, 0.8]),
    (2, [130, 97], [1.5, 1.2], [1.0, 0.0]),
    (2, [64, 64], [1.5, 1.5], [0.5, 0.5]),
    (2, [3, 5], [1.7, 1.1], [0.2, 0.9]),
    (2, [200, 131], [1.05, 1.95], [0.0, 1.0]),
    (3, [21, 18, 13], [1.5, 1.6, 1.8], [0.5, 0.2, 0.9]),
    (3, [40, 33, 35], [1.2, 1.9, 1.4], [1.0, 0.0, 0.6]),
    (2, [70, 41], [2.0, 1.01], [0.3, 0.7]),              # alpha = 2 (local) and near 1 (heaviest tails)
    (3, [17, 19, 21], [2.0, 2.0, 2.0], [0.5, 1.0, 0.0]),  # classical ADE on every axis
]


@pytest.mark.parametrize("precision", ["fp32", "fp32_simt"])
@pytest.mark.parametrize("case", PHI_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_fractional_term_matches_oracle(case, precision):
    dim, n, alpha, p = case
    _banner(f"phi {precision} dim={dim} n={n}")
    cfg = synth.small(dim, n, alpha=alpha, p=p, seed=31)
    cfg["g"] = [1.3, 0.7, 1.1][:dim]
    cfg["dx"] = 0.5
    rng = np.random.default_rng(17)
    C = rng.uniform(0.0, 1.0, synth.shape(cfg)).astype(np.float32)
    ref = oracle.phi(cfg, C.astype(np.float64))
    with _solver(cfg, precision) as s:
        got = s.apply_phi(torch.from_numpy(C).cuda()).cpu().numpy().astype(np.float64)
        got_host = s.apply_phi(C)
    assert np.array_equal(got, got_host.astype(np.float64))
    # C >= 0 and every weight >= 0: the scale is sum_k |K||C|
    nmax = max(n)
    scale = _phi_scale(cfg, C, ref)
    bound = 4 * nmax * 2.0**-24 * scale + 1e-30
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / (scale + 1e-30))
    assert _rel_l2(got, ref) < 2e-6


WALL_CASES = [
    (2, [96, 70], [1.4, 1.7], [1.0, 0.0]),
    (2, [64, 48], [1.2, 1.9], [0.3, 0.6]),
    (3, [24, 20, 18], [1.3, 1.6, 1.9], [0.0, 1.0, 0.5]),
]


@pytest.mark.parametrize("precision", ["fp32", "fp32_simt", "bf16x3"])
@pytest.mark.parametrize("case", WALL_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_wall_dominated_phi_within_its_own_magnitude(case, precision):
    """C = 1 on every wall and 1e-3 inside.  Each Phi value must be within
    eps-scaled sum_k |K_jk| |C_k| of the oracle, wall rows included: where the
    one-sided integral is empty (row 0 of I+, row N of I-) that magnitude is the
    other integral's alone, so a kernel that added s C(x_0) on the Toeplitz
    diagonal and cancelled it in the boundary column would fail here."""
    dim, n, alpha, p = case
    _banner(f"wall-dominated phi {precision} dim={dim} n={n}")
    cfg = synth.small(dim, n, alpha=alpha, p=p, seed=31)
    cfg["g"] = [0.9, 1.4, 1.2][:dim]
    cfg["dx"] = 0.25
    C = np.full(synth.shape(cfg), 1e-3, np.float32)
    for ax in range(dim):
        idx = [slice(None)] * dim
        idx[ax] = 0
        C[tuple(idx)] = 1.0
        idx[ax] = -1
        C[tuple(idx)] = 1.0
    ref = oracle.phi(cfg, C.astype(np.float64))
    with _solver(cfg, precision) as s:
        got = s.apply_phi(torch.from_numpy(C).cuda()).cpu().numpy().astype(np.float64)
    scale = _phi_scale(cfg, C, ref)  # C >= 0: sum_k |K||C| is the value itself
    rel = 4 * max(n) * 2.0**-24 if precision != "bf16x3" else 2.0**-14
    assert np.all(np.abs(got - ref) <= rel * scale + 1e-30), np.max(np.abs(got - ref) / (scale + 1e-30))


@pytest.mark.parametrize("case", PHI_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_fractional_term_bf16x3_matches_oracle(case):
    dim, n, alpha, p = case
    _banner(f"phi bf16x3 dim={dim} n={n}")
    cfg = synth.small(dim, n, alpha=alpha, p=p, seed=31)
    cfg["g"] = [1.3, 0.7, 1.1][:dim]
    cfg["dx"] = 0.5
    rng = np.random.default_rng(17)
    C = rng.uniform(0.0, 1.0, synth.shape(cfg)).astype(np.float32)
    ref = oracle.phi(cfg, C.astype(np.float64))
    with _solver(cfg, "bf16x3") as s:
        got = s.apply_phi(torch.from_numpy(C).cuda()).cpu().numpy().astype(np.float64)
    scale = _phi_scale(cfg, C, ref)
    assert np.all(np.abs(got - ref) <= 2.0**-14 * scale + 1e-30), np.max(np.abs(got - ref) / scale)
    err = _rel_l2(got, ref)
    print(f"[gpu-parity] bf16x3 phi rel L2 {err:.2e}", flush=True)
    assert err < 2e-5


TILE_CASES = [
    (2, [256, 96], [1.3, 1.7], [0.3, 0.8]),    # every axis a multiple of 16
    (2, [130, 97], [1.5, 1.2], [1.0, 0.0]),    # ragged, one-sided operators
    (3, [48, 33, 32], [1.5, 1.6, 1.8], [0.5, 0.2, 0.9]),
]


@pytest.mark.parametrize("choice", [f"fp32:{c}" for c in range(1, 17)] + [f"bf16x3:{c}" for c in range(1, 15)])
@pytest.mark.parametrize("case", TILE_CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}")
def test_every_tile_configuration(case, choice, monkeypatch):
    """Each explicitly selectable GEMM configuration (LBM_FP32_TILE / LBM_BF16_TILE)
    against the oracle, with the bounds of the default path.  The output buffer
    starts as NaN, so a tile that leaves an output unwritten fails."""
    precision, c = choice.split(":")
    dim, n, alpha, p = case
    _banner(f"phi {precision} tile {c} dim={dim} n={n}")
    monkeypatch.setenv("LBM_FP32_TILE" if precision == "fp32" else "LBM_BF16_TILE", c)
    cfg = synth.small(dim, n, alpha=alpha, p=p, seed=33)
    rng = np.random.default_rng(19)
    C = rng.uniform(0.0, 1.0, synth.shape(cfg)).astype(np.float32)
    ref = oracle.phi(cfg, C.astype(np.float64))
    with _solver(cfg, precision) as s:
        out = torch.full((dim,) + tuple(C.shape), float("nan"), device="cuda")
        s.apply_phi(torch.from_numpy(C).cuda(), out=out)
        got = out.cpu().numpy().astype(np.float64)
    assert np.isfinite(got).all(), int(np.count_nonzero(~np.isfinite(got)))
    rel = 4 * max(n) * 2.0**-24 if precision == "fp32" else 2.0**-14
    scale = _phi_scale(cfg, C, ref)
    assert np.all(np.abs(got - ref) <= rel * scale + 1e-30), np.max(np.abs(got - ref) / scale)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_apply_phi_on_the_solver_state(precision):
    """apply_phi(C = NULL) uses the solver's own C (and the split the collide
    kernel wrote): bitwise equal to applying it to a copy of C."""
    from paper_1706_09161_amd import LbmError, _lib

    cfg = synth.small(2, [96, 80], alpha=[1.4, 1.7], p=[0.3, 0.6], seed=34)
    with _solver(cfg, precision) as s:
        with pytest.raises(LbmError) as ei:
            s.apply_phi(None)
        assert ei.value.code == _lib.LBM_ESTATE
        s.set_C(synth.initial_C(cfg).astype(np.float32))
        s.step(3)
        a = s.apply_phi(None).cpu().numpy()
        b = s.apply_phi(s.get_C()).cpu().numpy()
    assert np.array_equal(a, b)


def test_bf16x3_split_is_not_plain_bf16():
    """The 3-term split must be far more accurate than a single BF16 rounding
    (2^-9 relative): guards against a silently dropped correction term."""
    cfg = synth.small(2, [256, 200], alpha=[1.3, 1.6], p=[0.4, 0.7], seed=32)
    rng = np.random.default_rng(18)
    C = rng.uniform(0.5, 1.0, synth.shape(cfg)).astype(np.float32)
    ref = oracle.phi(cfg, C.astype(np.float64))
    with _solver(cfg, "bf16x3") as s:
        got = s.apply_phi(C).astype(np.float64)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 2.0**-13


def test_end_to_end_small_workload_bf16x3():
    """The 64 x 64 workload (200 steps): split-BF16 GPU vs FP64 oracle, relative L2 <= 1e-4."""
    cfg = synth.config("c1_64sq")
    _banner("c1 end-to-end bf16x3")
    C0 = synth.initial_C(cfg)
    ref = oracle.run(cfg, C0.astype(np.float32).astype(np.float64), cfg["steps"])
    with _solver(cfg, "bf16x3") as s:
        s.set_C(C0.astype(np.float32))
        s.step(cfg["steps"])
        got = s.get_C(device=False)
    err = _rel_l2(got, ref)
    print(f"[gpu-parity] c1 bf16x3 rel L2 = {err:.3e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("dim,n,collision,with_source,c_wall", [
    (2, [37, 29], "MRT", False, 0.0),
    (2, [70, 66], "MRT", True, 0.25),
    (2, [33, 40], "BGK", True, 0.0),
    (2, [3, 3], "MRT", False, 0.5),
    (3, [19, 14, 11], "MRT", True, 0.0),
    (3, [9, 21, 16], "BGK", False, 0.3),
])
def test_one_step_matches_oracle(dim, n, collision, with_source, c_wall):
    """One full step from the same population state (set_f), every population of every node."""
    _banner(f"one-step dim={dim} n={n} {collision} src={with_source}")
    cfg = synth.small(dim, n, seed=41, collision=collision, with_source=with_source, c_wall=c_wall)
    S = synth.source(cfg)
    f0 = oracle.init(cfg, synth.initial_C(cfg))
    f0 = oracle.step(cfg, f0, 3, S=S)
    f32 = f0.astype(np.float32)
    ref = oracle.step(cfg, f32.astype(np.float64), 1, S=None if S is None else S.astype(np.float32).astype(np.float64))
    with _solver(cfg) as s:
        s.set_f(torch.from_numpy(f32).cuda())
        if S is not None:
            s.set_source(S.astype(np.float32))
        s.step(1)
        got = s.get_f(device=False).astype(np.float64)
        C = s.get_C(device=False).astype(np.float64)
    scale = np.abs(f0).max()
    assert np.abs(got - ref).max() <= 2e-6 * scale
    assert np.abs(C - ref.sum(axis=0)).max() <= 2e-6 * scale


def test_end_to_end_small_workload_fp32():
    """The 64 x 64 workload (200 steps, MRT): FP32 GPU vs FP64 oracle, relative L2 <= 1e-5."""
    cfg = synth.config("c1_64sq")
    _banner("c1 end-to-end")
    C0 = synth.initial_C(cfg)
    ref = oracle.run(cfg, C0.astype(np.float32).astype(np.float64), cfg["steps"])
    with _solver(cfg) as s:
        s.set_C(C0.astype(np.float32))
        s.step(cfg["steps"])
        got = s.get_C(device=False)
    err = _rel_l2(got, ref)
    print(f"[gpu-parity] c1 rel L2 = {err:.3e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("dim,n,collision,alpha", [(2, [75, 58], "MRT", None), (3, [24, 19, 21], "MRT", None),
                                                   (2, [41, 41], "BGK", None), (2, [50, 43], "MRT", [2.0, 2.0]),
                                                   (3, [20, 17, 15], "BGK", [2.0, 1.02, 2.0])])
def test_end_to_end_random_problems(dim, n, collision, alpha):
    cfg = synth.small(dim, n, seed=51, collision=collision, with_source=True, c_wall=0.1, alpha=alpha)
    _banner(f"end-to-end dim={dim} n={n} {collision}")
    C0 = synth.initial_C(cfg).astype(np.float32)
    S = synth.source(cfg).astype(np.float32)
    steps = 60
    ref = oracle.run(cfg, C0.astype(np.float64), steps, S=S.astype(np.float64))
    with _solver(cfg) as s:
        s.set_C(C0)
        s.set_source(torch.from_numpy(S).cuda())
        s.step(steps)
        got = s.get_C(device=False)
    assert _rel_l2(got, ref) <= 1e-5


def _sample_nodes(cfg, count, seed):
    """Random nodes plus every corner and a few wall nodes."""
    shape = synth.shape(cfg)
    nodes = synth.nodes(cfg)
    rng = np.random.default_rng(seed)
    pick = set(rng.integers(0, nodes, count).tolist())
    d = cfg["dim"]
    n = cfg["n"][:d]
    for corner in np.ndindex(*([2] * d)):
        c = [0 if b == 0 else n[mu] - 1 for mu, b in enumerate(corner)]
        idx = 0
        mul = 1
        for mu in range(d):
            idx += c[mu] * mul
            mul *= n[mu]
        pick.add(idx)
    for _ in range(8):  # wall nodes
        mu = int(rng.integers(0, d))
        c = [int(rng.integers(0, n[nu])) for nu in range(d)]
        c[mu] = 0 if rng.random() < 0.5 else n[mu] - 1
        idx = 0
        mul = 1
        for nu in range(d):
            idx += c[nu] * mul
            mul *= n[nu]
        pick.add(idx)
    return np.array(sorted(pick), dtype=np.int64)


@pytest.mark.parametrize("name,precision", [("c2_1024sq", "fp32"), ("c5_512sq_hidden", "fp32"),
                                            ("c2_1024sq", "bf16x3"), ("c4_4096sq", "fp32"),
                                            ("c4_4096sq", "bf16x3"), ("c3_256cube", "fp32")])
def test_full_size_sampled_step(name, precision):
    """At the benchmark's full size and launch configuration: after some GPU
    steps, one more GPU step is compared at sampled nodes with the oracle's
    step from the same populations."""
    cfg = synth.config(name)
    _banner(f"sampled full-size {name} {precision}")
    S = synth.source(cfg)
    S32 = None if S is None else S.astype(np.float32)
    with _solver(cfg, precision) as s:
        s.set_C(synth.initial_C(cfg).astype(np.float32))
        if S32 is not None:
            s.set_source(S32)
        s.step(20)
        f = s.get_f(device=False).astype(np.float64)
        s.step(1)
        f1 = s.get_f(device=False).reshape(2 * cfg["dim"] + 1, -1)
    nodes = _sample_nodes(cfg, 300, 7)
    ref = oracle.step_sampled(cfg, f, nodes, S=None if S32 is None else S32.astype(np.float64))
    got = f1[:, nodes].astype(np.float64)
    scale = np.abs(f).max()
    err = np.abs(got - ref).max() / scale
    print(f"[gpu-parity] {name} {precision} sampled max err / max|f| = {err:.3e}", flush=True)
    assert err <= (1e-5 if precision == "fp32" else 1e-4)


@pytest.mark.parametrize("base,n,precision", [("c2_1024sq", [12416, 12416], "fp32"),
                                              ("c3_256cube", [536, 536, 536], "fp32"),
                                              ("c3_256cube", [536, 536, 536], "bf16x3")])
def test_sampled_step_beyond_32bit_offsets(base, n, precision):
    """The largest grids: 7 fields of more than 2^30 floats each, so the
    kernels take their 64-bit offset variants (and the non-temporal stores of
    grids beyond the Infinity Cache).  One GPU step after 3 is compared at
    sampled nodes, the last node included, with the oracle's step from the
    same populations."""
    cfg = synth.config(base, n=n)
    nodes = synth.nodes(cfg)
    assert nodes * 7 * 4 >= 1 << 32
    _banner(f"64-bit offsets {base} n={n} {precision}")
    S = synth.source(cfg)
    S32 = None if S is None else S.astype(np.float32)
    with _solver(cfg, precision) as s:
        s.set_C(synth.initial_C(cfg).astype(np.float32))
        if S32 is not None:
            s.set_source(S32)
        s.step(3)
        f = s.get_f(device=False).astype(np.float64)
        s.step(1)
        f1 = s.get_f(device=False).reshape(2 * cfg["dim"] + 1, -1)
    pick = _sample_nodes(cfg, 200, 9)
    assert pick[-1] == nodes - 1
    ref = oracle.step_sampled(cfg, f, pick, S=None if S32 is None else S32.astype(np.float64))
    got = f1[:, pick].astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(f).max()
    print(f"[gpu-parity] 64-bit offsets {base} {precision}: sampled max err / max|f| = {err:.3e}", flush=True)
    assert err <= (1e-5 if precision == "fp32" else 1e-4)


@pytest.mark.parametrize("name", ["c4_4096sq", "c2_1024sq", "c3_256cube"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_full_size_phi_per_axis(name, precision):
    """The fractional term at full size, per axis (per alpha), on the state after
    20 steps: the GEMM launch of a step against the oracle's direct sums at
    sampled nodes.  Errors are measured against sum_k |K||C| of the same node,
    which is the oracle's Phi of |C| because every product-rule weight is
    >= 0 (C itself changes sign after a few steps, so Phi can cancel)."""
    cfg = synth.config(name)
    _banner(f"full-size phi per axis {name} {precision}")
    with _solver(cfg, precision) as s:
        s.set_C(synth.initial_C(cfg).astype(np.float32))
        s.step(20)
        C = s.get_C(device=False)
        got = s.apply_phi(None).cpu().numpy().reshape(cfg["dim"], -1)
    nodes = _sample_nodes(cfg, 400, 11)
    ref = oracle.phi_at(cfg, C.astype(np.float64), nodes)
    mag = oracle.phi_at(cfg, np.abs(C).astype(np.float64), nodes)  # sum_k |K||C|
    bound = 4 * max(cfg["n"]) * 2.0**-24 if precision == "fp32" else 2.0**-14
    for mu in range(cfg["dim"]):
        g, r = got[mu, nodes].astype(np.float64), ref[mu]
        rel = np.abs(g - r) / np.maximum(mag[mu], 1e-30)
        l2 = float(np.linalg.norm(g - r) / np.linalg.norm(r))
        print(f"[gpu-parity] {name} {precision} axis {mu} alpha={cfg['alpha'][mu]}: "
              f"rel L2 {l2:.2e}, max rel {rel.max():.2e}", flush=True)
        assert rel.max() <= bound


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_step_graph_matches_direct_launches(precision, monkeypatch):
    """lbm_fade_step replays a captured graph of 10 steps: every replay, with
    eager work (copies, apply_phi, a changed source) between replays, must give
    bitwise the populations of direct launches."""
    cfg = synth.small(2, [160, 96], alpha=[1.4, 1.7], p=[0.3, 0.8], seed=35, with_source=True)
    C0 = synth.initial_C(cfg).astype(np.float32)
    S = synth.source(cfg).astype(np.float32)

    def run(graph: bool):
        monkeypatch.setenv("LBM_STEP_GRAPH", "1" if graph else "0")
        out = []
        with _solver(cfg, precision) as s:
            s.set_C(C0)
            for n in (25, 13, 30, 10, 21):
                s.step(n)
                out.append(s.get_f(device=False))
                out.append(s.apply_phi(None).cpu().numpy())
                if n == 13:
                    s.set_source(S)  # the graph is captured again with the source
                if n == 10:
                    s.set_source(2 * S)  # same buffer, new values
        return out

    direct, graph = run(False), run(True)
    for k, (a, b) in enumerate(zip(direct, graph)):
        assert np.array_equal(a, b), k


def test_error_codes_on_device():
    from paper_1706_09161_amd import LbmError, _lib

    cfg = synth.small(2, [16, 16], seed=3)
    with _solver(cfg, nonfinite_check_every=1) as s:
        with pytest.raises(LbmError) as ei:
            s.step(1)
        assert ei.value.code == _lib.LBM_ESTATE
        C0 = np.ones((16, 16), np.float32)
        C0[5, 5] = np.nan
        s.set_C(C0)
        with pytest.raises(LbmError) as ei:
            s.step(3)
        assert ei.value.code == _lib.LBM_ENONFINITE
        with pytest.raises(ValueError):
            s.set_C(np.ones(10, np.float32))


def test_zero_steps_and_repeat_calls_are_consistent():
    cfg = synth.small(2, [50, 34], seed=8)
    C0 = synth.initial_C(cfg).astype(np.float32)
    with _solver(cfg) as s:
        s.set_C(C0)
        s.step(0)
        a = s.get_C(device=False)
        s.step(5)
        s.step(5)
        b = s.get_C(device=False)
        s.set_C(C0)
        s.step(10)
        c = s.get_C(device=False)
    ref0 = oracle.moment(cfg, oracle.init(cfg, C0.astype(np.float64)))
    assert np.abs(a - ref0).max() < 1e-5
    assert np.array_equal(b, c)  # deterministic


@pytest.mark.parametrize("name,precision,bound", [("c2_1024sq", "fp32", 1e-5), ("c2_1024sq", "bf16x3", 1e-4),
                                                  ("c3_256cube", "fp32", 1e-5), ("c3_256cube", "bf16x3", 1e-4),
                                                  ("c4_4096sq", "fp32", 1e-5), ("c4_4096sq", "bf16x3", 1e-4)])
def test_full_workload_against_stored_oracle(name, precision, bound):
    """The workloads at full size and full step count (1024^2 x 2000 steps;
    256^3 x 500 steps with its point source; 4096^2 x 1000 steps) against the
    stored FP64 oracle result on the sub-grid of every stride-th node
    (tests/golden/make_reference.py; 4, 8 and 8 here), and at the intermediate
    step counts the file also holds."""
    import glob
    import os

    from conftest import GOLDEN

    cfg = synth.config(name)
    hits = sorted(glob.glob(os.path.join(GOLDEN, f"ref_{name}_{cfg['steps']}steps_every*.npz")))
    if not hits:
        pytest.skip(f"no stored oracle result for {name} (tests/golden/make_reference.py writes it)")
    ref = np.load(hits[0])
    stride = int(ref["stride"])
    marks = [int(m) for m in ref["marks"]] if "marks" in ref.files else []
    _banner(f"full workload {name} {precision} (marks {marks})")
    S = synth.source(cfg)
    sl = (slice(None, None, stride),) * cfg["dim"]
    errs = {}
    with _solver(cfg, precision) as s:
        s.set_C(synth.initial_C(cfg).astype(np.float32))
        if S is not None:
            s.set_source(S.astype(np.float32))
        done = 0
        for m in marks + [cfg["steps"]]:
            s.step(m - done)
            done = m
            C = s.get_C(device=False)
            want = ref["C"] if m == cfg["steps"] else ref[f"C_at_{m}"]
            errs[m] = _rel_l2(C[sl], want)
    print(f"[gpu-parity] {name} {precision} rel L2 vs stored oracle by step: "
          + ", ".join(f"{m}: {e:.3e}" for m, e in errs.items()), flush=True)
    for m, e in errs.items():
        assert e <= bound, (m, e)


def test_4096_mfma_sums_beat_the_plain_fp32_sums():
    """At 4096^2 the step's FP32 error is set by how the fractional term is
    summed: to the right of a pulse the one-sided gamma = 0.8 integral makes
    Phi ~ 4 where C ~ 1e-4, and the collision takes second differences of Phi.
    The MFMA kernel spreads every pulse over eight FP32 running sums (k groups
    dealt round robin to four wavefronts, two accumulator sets each); the
    plain SIMT kernel sums each output in one.  At the stored intermediate
    step counts the MFMA path must be closer to the FP64 oracle than the SIMT
    path (a summation mistake would show against it), and the split-BF16 path
    inside 1e-4."""
    import glob
    import os

    from conftest import GOLDEN

    cfg = synth.config("c4_4096sq")
    hits = sorted(glob.glob(os.path.join(GOLDEN, f"ref_c4_4096sq_{cfg['steps']}steps_every*.npz")))
    if not hits:
        pytest.skip("no stored oracle result for c4_4096sq")
    ref = np.load(hits[0])
    stride = int(ref["stride"])
    marks = [int(m) for m in ref["marks"]]
    assert marks, "the 4096^2 reference holds no intermediate step counts"
    sl = (slice(None, None, stride),) * 2
    errs = {}
    for precision in ("fp32", "fp32_simt", "bf16x3"):
        _banner(f"4096^2 {precision} to steps {marks}")
        with _solver(cfg, precision) as s:
            s.set_C(synth.initial_C(cfg).astype(np.float32))
            done = 0
            for m in marks:
                s.step(m - done)
                done = m
                errs[(precision, m)] = _rel_l2(s.get_C(device=False)[sl], ref[f"C_at_{m}"])
    print("[gpu-parity] 4096^2 rel L2 by (path, step): "
          + ", ".join(f"{k}: {v:.3e}" for k, v in errs.items()), flush=True)
    for m in marks:
        assert errs[("fp32", m)] < errs[("fp32_simt", m)], m
        assert errs[("fp32", m)] <= 1e-5, m
        assert errs[("bf16x3", m)] <= 1e-4, m
