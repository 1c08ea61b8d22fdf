"""The collide-stream kernel's march length (rows per wavefront in 2D, z
planes per workgroup in 3D, chosen from the grid size) changes only how the
nodes are dealt out, never what a node computes: runs with the march forced
through LBM_COLLIDE_ROWS to short, long, odd and grid-exceeding values give
the populations and C of the default launch bit for bit, on ragged grids
(partial 64-column strips, a last chunk shorter than the march), with and
without a source, in FP32 and split-BF16 and
with the space-dependent fields.  The same holds for the non-temporal output
stores that large grids use (forced here through LBM_COLLIDE_NT).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # dim, n, precision, source, space-dependent fields, march lengths
    (2, [203, 77], "fp32", True, False, [1, 2, 3, 4, 5, 8, 13, 16, 32, 100]),
    (2, [130, 45], "bf16x3", False, False, [1, 4, 7, 16]),
    (2, [97, 61], "fp32", True, True, [1, 3, 4, 9, 64]),
    (3, [70, 29, 23], "fp32", True, False, [1, 2, 3, 5, 8, 16, 64]),
    (3, [65, 13, 17], "bf16x3", True, False, [1, 4, 9]),
    (3, [33, 20, 9], "fp32", False, True, [1, 2, 7, 32]),
]


def _run(cfg, precision, S, D, Cw, steps):
    from paper_1706_09161_amd import LbmFade

    with LbmFade.from_config(cfg, precision=precision) as s:
        if D is not None:
            s.set_diffusion(D)
            s.set_wall(Cw)
        s.set_C(synth.initial_C(cfg).astype(np.float32))
        if S is not None:
            s.set_source(S)
        s.step(steps)
        return s.get_f(device=False).copy(), s.get_C(device=False).copy()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d-{'x'.join(map(str, c[1]))}-{c[2]}-S{int(c[3])}-V{int(c[4])}")
def test_march_length_does_not_change_the_result(case, monkeypatch):
    dim, n, precision, with_source, var, marches = case
    print(f"[gpu-march] dim={dim} n={n} {precision} src={with_source} var={var}", flush=True)
    cfg = synth.small(dim, n, seed=71, with_source=with_source, c_wall=0.1)
    S = synth.source(cfg)
    S = None if S is None else S.astype(np.float32)
    D = Cw = None
    if var:
        D = synth.random_tensor_field(cfg, seed=72).astype(np.float32)
        Cw = synth.random_wall_values(cfg, seed=73).astype(np.float32)
    steps = 13  # one replay of the 10-step graph and three single steps
    monkeypatch.delenv("LBM_COLLIDE_ROWS", raising=False)
    monkeypatch.setenv("LBM_COLLIDE_NT", "0")
    f_ref, C_ref = _run(cfg, precision, S, D, Cw, steps)
    assert np.isfinite(C_ref).all()
    runs = [(str(m), "0") for m in marches] + [("0", "1"), (str(marches[1]), "1")]
    for rows, nt in runs:
        monkeypatch.setenv("LBM_COLLIDE_ROWS", rows)
        monkeypatch.setenv("LBM_COLLIDE_NT", nt)
        assert os.environ["LBM_COLLIDE_NT"] == nt
        f, C = _run(cfg, precision, S, D, Cw, steps)
        assert np.array_equal(f.view(np.uint32), f_ref.view(np.uint32)), (rows, nt)
        assert np.array_equal(C.view(np.uint32), C_ref.view(np.uint32)), (rows, nt)
