"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its struct layouts agree with the C compiler's.  No
compute calls (runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "lbm_fade.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"LBM_API\s+[\w\s\*]*?\b(lbm_(?:fade|rw)_\w+)\s*\(", text)))


def test_header_declares_the_abi():
    names = _declared()
    for required in ("lbm_fade_create", "lbm_fade_step", "lbm_fade_get_C", "lbm_fade_adjoint"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1706_09161_amd import _lib

    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTED) == _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(set(re.findall(r" T (lbm_(?:fade|rw)_\w+)", out)))
    assert exported == _declared()


def test_struct_layout_matches_c_compiler(tmp_path):
    from paper_1706_09161_amd import _lib

    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lbm_fade.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(lbm_grid), offsetof(lbm_grid, dx),"
        " sizeof(lbm_params), offsetof(lbm_params, collision), sizeof(lbm_grads), offsetof(lbm_grads, dp));"
        "printf(\"%zu %zu %zu\\n\", sizeof(lbm_rw_params), offsetof(lbm_rw_params, dt), offsetof(lbm_rw_params, seed));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    expect = [ctypes.sizeof(_lib.lbm_grid), _lib.lbm_grid.dx.offset, ctypes.sizeof(_lib.lbm_params),
              _lib.lbm_params.collision.offset, ctypes.sizeof(_lib.lbm_grads), _lib.lbm_grads.dp.offset,
              ctypes.sizeof(_lib.lbm_rw_params), _lib.lbm_rw_params.dt.offset, _lib.lbm_rw_params.seed.offset]
    assert vals == expect


def test_version_string():
    from paper_1706_09161_amd import version

    assert "gfx950" in version()


def test_null_arguments_rejected_without_device():
    """Argument checks that return before any device call."""
    from paper_1706_09161_amd import _lib

    L = _lib.lib()
    assert L.lbm_fade_create(None, 5, None, None) == _lib.LBM_EINVAL
    h = ctypes.c_void_p()
    assert L.lbm_fade_create(None, 5, None, ctypes.byref(h)) == _lib.LBM_EINVAL
    assert h.value is None
    assert L.lbm_fade_step(None, 1, None) == _lib.LBM_EINVAL
    assert b"null" in L.lbm_fade_last_error()
    L.lbm_fade_destroy(None)  # NULL-safe


def test_invalid_parameters_rejected_before_device_use():
    from paper_1706_09161_amd import _lib

    L = _lib.lib()
    g = _lib.lbm_grid()
    g.dim, g.dx, g.dt = 2, 1.0, 1.0
    g.n[0], g.n[1], g.n[2] = 16, 16, 1
    P = _lib.lbm_params()
    for mu in range(2):
        P.alpha[mu], P.p[mu], P.g[mu] = 1.5, 0.5, 1.0
    P.D[0], P.D[3] = 0.1, 0.1
    P.tau_free[0] = P.tau_free[1] = 1.0
    P.tau0 = 1.0
    P.collision = _lib.LBM_MRT
    h = ctypes.c_void_p()
    bad = []
    for field, idx, val in [("alpha", 0, 1.0), ("alpha", 1, 2.5), ("p", 0, -0.1), ("g", 1, 0.0),
                            ("tau_free", 0, 0.5), ("D", 1, 0.5)]:
        saved = getattr(P, field)[idx]
        getattr(P, field)[idx] = val
        if field == "D":
            P.D[2] = val  # symmetric but not positive definite
        bad.append(L.lbm_fade_create(ctypes.byref(g), 5, ctypes.byref(P), ctypes.byref(h)))
        getattr(P, field)[idx] = saved
        if field == "D":
            P.D[2] = 0.0
    assert all(rc == _lib.LBM_EINVAL for rc in bad), bad
    assert L.lbm_fade_create(ctypes.byref(g), 7, ctypes.byref(P), ctypes.byref(h)) == _lib.LBM_EINVAL
    P.collision = _lib.LBM_BGK
    P.D[3] = 0.2  # anisotropic D is not allowed with BGK
    assert L.lbm_fade_create(ctypes.byref(g), 5, ctypes.byref(P), ctypes.byref(h)) == _lib.LBM_EINVAL


def test_random_walk_parameters_rejected_before_device_use():
    from paper_1706_09161_amd import _lib

    L = _lib.lib()
    P = _lib.lbm_rw_params()
    P.dim = 2
    for mu in range(2):
        P.lo[mu], P.hi[mu], P.alpha[mu], P.p[mu], P.D[mu], P.g[mu] = 0.0, 1.0, 1.5, 0.5, 0.1, 1.0
    P.dt = 1e-3
    bad = []
    for field, value in (("dim", 4), ("dt", 0.0)):
        Q = _lib.lbm_rw_params.from_buffer_copy(P)
        setattr(Q, field, value)
        bad.append(Q)
    for field, value in (("alpha", 1.0), ("alpha", 2.5), ("p", 1.5), ("D", -1.0), ("g", 0.0), ("hi", 0.0)):
        Q = _lib.lbm_rw_params.from_buffer_copy(P)
        getattr(Q, field)[1] = value
        bad.append(Q)
    c = (ctypes.c_double * 3)(0.5, 0.5, 0.0)
    for Q in bad:
        assert L.lbm_rw_init_gaussian(ctypes.byref(Q), c, 0.1, 10, 0, None, None, None) == _lib.LBM_EINVAL
        assert L.lbm_rw_walk(ctypes.byref(Q), None, None, 10, 0, 0, 5, None) == _lib.LBM_EINVAL
    assert L.lbm_rw_walk(ctypes.byref(P), None, None, 10, 0, 0, 5, None) == _lib.LBM_EINVAL  # null buffers
    assert L.lbm_rw_walk(ctypes.byref(P), None, None, 10, 0, 2**32 - 3, 5, None) == _lib.LBM_EINVAL  # step range
    assert b"null" in L.lbm_fade_last_error() or b"step" in L.lbm_fade_last_error()
    assert L.lbm_rw_walk(ctypes.byref(P), None, None, 0, 0, 0, 5, None) == _lib.LBM_OK  # nothing to do
