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
    return sorted(set(re.findall(r"LBM_API\s+[\w\s\*]*?\b(lbm_fade_\w+)\s*\(", text)))


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
    exported = sorted(set(re.findall(r" T (lbm_fade_\w+)", out)))
    assert exported == _declared()


def test_struct_layout_matches_c_compiler(tmp_path):
    from paper_1706_09161_amd import _lib

    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lbm_fade.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(lbm_grid), offsetof(lbm_grid, dx),"
        " sizeof(lbm_params), offsetof(lbm_params, collision), sizeof(lbm_grads), offsetof(lbm_grads, dp));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    expect = [ctypes.sizeof(_lib.lbm_grid), _lib.lbm_grid.dx.offset, ctypes.sizeof(_lib.lbm_params),
              _lib.lbm_params.collision.offset, ctypes.sizeof(_lib.lbm_grads), _lib.lbm_grads.dp.offset]
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
