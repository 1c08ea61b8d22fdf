"""ctypes declarations of the C ABI in include/lbm_fade.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmfade.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_D2Q5, LBM_D3Q7 = 5, 7
LBM_BGK, LBM_MRT = 0, 1
LBM_FP32, LBM_BF16X3, LBM_FP32_SIMT = 0, 1, 2
LBM_FLUX_RL, LBM_FLUX_CAPUTO = 0, 1
LBM_NOALLOC_SCRATCH_BYTES = 16 << 20

ERROR_NAMES = {LBM_EINVAL: "LBM_EINVAL", LBM_ENOMEM: "LBM_ENOMEM", LBM_EDEVICE: "LBM_EDEVICE",
               LBM_ENONFINITE: "LBM_ENONFINITE", LBM_ESTATE: "LBM_ESTATE"}

# Every symbol include/lbm_fade.h declares.
EXPORTED = ["lbm_fade_create", "lbm_fade_destroy", "lbm_fade_set_C", "lbm_fade_set_source", "lbm_fade_set_diffusion",
            "lbm_fade_set_wall", "lbm_fade_step",
            "lbm_fade_get_C", "lbm_fade_get_f", "lbm_fade_set_f", "lbm_fade_apply_phi", "lbm_fade_apply_phi_noalloc",
            "lbm_fade_adjoint",
            "lbm_fade_last_error", "lbm_fade_version", "lbm_rw_init_gaussian", "lbm_rw_walk", "lbm_rw_histogram"]


class lbm_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double), ("dt", ctypes.c_double)]


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double * 3),
        ("p", ctypes.c_double * 3),
        ("g", ctypes.c_double * 3),
        ("D", ctypes.c_double * 9),
        ("u", ctypes.c_double * 3),
        ("tau_free", ctypes.c_double * 4),
        ("tau0", ctypes.c_double),
        ("c_wall", ctypes.c_double),
        ("collision", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("nonfinite_check_every", ctypes.c_int32),
        ("flux_form", ctypes.c_int32),
    ]


class lbm_rw_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("alpha", ctypes.c_double * 3),
        ("p", ctypes.c_double * 3),
        ("D", ctypes.c_double * 3),
        ("g", ctypes.c_double * 3),
        ("u", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class lbm_grads(ctypes.Structure):
    _fields_ = [("dD", ctypes.c_double * 9), ("du", ctypes.c_double * 3), ("dp", ctypes.c_double * 3)]


class LbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblbmfade.so; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1706_09161_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    vp = ctypes.c_void_p
    fp = ctypes.c_void_p  # float* (host or device address)
    sig = {
        "lbm_fade_create": (ctypes.c_int, [ctypes.POINTER(lbm_grid), ctypes.c_int32, ctypes.POINTER(lbm_params),
                                           ctypes.POINTER(ctypes.c_void_p)]),
        "lbm_fade_destroy": (None, [H]),
        "lbm_fade_set_C": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_set_source": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_set_diffusion": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_set_wall": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_step": (ctypes.c_int, [H, ctypes.c_int64, vp]),
        "lbm_fade_get_C": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_get_f": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_set_f": (ctypes.c_int, [H, fp, ctypes.c_int32, vp]),
        "lbm_fade_apply_phi": (ctypes.c_int, [H, fp, fp, ctypes.c_int32, vp]),
        "lbm_fade_apply_phi_noalloc": (ctypes.c_int, [ctypes.POINTER(lbm_grid), ctypes.POINTER(lbm_params), fp, fp,
                                                      vp]),
        "lbm_fade_adjoint": (ctypes.c_int, [H, ctypes.c_int64, ctypes.c_int32, fp, ctypes.c_int32,
                                            ctypes.POINTER(lbm_grads), fp, fp, vp]),
        "lbm_rw_init_gaussian": (ctypes.c_int, [ctypes.POINTER(lbm_rw_params), ctypes.POINTER(ctypes.c_double),
                                                ctypes.c_double, ctypes.c_int64, ctypes.c_int64, vp, vp, vp]),
        "lbm_rw_walk": (ctypes.c_int, [ctypes.POINTER(lbm_rw_params), vp, vp, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64, vp]),
        "lbm_rw_histogram": (ctypes.c_int, [ctypes.POINTER(lbm_rw_params), vp, vp, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.c_double, vp, vp]),
        "lbm_fade_last_error": (ctypes.c_char_p, []),
        "lbm_fade_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_fade_last_error().decode())
