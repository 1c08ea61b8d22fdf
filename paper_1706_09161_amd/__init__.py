"""MI355X (gfx950) lattice Boltzmann step for the space-fractional
advection-diffusion equation (Cartalade, Younsi, Neel, arXiv:1706.09161).

The compute path is liblbmfade.so (hand-written HIP, C ABI in
include/lbm_fade.h); this package only marshals arguments to it.
"""
from .solver import LbmFade, apply_phi_noalloc, version  # noqa: F401
from ._lib import LbmError, LIB_PATH  # noqa: F401

__all__ = ["LbmFade", "LbmError", "apply_phi_noalloc", "version", "LIB_PATH"]
