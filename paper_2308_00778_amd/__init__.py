"""MI355X-native LSQR for the Gaia AVU-GSR astrometric system.

The computation lives in liblsqr.so (HIP kernels for gfx950 behind the C ABI
of include/lsqr.h); this package only marshals torch tensors into it.
"""
from .lsqr import (LSQR_E_HIP, LSQR_E_INVALID, LSQR_E_NOMEM, LSQR_E_STATE,
                   LSQR_E_UNSUPPORTED, LSQR_OK, SYMBOLS, Info, LsqrError, LsqrSystem,
                   load_library)

__all__ = ["LsqrSystem", "LsqrError", "Info", "load_library", "SYMBOLS", "LSQR_OK",
           "LSQR_E_INVALID", "LSQR_E_HIP", "LSQR_E_NOMEM", "LSQR_E_STATE", "LSQR_E_UNSUPPORTED"]
