"""MI355X-native canonical density-matrix perturbation theory.

The computation lives in libdmpt.so (HIP, gfx950; C ABI in include/dmpt.h).
This package only marshals torch tensors into that library.
"""
from ._lib import load, Options, Stats, STATUS_NAMES, LIB_PATH  # noqa: F401
from .api import Context, DMPTError, options  # noqa: F401

__all__ = ["Context", "DMPTError", "options", "load", "LIB_PATH"]
