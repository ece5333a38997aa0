"""MI355X-native split second-order Godunov sweep for the 2D Euler equations.

The compute path is libhydro.so (hand-written HIP kernels for gfx950 behind the
C ABI of include/hydro.h); this package is its thin Python binding, plus the
seeded input generators (``inputs``).  Importing it does not touch the GPU.
"""
from ._lib import HydroError, LIB_PATH  # noqa: F401

__all__ = ["HydroError", "LIB_PATH"]
