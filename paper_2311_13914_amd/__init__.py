"""MI355X (gfx950) AMG-preconditioned CG for the decoupled Bidomain step.

The solve path lives in the HIP library libbidomain.so (C ABI: include/bidomain.h);
this package holds its sources (csrc/), the build script and the ctypes binding.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import load, LIB_PATH, exported_symbols, BidomainError  # noqa: F401
