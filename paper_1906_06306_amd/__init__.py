"""MI355X (gfx950) relativistic particle-in-cell step of arXiv 1906.06306.

The method (Boris push with linear interpolation of Yee-staggered fields,
ZigZag charge-conserving deposit, FDTD field update) runs in hand-written HIP
kernels behind the C ABI declared in ``include/pic.h``; this package is the
Python binding (``_lib``), a small driver (``sim.PicSim``) and the build
script.  The library fails loudly if ``_build/libpic.so`` is missing.
"""
from ._lib import lib, LIB_PATH, PicError  # noqa: F401
from . import _lib as abi  # noqa: F401

__all__ = ["lib", "LIB_PATH", "PicError", "abi"]
