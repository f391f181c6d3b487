"""MI355X (gfx950) threshold random hyperbolic graph generation.

The band-based neighbour query of von Looz et al. (HPEC 2016, Algorithm 1)
as hand-written HIP kernels behind the C ABI in include/rhg.h; ``rhg`` is the
Python binding (ctypes, argument marshalling only).
"""
from . import rhg  # noqa: F401

__all__ = ["rhg"]
