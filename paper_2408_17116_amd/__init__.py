"""MI355X-native H-matrix direct solver for the Chebyshev-based Nystrom BIE.

The solver lives in libcbie.so (hand-written HIP for gfx950, C-ABI declared in
include/cbie.h); `cbie` is its thin ctypes binding.
"""
from . import cbie  # noqa: F401
