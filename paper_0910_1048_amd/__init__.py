"""MI355X-native sign(H_W) b for the Wilson kernel at nonzero chemical potential.

The numerical work runs in libsgn.so (hand-written HIP for gfx950 behind the
C ABI declared in include/sgn.h); this package is its ctypes binding.
"""
from .binding import *  # noqa: F401,F403
from .binding import lib, LIB_PATH, HEADER, exported_symbols, SgnError, Context, Lattice, Deflation  # noqa: F401
