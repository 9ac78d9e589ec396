"""MI355X-native iterated stencil sweeps with temporal computation folding.

The compute path is libstencil.so (hand-written HIP for gfx950) behind the C
ABI in include/stencil.h; this package is its thin ctypes binding.  Importing
it fails loudly if the library has not been built.
"""

from .binding import *  # noqa: F401,F403
from .binding import Plan, BatchedRun, StencilError, make_grid, lib, LIB_PATH, EXPORTS  # noqa: F401
