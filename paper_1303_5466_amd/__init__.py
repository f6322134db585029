"""MI355X-native recursive-skeletonisation direct solver for 2-D volume
integral equations (Corona, Martinsson, Zorin, "An O(N) Direct Solver for
Integral Equations on the Plane").

The solver itself is the native library librsd.so (C interface in
include/rsd.h, HIP kernels for gfx950 under csrc/); `rsd` is its ctypes
binding.  Importing this package does not require a GPU.
"""
from . import rsd  # noqa: F401
from .rsd import Factor, Plan, RsdError, detect_grid  # noqa: F401
