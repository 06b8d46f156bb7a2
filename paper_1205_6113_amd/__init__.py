"""Combined-preconditioned conjugate gradients (ILU(0) + classical AMG) on MI355X.

The solver lives in libcpc.so (HIP kernels for gfx950 behind the C-ABI declared
in include/cpc.h); this package is its Python binding.
"""
from ._lib import CpcError, LIB_PATH, load  # noqa: F401
from .solver import BatchSolver, Solver, options, setup_status  # noqa: F401
