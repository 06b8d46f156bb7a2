"""Combined-preconditioned conjugate gradients (ILU(0) + classical AMG) on MI355X.

The solver lives in libcpc.so (HIP kernels for gfx950 behind the C-ABI declared
in include/cpc.h); this package is its Python binding.
"""
from ._lib import (CPC_E_ARG, CPC_E_BREAKDOWN, CPC_E_DEVICE, CPC_E_MAXIT, CPC_E_NOMEM,  # noqa: F401
                   CPC_E_NOT_SPD, CPC_OK, CpcError, LIB_PATH, load)
from .solver import BatchSolver, Solver, options, setup_status, spgemm  # noqa: F401
