"""Oracle for the combined-preconditioned CG method (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package. It shares no code with the product library.
"""
from .oracle import (  # noqa: F401
    OR_OK, OR_E_ARG, OR_E_NOT_SPD, OR_E_BREAKDOWN, OR_E_MAXIT, OR_E_NOMEM,
    PREC_COMBINED, PREC_AMG, PREC_ILU, PREC_ADDITIVE, PREC_NONE,
    OP_VCYCLE, OP_FGS, OP_BGS, OP_COMBINED_GS, OP_COMBINED_SWAP, PREC_AMG_ILU, PREC_BBAR,
    build_oracle, Hierarchy, ilu0, validate, rs_split, tpfa_logk_gradient, misfit_gradient,
)
