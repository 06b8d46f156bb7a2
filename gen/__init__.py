"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package draws random fields and assembles two-point-flux pressure matrices
on Cartesian grids. It holds none of the solver's arithmetic (no PCG, no
preconditioner, no factorisation, no coarsening).
"""
from .tpfa import (  # noqa: F401
    Problem,
    correlated_field,
    channel_facies,
    tpfa_system,
    config1,
    config2,
    config3,
    config4,
    config4_sizes,
    config5,
    scaled_config,
    csr_to_dense,
)
from .wide import hub_chain, wide_band  # noqa: F401,E402
