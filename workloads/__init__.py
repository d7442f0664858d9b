"""Seeded synthetic inputs shared by the oracle's tests, the GPU tests and the benchmark.

Nothing here performs any step of the solver; it only builds matrices and
right-hand sides.
"""
from .q1hex import (  # noqa: F401
    CSR,
    AmplitudeFamily,
    KHAT,
    MASS_COEF,
    MHAT,
    OFFSETS,
    SourceFamily,
    amplitude_family,
    assemble,
    batch_systems,
    element_sigma,
    mass_1d,
    mass_matrix,
    multi_rhs,
    pattern_size,
    problem,
    q1hex,
    source_family,
    stiffness_1d,
)
