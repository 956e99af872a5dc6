"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package draws parameter sets, bitstrings, coherent amplitudes and per-mode
observable matrices from fixed seeds.  It performs none of the method's
arithmetic: no master-equation terms, no generating-function scaling, no
time stepping.  Both the CPU oracle and the HIP path consume what it returns.
"""

from .workloads import (  # noqa: F401
    TWO_PI,
    System,
    Workload,
    single_mode_c0,
    seeded_system,
    three_mode_c1,
    batch_c2,
    grad_c3,
    grad_c3b,
    large_c4,
    projector_factors,
    parity_factors,
    quadrature_factors,
    annihilation_factors,
    table1_network,
    fock_state,
    coherent_state,
    random_system,
    random_product_operator,
    random_sparse_operator,
    random_normal_coeffs,
)
