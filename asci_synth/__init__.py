"""Seeded synthetic inputs for the ASCI determinant search.

This package draws integrals, determinant sets and coefficients.  It holds none of
the method's arithmetic (no matrix elements, no energies, no scores), so both the
CPU oracle and the HIP path may take their inputs from it.
"""
from .gen import (  # noqa: F401
    WORKLOADS,
    aufbau,
    coefficients,
    hilbert_dim,
    integrals,
    level_dets,
    make_case,
    uniform_dets,
    workload,
    batch_specs,
    small_batch_specs,
)
