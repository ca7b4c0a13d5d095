"""Seeded, synthetic inputs shared by the oracle, the tests, the bench and the
Python binding.

This package holds the *inputs* of the method only: the moment sequence of the
weight exp(-x**beta) on [0, inf) (Section 2, eq. ``moments``), its derivative in
beta, and the recipes that pick (beta, N, precision) for the workloads.  It holds
none of the method's arithmetic (no scaling, no factorisation, no rounding of
matrix entries): the oracle and the HIP library each do that on their own.
"""

from .moments import (  # noqa: F401
    Dyadic,
    moments,
    dmoments_dbeta,
    exact_moment_fraction,
    is_exact_beta,
    trace_log2,
    precision_rule,
    batch_configs,
    pack_limbs,
    unpack_limbs,
)
