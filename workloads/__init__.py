"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds only random-input construction (sparsity patterns, dense
factor matrices, value draws).  It contains none of the FusedMM arithmetic, so
both the GPU path and the CPU oracle may consume what it produces.
"""

from .generators import (  # noqa: F401
    CsrPattern,
    er_exact_degree,
    rmat,
    dense_normal,
    batch_er,
    tiny_case,
    workload,
    content_hash,
)
