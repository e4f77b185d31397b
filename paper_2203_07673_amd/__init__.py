"""Local FusedMM (SDDMM -> SpMM) for AMD Instinct MI355X.

The compute lives in libfmm.so (hand-written HIP for gfx950, C ABI in
include/fmm.h); this package is its Python binding.
"""
from ._capi import FmmError, load as _load_library  # noqa: F401
from .fusedmm import (  # noqa: F401
    NOALLOC_SCRATCH_BYTES,
    BatchPlan,
    Pattern,
    als_residual,
    als_sweep,
    cg_lines,
    device_info,
    dtype_code,
    fusedmm_a,
    fusedmm_a_backward_raw,
    fusedmm_a_backward_values_raw,
    fusedmm_a_noalloc_raw,
    fusedmm_a_raw,
    fusedmm_b,
    fusedmm_b_backward_raw,
    fusedmm_b_backward_values_raw,
    fusedmm_b_raw,
    gat,
    gat_autotune,
    gat_backward,
    gat_edge_values,
    gat_forward,
    gat_forward_unfused,
    gat_scores,
    sddmm,
    sddmm_raw,
    set_tuning,
    spmm_a,
    spmm_a_raw,
    spmm_b,
    spmm_b_raw,
    stream_copy,
    stream_gather,
    stream_read,
    to_bf16,
)

__version__ = "0.1.0"
