"""ctypes binding of libfmm.so: one Python function per C entry point, same names.

Argument marshalling only.  Every computation runs in the HIP library; if the
library is missing or was built for another GPU the import fails loudly (there is
no CPU fallback).  torch is imported first so that the HIP runtime torch ships is
the one libfmm.so binds to (both carry the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime before libfmm.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm.so")

FMM_OK = 0
FMM_F32, FMM_BF16, FMM_F64 = 0, 1, 2
FMM_CSR, FMM_CSC = 0, 1
FMM_FUSED, FMM_UNFUSED = 0, 1
FMM_DC_BF16 = 2
FMM_VARIANT_AUTO, FMM_VARIANT_DEEP, FMM_VARIANT_MEDIUM, FMM_VARIANT_SHALLOW = 0, 1, 2, 3
(FMM_OP_SDDMM, FMM_OP_SPMM_A, FMM_OP_SPMM_B, FMM_OP_FUSEDMM_A, FMM_OP_FUSEDMM_B, FMM_OP_FUSEDMM_A_BWD,
 FMM_OP_FUSEDMM_B_BWD, FMM_OP_SDDMM_BWD, FMM_OP_SPMM_A_BWD, FMM_OP_SPMM_B_BWD,
 FMM_OP_FUSEDMM_A_BWD_VALUES, FMM_OP_FUSEDMM_B_BWD_VALUES) = range(12)

STATUS_NAMES = {0: "FMM_OK", -1: "FMM_ERR_NULL", -2: "FMM_ERR_DIM", -3: "FMM_ERR_DTYPE", -4: "FMM_ERR_ORIENT",
                -5: "FMM_ERR_INDEX", -6: "FMM_ERR_NONCANONICAL", -7: "FMM_ERR_WORKSPACE",
                -8: "FMM_ERR_UNSUPPORTED", -9: "FMM_ERR_HIP", -10: "FMM_ERR_STATE"}
FMM_BATCH_FWD, FMM_BATCH_BWD, FMM_BATCH_DC_BF16 = 1, 2, 4
FMM_GAT_SOFTMAX = 1


class fmm_sparse(ctypes.Structure):
    _fields_ = [
        ("orient", ctypes.c_int32),
        ("rows", ctypes.c_int32),
        ("cols", ctypes.c_int32),
        ("nnz", ctypes.c_int32),
        ("ptr", ctypes.c_void_p),
        ("idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
        ("perm", ctypes.c_void_p),
        ("long_len", ctypes.c_int32),
        ("n_chunks", ctypes.c_int32),
        ("n_splits", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("chunks", ctypes.c_void_p),
        ("splits", ctypes.c_void_p),
        ("order", ctypes.c_void_p),
        ("hot", ctypes.c_void_p),
    ]


class fmm_batch_graph(ctypes.Structure):
    _fields_ = [
        ("csr", fmm_sparse),
        ("csc", fmm_sparse),
        ("A", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("dC", ctypes.c_void_p),
        ("C", ctypes.c_void_p),
        ("dA", ctypes.c_void_p),
        ("dB", ctypes.c_void_p),
    ]


class fmm_batch_info(ctypes.Structure):
    _fields_ = [
        ("tile_nnz", ctypes.c_int32),
        ("xcd_aware", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
        ("row_schedule", ctypes.c_int32),
        ("col_schedule", ctypes.c_int32),
        ("n_tiles", ctypes.c_int32),
        ("n_workgroups", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32),
        ("best_ms", ctypes.c_float),
        ("graph_captured", ctypes.c_int32),
    ]


class FmmError(RuntimeError):
    def __init__(self, fn, status, msg, hip_error=0):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        extra = f", hipError {hip_error}" if status == -9 else ""
        super().__init__(f"{fn} -> {self.name}: {msg}{extra}")


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_D = ctypes.c_double
_SP = ctypes.POINTER(fmm_sparse)

# name -> argtypes (restype is int32 status unless listed in _RESTYPE)
SIGNATURES = {
    "fmm_abi_version": [],
    "fmm_status_string": [_I32],
    "fmm_last_hip_error": [],
    "fmm_device_info": [ctypes.POINTER(_I32), ctypes.c_char_p, _I32],
    "fmm_set_tuning": [_I32, _I32],
    "fmm_stream_copy": [_P, _P, _SZ, _P],
    "fmm_stream_read": [_P, _SZ, ctypes.c_uint32, _P, _P],
    "fmm_stream_gather": [_P, _SZ, _P, _I64, ctypes.c_uint32, _P, _P],
    "fmm_gather_hints": [_SP, _P, _I32, _I32, _P, _P],
    "fmm_validate": [_SP, _P],
    "fmm_csr_to_csc_workspace": [_I32, _I32, _I32, ctypes.POINTER(_SZ)],
    "fmm_csr_to_csc": [_I32, _I32, _I32, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _SZ, _P],
    "fmm_gather_values": [_P, _P, _I32, _P, _I32, _P],
    "fmm_gat_backward_workspace": [_SP, _SP, _I32, _I32, ctypes.POINTER(_SZ)],
    "fmm_gat_backward": [_SP, _SP, _P, _P, _P, _P, _P, _P, _P, _P, _I32, _I32, _D, _I32, _P, _P, _P, _P, _P, _SZ, _P],
    "fmm_fusedmm_a_backward_values": [_SP, _P, _P, _P, _I32, _I32, _P, _P, _I32, _P, _SZ, _P],
    "fmm_fusedmm_b_backward_values": [_SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _I32, _P, _SZ, _P],
    "fmm_line_order_workspace": [_I32, ctypes.POINTER(_SZ)],
    "fmm_line_order": [_P, _I32, _I32, _P, _P, _SZ, _P],
    "fmm_schedule_workspace": [_I32, ctypes.POINTER(_SZ)],
    "fmm_schedule_count": [_P, _I32, _I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), _P, _SZ, _P],
    "fmm_schedule_fill": [_P, _I32, _I32, _I32, _P, _P, _P, _SZ, _P],
    "fmm_f32_to_bf16": [_P, _P, _I64, _P],
    "fmm_workspace_size": [_I32, _SP, _SP, _I32, _I32, ctypes.POINTER(_SZ)],
    "fmm_sddmm": [_SP, _P, _P, _I32, _I32, _P, _D, _P, _SZ, _P],
    "fmm_spmm_a": [_SP, _P, _P, _I32, _I32, _P, _D, _P, _SZ, _P],
    "fmm_spmm_b": [_SP, _P, _I32, _P, _I32, _I32, _P, _D, _P, _SZ, _P],
    "fmm_fusedmm_a": [_SP, _P, _P, _I32, _I32, _P, _I32, _P, _P, _SZ, _P],
    "fmm_fusedmm_a_noalloc": [_SP, _P, _P, _I32, _I32, _P, _P],
    "fmm_fusedmm_b": [_SP, _P, _P, _I32, _I32, _P, _I32, _P, _P, _SZ, _P],
    "fmm_fusedmm_a_backward": [_SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _I32, _P, _P, _P, _SZ, _P],
    "fmm_fusedmm_b_backward": [_SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _I32, _P, _P, _P, _SZ, _P],
    "fmm_sddmm_backward": [_SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _P, _SZ, _P],
    "fmm_spmm_a_backward": [_SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _P, _SZ, _P],
    "fmm_spmm_b_backward": [_SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _P, _SZ, _P],
    "fmm_launch_shape": [_SP, _I32, _I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                         ctypes.POINTER(_I32)],
    "fmm_autotune": [_I32, _SP, _SP, _P, _P, _P, _I32, _I32, _P, _P, _P, _P, _SZ, _P],
    "fmm_gat_scores": [_P, _I32, _I32, _I32, _P, _P, _P, _P, _P],
    "fmm_gat_workspace": [_SP, _I32, _I32, ctypes.POINTER(_SZ)],
    "fmm_gat_forward": [_SP, _P, _P, _P, _I32, _I32, _D, _I32, _P, _P, _P, _SZ, _P],
    "fmm_gat_edge_values": [_SP, _P, _P, _I32, _D, _I32, _P, _P],
    "fmm_cg_work_size": [_I32, _I32, ctypes.POINTER(_SZ)],
    "fmm_cg_lines": [_SP, _P, _I32, _I32, _P, ctypes.c_float, _I32, _P, _P, _SZ, _P, _SZ, _P],
    "fmm_residual_workspace": [_SP, ctypes.POINTER(_SZ)],
    "fmm_sddmm_residual": [_SP, _P, _P, _I32, _I32, _P, _P, _SZ, _P],
    "fmm_batch_plan_create": [ctypes.POINTER(fmm_batch_graph), _I32, _I32, _I32, _I32, ctypes.POINTER(_P)],
    "fmm_batch_autotune": [_P, _P],
    "fmm_batch_run": [_P, _P],
    "fmm_batch_capture": [_P, _P],
    "fmm_batch_launch": [_P, _P],
    "fmm_batch_plan_info": [_P, ctypes.POINTER(fmm_batch_info)],
    "fmm_batch_set_schedule": [_P, _I32, _I32, _I32, _I32],
    "fmm_batch_plan_destroy": [_P],
}
_RESTYPE = {"fmm_status_string": ctypes.c_char_p, "fmm_batch_plan_destroy": None}

_lib = None


def load(path: str = LIB_PATH):
    """Load libfmm.so (raises if it is missing) and attach argument types."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libfmm.so not found at {path}: build it with "
                          f"`python -c 'import __graft_entry__ as g; g.build()'` or "
                          f"`python paper_2203_07673_amd/build.py`")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = _RESTYPE.get(name, ctypes.c_int32)
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().fmm_status_string(status).decode()


def check(fn: str, status: int):
    if status != FMM_OK:
        lib = load()
        raise FmmError(fn, status, status_string(status), lib.fmm_last_hip_error())


def call(name: str, *args):
    """Call a status-returning entry point and raise FmmError on failure."""
    st = getattr(load(), name)(*args)
    check(name, st)
    return st


def exported_symbols():
    return list(SIGNATURES)
