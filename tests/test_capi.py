"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/fmm.h, and rejects invalid arguments with the documented status
before touching the device (pointer values below are never dereferenced)."""
import ctypes
import os
import re

import pytest

import paper_2203_07673_amd as F
from paper_2203_07673_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = C.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in C.SIGNATURES, n
    assert lib.fmm_abi_version() == 4


def test_status_strings():
    for code in range(0, -11, -1):
        assert C.status_string(code) and C.status_string(code) != "unknown status"
    assert C.status_string(5) == "unknown status"


FAKE = 0x100000  # 16-byte aligned, never dereferenced


def _desc(orient=C.FMM_CSR, rows=4, cols=5, nnz=6):
    d = C.fmm_sparse()
    d.orient, d.rows, d.cols, d.nnz = orient, rows, cols, nnz
    d.ptr, d.idx, d.val = FAKE, FAKE, FAKE
    return d


def _fa(d, r=32, dtype=C.FMM_F32, A=FAKE, B=FAKE, Cp=FAKE, flags=0, R=None, ws=None, wsb=0):
    return C.load().fmm_fusedmm_a(ctypes.byref(d) if d is not None else None, A, B, r, dtype, Cp, flags, R, ws, wsb,
                                  None)


def test_argument_errors_forward():
    d = _desc()
    assert _fa(None) == -1
    assert _fa(_desc(orient=C.FMM_CSC)) == -4
    assert _fa(_desc(orient=7)) == -4
    assert _fa(_desc(rows=-1)) == -2
    assert _fa(d, r=0) == -3
    assert _fa(d, dtype=9) == -3
    assert _fa(d, r=12, dtype=C.FMM_BF16) == -3          # bf16 needs r % 8 == 0
    assert _fa(d, r=2048) == -3
    assert _fa(d, r=301) == -3                           # r % 4 != 0 above 256
    assert _fa(d, A=None) == -1
    assert _fa(d, Cp=None) == -1
    assert _fa(d, A=FAKE + 4) == -8                      # misaligned vector rows
    assert _fa(d, flags=5) == -2
    assert _fa(d, flags=C.FMM_UNFUSED, R=None) == -7     # unfused needs R workspace
    d.variant = 4
    assert _fa(d) == -2
    d.variant = 0
    d.ptr = None
    assert _fa(d) == -1


def test_workspace_rules_with_schedule():
    d = _desc()
    d.long_len, d.n_chunks, d.n_splits = 4, 10, 2
    d.chunks, d.splits = FAKE, FAKE
    lib = C.load()
    nb = ctypes.c_size_t(0)
    csc = _desc(orient=C.FMM_CSC)
    assert lib.fmm_workspace_size(C.FMM_OP_FUSEDMM_A, ctypes.byref(d), ctypes.byref(csc), 32, C.FMM_F32,
                                  ctypes.byref(nb)) == 0
    assert nb.value == 10 * 32 * 4
    assert lib.fmm_workspace_size(C.FMM_OP_FUSEDMM_A, ctypes.byref(d), ctypes.byref(csc), 32, C.FMM_F64,
                                  ctypes.byref(nb)) == 0
    assert nb.value == 10 * 32 * 8
    assert lib.fmm_workspace_size(C.FMM_OP_SDDMM, ctypes.byref(d), None, 32, C.FMM_F32, ctypes.byref(nb)) == 0
    assert nb.value == 0
    assert _fa(d, ws=None) == -7
    assert _fa(d, ws=FAKE, wsb=100) == -7
    assert _fa(d, ws=FAKE + 8, wsb=1 << 20) == -7        # misaligned workspace
    d.chunks = None
    assert _fa(d, ws=FAKE, wsb=1 << 20) == -1


def test_argument_errors_backward_and_prep():
    lib = C.load()
    csr, csc = _desc(), _desc(orient=C.FMM_CSC)
    bad = _desc(orient=C.FMM_CSC, rows=3)
    args = (FAKE, FAKE, FAKE, 32, C.FMM_F32, FAKE, FAKE, 0, None, None, None, 0, None)
    assert lib.fmm_fusedmm_a_backward(ctypes.byref(csr), ctypes.byref(bad), *args) == -2
    assert lib.fmm_fusedmm_a_backward(ctypes.byref(csc), ctypes.byref(csr), *args) == -4
    assert lib.fmm_fusedmm_b_backward(None, ctypes.byref(csc), *args) == -1
    uargs = (FAKE, FAKE, FAKE, 32, C.FMM_F32, FAKE, FAKE, C.FMM_UNFUSED, None, None, None, 0, None)
    assert lib.fmm_fusedmm_a_backward(ctypes.byref(csr), ctypes.byref(csc), *uargs) == -7
    # a bfloat16 dC: bfloat16 storage and the fused adjoint only; other flag bits are errors
    for fn in (lib.fmm_fusedmm_a_backward, lib.fmm_fusedmm_b_backward):
        for dtype, flags, want in ((C.FMM_F32, C.FMM_DC_BF16, -8), (C.FMM_F64, C.FMM_DC_BF16, -8),
                                   (C.FMM_BF16, C.FMM_UNFUSED | C.FMM_DC_BF16, -8), (C.FMM_BF16, 4, -2),
                                   (C.FMM_F32, 4, -2)):
            fargs = (FAKE, FAKE, FAKE, 32, dtype, FAKE, FAKE, flags, None, None, None, 0, None)
            assert fn(ctypes.byref(csr), ctypes.byref(csc), *fargs) == want, (dtype, flags)
    nb = ctypes.c_size_t(0)
    assert lib.fmm_csr_to_csc_workspace(10, 10, 100, ctypes.byref(nb)) == 0 and nb.value > 800
    assert lib.fmm_csr_to_csc_workspace(-1, 10, 100, ctypes.byref(nb)) == -2
    assert lib.fmm_csr_to_csc(10, 10, 100, FAKE, FAKE, None, 0, FAKE, FAKE, None, FAKE, None, 0, None) == -7
    assert lib.fmm_csr_to_csc(10, 10, 100, None, FAKE, None, 0, FAKE, FAKE, None, FAKE, FAKE, 1 << 30, None) == -1
    assert lib.fmm_csr_to_csc(10, 10, 100, FAKE, FAKE, FAKE, 5, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == -3
    n1, n2 = ctypes.c_int32(0), ctypes.c_int32(0)
    assert lib.fmm_schedule_count(FAKE, 10, 4, 8, ctypes.byref(n1), ctypes.byref(n2), FAKE, 1 << 20, None) == -2
    assert lib.fmm_schedule_count(FAKE, 10, 8, 0, ctypes.byref(n1), ctypes.byref(n2), FAKE, 1 << 20, None) == -2
    assert lib.fmm_schedule_count(FAKE, 10, 8, 8, ctypes.byref(n1), ctypes.byref(n2), None, 0, None) == -7
    assert lib.fmm_f32_to_bf16(None, None, -1, None) == -2
    assert lib.fmm_f32_to_bf16(None, FAKE, 4, None) == -1
    assert lib.fmm_validate(None, None) == -1
    assert lib.fmm_set_tuning(3, 1) == -8
    assert lib.fmm_set_tuning(32, 0) == -2
    assert lib.fmm_set_tuning(0, 0) == 0


def test_python_layer_checks_before_calling():
    import torch
    with pytest.raises(TypeError):
        F.dtype_code(torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError):
        F.Pattern([0, 1], [0], [1.0], (1, 1), device="cpu")


def test_batch_plan_argument_errors():
    lib = C.load()
    plan = ctypes.c_void_p()
    arr = (C.fmm_batch_graph * 2)()
    for x in arr:
        x.csr = _desc()
        x.csc = _desc(orient=C.FMM_CSC)
        x.A = x.B = x.dC = x.C = x.dA = x.dB = FAKE
    create = lib.fmm_batch_plan_create
    assert create(None, 2, 64, C.FMM_F32, 3, ctypes.byref(plan)) == -1
    assert create(arr, 0, 64, C.FMM_F32, 3, ctypes.byref(plan)) == -2
    assert create(arr, 2, 64, C.FMM_F32, 0, ctypes.byref(plan)) == -2
    assert create(arr, 2, 64, C.FMM_F64, 3, ctypes.byref(plan)) == -3
    assert create(arr, 2, 12, C.FMM_BF16, 3, ctypes.byref(plan)) == -3
    assert create(arr, 2, 2048, C.FMM_F32, 3, ctypes.byref(plan)) == -3
    dc16 = C.FMM_BATCH_DC_BF16
    assert create(arr, 2, 64, C.FMM_BF16, dc16, ctypes.byref(plan)) == -2        # no pass asked for
    assert create(arr, 2, 64, C.FMM_BF16, 3 | 8, ctypes.byref(plan)) == -2       # an unknown flag bit
    assert create(arr, 2, 64, C.FMM_F32, 3 | dc16, ctypes.byref(plan)) == -8     # bf16 dC needs bf16 storage
    assert create(arr, 2, 64, C.FMM_BF16, 1 | dc16, ctypes.byref(plan)) == -8    # and the adjoint
    arr[1].csc = _desc(orient=C.FMM_CSR)
    assert create(arr, 2, 64, C.FMM_F32, 3, ctypes.byref(plan)) == -4
    arr[1].csc = _desc(orient=C.FMM_CSC, rows=9)
    assert create(arr, 2, 64, C.FMM_F32, 3, ctypes.byref(plan)) == -2
    arr[1].csc = _desc(orient=C.FMM_CSC)
    arr[1].A = FAKE + 4
    assert create(arr, 2, 64, C.FMM_F32, 3, ctypes.byref(plan)) == -8
    arr[1].A = FAKE
    arr[0].dB = None
    assert create(arr, 2, 64, C.FMM_F32, 3, ctypes.byref(plan)) == -1
    info = C.fmm_batch_info()
    assert lib.fmm_batch_plan_info(None, ctypes.byref(info)) == -1
    assert lib.fmm_batch_run(None, None) == -1
    assert lib.fmm_batch_launch(None, None) == -1
    assert lib.fmm_batch_autotune(None, None) == -1
    assert lib.fmm_batch_set_schedule(None, 1, 0, 0, 0) == -1


def test_line_order_argument_errors():
    lib = C.load()
    nb = ctypes.c_size_t(0)
    assert lib.fmm_line_order_workspace(-1, ctypes.byref(nb)) == -2
    assert lib.fmm_line_order_workspace(10, None) == -1
    assert lib.fmm_line_order_workspace(100000, ctypes.byref(nb)) == 0 and nb.value >= 4 * 100000
    need = nb.value
    assert lib.fmm_line_order(FAKE, -1, 8, FAKE, FAKE, need, None) == -2
    assert lib.fmm_line_order(FAKE, 100000, 0, FAKE, FAKE, need, None) == -2      # long_len >= 1
    assert lib.fmm_line_order(None, 100000, 8, FAKE, FAKE, need, None) == -1
    assert lib.fmm_line_order(FAKE, 100000, 8, None, FAKE, need, None) == -1
    assert lib.fmm_line_order(FAKE, 100000, 8, FAKE, FAKE, need - 1, None) == -7  # workspace too small
    assert lib.fmm_line_order(FAKE, 100000, 8, FAKE, FAKE + 4, need, None) == -7  # misaligned workspace
    assert lib.fmm_line_order(None, 0, 8, None, None, 0, None) == 0              # nothing to order


def test_value_gradient_argument_errors():
    lib = C.load()
    d = _desc()
    assert lib.fmm_fusedmm_a_backward_values(None, FAKE, FAKE, FAKE, 32, 0, FAKE, None, 0, None, 0, None) == -1
    assert lib.fmm_fusedmm_a_backward_values(ctypes.byref(_desc(orient=C.FMM_CSC)), FAKE, FAKE, FAKE, 32, 0, FAKE,
                                             None, 0, None, 0, None) == -4
    assert lib.fmm_fusedmm_a_backward_values(ctypes.byref(d), FAKE, FAKE, FAKE, 32, 0, None, None, 0, None, 0,
                                             None) == -1                                     # dS required
    assert lib.fmm_fusedmm_a_backward_values(ctypes.byref(d), FAKE, FAKE, FAKE, 32, 0, FAKE, None, 3, None, 0,
                                             None) == -2                                     # bad flags
    assert lib.fmm_fusedmm_a_backward_values(ctypes.byref(d), FAKE, FAKE, FAKE, 32, 0, FAKE, FAKE, 1, None, 0,
                                             None) == -8                                     # unfused: no dA
    assert lib.fmm_fusedmm_a_backward_values(ctypes.byref(d), FAKE, FAKE, FAKE, 12, 1, FAKE, None, 0, None, 0,
                                             None) == -3                                     # bf16 needs r % 8
    dc = _desc(orient=C.FMM_CSC)
    dc.perm = None
    assert lib.fmm_fusedmm_b_backward_values(ctypes.byref(d), ctypes.byref(dc), FAKE, FAKE, FAKE, 32, 0, FAKE, None,
                                             0, None, 0, None) == -1                         # fused needs perm
    assert lib.fmm_gather_values(FAKE, FAKE, 1, FAKE, 10, None) == -3                        # values are f32/f64
    assert lib.fmm_gather_values(None, FAKE, 0, FAKE, 10, None) == -1
    assert lib.fmm_gather_values(FAKE, FAKE, 0, FAKE, -1, None) == -2
    assert lib.fmm_gather_values(None, None, 0, None, 0, None) == 0


def test_gat_backward_argument_errors():
    lib = C.load()
    dr, dc = _desc(rows=5, cols=5), _desc(orient=C.FMM_CSC, rows=5, cols=5)
    nb = ctypes.c_size_t(0)
    assert lib.fmm_gat_backward_workspace(ctypes.byref(dr), ctypes.byref(dc), 8, 0, ctypes.byref(nb)) == 0
    assert lib.fmm_gat_backward_workspace(ctypes.byref(dr), ctypes.byref(dc), 8, 7, ctypes.byref(nb)) == -3

    def call(S1=dr, S2=dc, r=8, dtype=0, flags=1, ws=FAKE, wsb=None, dH=FAKE, da1=FAKE, lse=FAKE):
        return lib.fmm_gat_backward(ctypes.byref(S1) if S1 is not None else None, ctypes.byref(S2), FAKE, FAKE, FAKE,
                                    FAKE, FAKE, FAKE, lse, FAKE, r, dtype, 0.2, flags, dH, da1, FAKE, None, ws,
                                    nb.value if wsb is None else wsb, None)
    assert call(S1=None) == -1
    assert call(S1=_desc(orient=C.FMM_CSC, rows=5, cols=5)) == -4
    assert call(S1=_desc(rows=5, cols=6)) == -2                 # attention needs a square pattern
    assert call(flags=4) == -2                                   # an unknown flag bit
    assert call(flags=C.FMM_GAT_SOFTMAX | C.FMM_DC_BF16) == -8    # a bf16 dO needs bf16 features
    assert call(flags=C.FMM_DC_BF16, dtype=2) == -8
    assert call(dH=None) == -1
    assert call(da1=None) == -1
    assert call(wsb=0) == -7
    assert call(ws=FAKE + 16) == -7                              # workspace is 256-byte aligned
    assert call(r=12, dtype=1) == -3                             # bf16 needs r % 8 == 0
    assert call(lse=None) == -1                                  # the softmax adjoint needs the forward's lse


def test_stream_probe_argument_errors():
    lib = C.load()
    assert lib.fmm_stream_copy(FAKE, FAKE, 0, None) == 0       # nothing to do
    assert lib.fmm_stream_copy(None, FAKE, 64, None) == -1
    assert lib.fmm_stream_copy(FAKE, FAKE, 60, None) == -2     # not a multiple of 16
    assert lib.fmm_stream_copy(FAKE + 4, FAKE, 64, None) == -8  # misaligned
    assert lib.fmm_stream_read(FAKE, 64, 0, None, None) == -1
    assert lib.fmm_stream_read(FAKE, 24, 0, FAKE, None) == -2
    assert lib.fmm_stream_read(FAKE + 8, 64, 0, FAKE, None) == -8
    assert lib.fmm_stream_gather(FAKE, 64, FAKE, 0, 0, FAKE, None) == 0          # no rows
    assert lib.fmm_stream_gather(None, 64, FAKE, 4, 0, FAKE, None) == -1
    assert lib.fmm_stream_gather(FAKE, 64, None, 4, 0, FAKE, None) == -1
    assert lib.fmm_stream_gather(FAKE, 64, FAKE, 4, 0, None, None) == -1
    assert lib.fmm_stream_gather(FAKE, 64, FAKE, -4, 0, FAKE, None) == -2
    assert lib.fmm_stream_gather(FAKE + 8, 64, FAKE, 4, 0, FAKE, None) == -8    # misaligned
    for rb in (0, 8, 48, 2048):  # rows of 16 * 2^k bytes, k <= 6
        assert lib.fmm_stream_gather(FAKE, rb, FAKE, 4, 0, FAKE, None) == -2, rb


def test_caller_buffers_are_checked():
    """Outputs and workspaces a caller hands in are checked for device, dtype, layout and
    size before any launch (the kernels would write outside a short or narrow buffer)."""
    import torch

    from paper_2203_07673_amd.fusedmm import _check_buf
    cpu = torch.device("cpu")
    ok = torch.zeros(4, 3)
    assert _check_buf("out", ok, cpu, torch.float32, (4, 3)) is ok
    assert _check_buf("R_ws", torch.zeros(10), cpu, torch.float32, min_numel=10) is not None
    for bad, exc in ((torch.zeros(4, 3, dtype=torch.float64), TypeError), (torch.zeros(3, 3), ValueError),
                     (torch.zeros(3, 4).t(), ValueError), ([0.0] * 12, TypeError)):
        with pytest.raises(exc):
            _check_buf("out", bad, cpu, torch.float32, (4, 3))
    with pytest.raises(ValueError):
        _check_buf("R_ws", torch.zeros(9), cpu, torch.float32, min_numel=10)


def test_upstream_gradient_dtype_rules():
    """Which upstream-gradient dtypes the adjoint wrappers take: the output dtype always; a
    bfloat16 one only with bfloat16 storage and the fused adjoint."""
    import torch

    from paper_2203_07673_amd.fusedmm import _dc_flag
    f32, bf16, f64 = (torch.zeros(1, dtype=d) for d in (torch.float32, torch.bfloat16, torch.float64))
    assert _dc_flag(f32, C.FMM_F32, torch.float32, True) == 0
    assert _dc_flag(f32, C.FMM_BF16, torch.float32, False) == 0
    assert _dc_flag(bf16, C.FMM_BF16, torch.float32, True) == C.FMM_DC_BF16
    assert _dc_flag(f64, C.FMM_F64, torch.float64, True) == 0
    with pytest.raises(ValueError):
        _dc_flag(bf16, C.FMM_BF16, torch.float32, False)  # the unfused adjoint reads dC as float32
    for dc, code, odt in ((bf16, C.FMM_F32, torch.float32), (f64, C.FMM_F32, torch.float32),
                          (f32, C.FMM_F64, torch.float64), (f64, C.FMM_BF16, torch.float32)):
        with pytest.raises(TypeError):
            _dc_flag(dc, code, odt, True)


def test_als_helpers_check_shapes_before_calling():
    """cg_lines gathers F at a line's minor indices and als_residual reads A and B by row
    and column: misshapen operands are refused before any library call (a stand-in
    pattern suffices, since nothing reaches the device)."""
    import torch

    class _Pattern:
        m, n, device = 6, 5, torch.device("cpu")

        def descriptor(self, orient):
            return None

    P = _Pattern()
    x = torch.zeros(6, 4)
    with pytest.raises(ValueError):  # rows as lines: F needs a row per column (5)
        F.cg_lines(P, C.FMM_CSR, torch.zeros(6, 4), x, 1.0, 1, x.clone())
    with pytest.raises(ValueError):  # columns as lines: F needs a row per row (6)
        F.cg_lines(P, C.FMM_CSC, torch.zeros(5, 4), torch.zeros(5, 4), 1.0, 1, torch.zeros(5, 4))
    with pytest.raises(ValueError):
        F.als_residual(P, torch.zeros(6, 4), torch.zeros(6, 4))
    with pytest.raises(TypeError):
        F.als_residual(P, torch.zeros(6, 4), torch.zeros(5, 4, dtype=torch.float64))


def test_raw_wrappers_refuse_bad_buffers_before_calling():
    """The raw wrappers check shapes, dtypes and caller-supplied buffers before touching
    the library; a stand-in pattern (no descriptor, no workspace) shows that nothing is
    called when a check fails."""
    import torch

    class _Pattern:
        m, n, nnz, device = 6, 5, 9, torch.device("cpu")
        val, val_dtype = torch.zeros(9), torch.float32

    P = _Pattern()
    A, B, G = torch.zeros(6, 4), torch.zeros(5, 4), torch.zeros(6, 4)
    cases = [
        (lambda: F.fusedmm_a_raw(P, A, B, out=torch.zeros(5, 4)), ValueError),
        (lambda: F.fusedmm_a_raw(P, A, B, out=torch.zeros(6, 4, dtype=torch.float64)), TypeError),
        (lambda: F.fusedmm_a_raw(P, A, B, fused=False, R_ws=torch.zeros(8)), ValueError),
        (lambda: F.fusedmm_b_raw(P, A, B, out=torch.zeros(6, 4)), ValueError),
        (lambda: F.fusedmm_a_raw(P, A, torch.zeros(5, 4, dtype=torch.float64)), TypeError),
        (lambda: F.fusedmm_a_backward_raw(P, A, B, G, dA=torch.zeros(6, 3)), ValueError),
        (lambda: F.fusedmm_a_backward_raw(P, A, B, G.double()), TypeError),
        (lambda: F.fusedmm_b_backward_raw(P, A, B, torch.zeros(6, 4)), ValueError),   # dC is n x r here
        (lambda: F.fusedmm_a_backward_values_raw(P, A, B, G, dS=torch.zeros(8)), ValueError),
        (lambda: F.sddmm_raw(P, A, B, out=torch.zeros(8)), ValueError),
        (lambda: F.spmm_a_raw(P, B, w=torch.zeros(8)), ValueError),
        (lambda: F.spmm_b_raw(P, A, out=torch.zeros(5, 4).t()), ValueError),
    ]
    for k, (call, exc) in enumerate(cases):
        with pytest.raises(exc):
            call()


def test_batch_plan_refuses_mismatched_graphs_before_calling():
    """BatchPlan checks every graph before the plan is created: a pattern whose stored
    values are float64 (the batch kernel reads float32 values) and a pattern on another
    device than graph 0's are refused with no library call (stand-in patterns, which
    have no descriptor)."""
    import torch

    class _Pattern:
        m, n, nnz, device = 6, 5, 9, torch.device("cpu")
        val, val_dtype = torch.zeros(9), torch.float32

    class _Float64Pattern(_Pattern):
        val, val_dtype = torch.zeros(9, dtype=torch.float64), torch.float64

    class _OtherDevicePattern(_Pattern):
        device = torch.device("meta")

    A, B, G = torch.zeros(6, 8), torch.zeros(5, 8), torch.zeros(6, 8)
    with pytest.raises(TypeError):
        F.BatchPlan([_Pattern(), _Float64Pattern()], [A, A], [B, B], [G, G])
    with pytest.raises(ValueError):
        F.BatchPlan([_Pattern(), _OtherDevicePattern()], [A, A], [B, B], [G, G])
