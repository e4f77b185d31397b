"""GPU parity: every call of the C ABI against the FP64 oracle on seeded inputs.

Sizes span several blocks and ragged tails; dtypes float32 (gate 1e-5), bfloat16
storage (gate 2e-2 against the oracle on the original float32 values, and 1e-5
against the oracle on the bfloat16-rounded values, which isolates accumulation
error) and float64 (gate 1e-12).  Integer results (transpose, schedule, validation)
must match exactly.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from paper_2203_07673_amd import _capi as C
from tests.gates import TOL_BF16, TOL_F32, TOL_F64
from tests.gpu_helpers import (dev, gate, host, log, ref_fusedmm_a, ref_fusedmm_a_backward, ref_fusedmm_b,
                               ref_fusedmm_b_backward, ref_sddmm)
from workloads import CsrPattern, dense_normal, er_exact_degree, rmat, tiny_case, workload

pytestmark = pytest.mark.gpu

TOL = {torch.float32: TOL_F32, torch.bfloat16: TOL_BF16, torch.float64: TOL_F64}


def _pattern(S, **kw):
    return F.Pattern.from_csr(S, **kw)


def _inputs(S, r, seed, dtype):
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A = dense_normal(S.m, r, seed, dtype=npdt)
    B = dense_normal(S.n, r, seed + 1, dtype=npdt)
    return A, B


def _to_dev(x, dtype):
    """Upload; bfloat16 storage is produced by the library's own rounding kernel."""
    if dtype == torch.bfloat16:
        return F.to_bf16(dev(x))
    return dev(x, dtype)


def _ref_inputs(x, dtype):
    return oracle.bf16_round(x) if dtype == torch.bfloat16 else x


CASES = [
    # (name, pattern builder)
    ("er300x200_d9", lambda: er_exact_degree(300, 200, 9, seed=101)),
    ("er1000_d32", lambda: er_exact_degree(1000, 1000, 32, seed=102)),
    ("rmat10", lambda: rmat(10, 8, seed=103)),
    ("tiny_dense", lambda: tiny_case(17, 13, 1, 0.6, seed=104, dtype=np.float32)["S"]),
]


@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_transpose_bit_exact(case):
    S = dict(CASES)[case]()
    log(f"transpose {case} m={S.m} n={S.n} nnz={S.nnz}")
    P = _pattern(S)
    colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
    torch.cuda.synchronize()
    assert np.array_equal(P.colptr.cpu().numpy(), colptr)
    assert np.array_equal(P.rowidx.cpu().numpy(), rowidx)
    assert np.array_equal(P.perm.cpu().numpy(), perm)
    assert np.array_equal(P.valT.cpu().numpy().view(np.uint32), valT.view(np.uint32))


@pytest.mark.parametrize("shape", [(0, 5), (5, 0), (1, 1), (3, 1), (1, 7), (4, 4)])
def test_transpose_degenerate(shape):
    m, n = shape
    S = tiny_case(m, n, 1, 0.5 if m * n > 1 else 1.0, seed=7, dtype=np.float32)["S"]
    log(f"transpose degenerate {shape} nnz={S.nnz}")
    P = _pattern(S)
    colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
    torch.cuda.synchronize()
    assert np.array_equal(P.colptr.cpu().numpy(), colptr)
    assert np.array_equal(P.rowidx.cpu().numpy(), rowidx)
    assert np.array_equal(P.perm.cpu().numpy(), perm)


def test_transpose_large_rmat_bit_exact():
    S = rmat(16, 16, seed=105)
    log(f"transpose rmat16 nnz={S.nnz}")
    P = _pattern(S)
    colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
    torch.cuda.synchronize()
    assert np.array_equal(P.colptr.cpu().numpy(), colptr)
    assert np.array_equal(P.rowidx.cpu().numpy(), rowidx)
    assert np.array_equal(P.perm.cpu().numpy(), perm)


def _validate(m, n, rowptr, colidx):
    d = C.fmm_sparse()
    d.orient, d.rows, d.cols, d.nnz = C.FMM_CSR, m, n, len(colidx)
    rp = dev(np.asarray(rowptr, np.int32))
    ci = dev(np.asarray(colidx if len(colidx) else [0], np.int32))
    d.ptr, d.idx = rp.data_ptr(), ci.data_ptr()
    st = C.load().fmm_validate(ctypes.byref(d), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_validate_codes():
    log("validate codes")
    assert _validate(2, 3, [0, 2, 3], [0, 2, 1]) == 0
    assert _validate(2, 3, [0, 0, 0], []) == 0
    assert _validate(2, 3, [0, 2, 3], [0, 3, 1]) == -5      # column out of range
    assert _validate(2, 3, [0, 2, 3], [0, -1, 1]) == -5     # negative column
    assert _validate(2, 3, [0, 2, 3], [2, 0, 1]) == -6      # unsorted
    assert _validate(2, 3, [0, 2, 3], [1, 1, 1]) == -6      # duplicate
    assert _validate(2, 3, [0, 3, 2], [0, 1, 2]) == -5      # rowptr decreasing
    assert _validate(2, 3, [1, 2, 3], [0, 1, 2]) == -5      # rowptr[0] != 0
    assert _validate(2, 3, [0, 2, 2], [0, 1, 2]) == -5      # rowptr[m] != nnz


def test_schedule_exact():
    S = rmat(12, 16, seed=106)
    log(f"schedule rmat12 nnz={S.nnz}")
    P = _pattern(S, long_len=64, chunk=32)
    sch = P.schedules["csr"]
    lens = np.diff(S.rowptr.astype(np.int64))
    exp_chunks, exp_splits = [], []
    for i, ln in enumerate(lens):
        if ln > 64:
            first = len(exp_chunks)
            b = int(S.rowptr[i])
            c = (int(ln) + 31) // 32
            for k in range(c):
                exp_chunks.append((i, b + 32 * k, min(b + 32 * (k + 1), int(S.rowptr[i + 1]))))
            exp_splits.append((i, first, c))
    assert sch["n_chunks"] == len(exp_chunks) and sch["n_splits"] == len(exp_splits)
    assert np.array_equal(sch["chunks"].cpu().numpy().reshape(-1, 3), np.array(exp_chunks))
    assert np.array_equal(sch["splits"].cpu().numpy().reshape(-1, 3), np.array(exp_splits))


def test_bf16_rounding_matches_oracle():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32),
                        np.array([0.0, -0.0, np.inf, -np.inf, 3.4e38, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1e-40],
                                 np.float32)])
    log("bf16 rounding")
    y = F.to_bf16(dev(x)).view(torch.int16).cpu().numpy().view(np.uint16)
    ref = (oracle.bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(y, ref)
    ynan = F.to_bf16(dev(np.array([np.nan], np.float32))).float().cpu().numpy()
    assert np.isnan(ynan[0])
    # 8-wide groups plus a ragged tail, and a source that is not 16-byte aligned (one-per-thread path)
    xd = dev(x)
    for lo, hi in ((0, 13), (0, 100003), (1, 100004), (3, 11)):
        y = F.to_bf16(xd[lo:hi]).view(torch.int16).cpu().numpy().view(np.uint16)
        assert np.array_equal(y, ref[lo:hi]), (lo, hi)


FWD_SHAPES = [
    # (pattern builder, r, split?)
    (lambda: er_exact_degree(300, 200, 9, seed=111), 1, False),
    (lambda: er_exact_degree(300, 200, 9, seed=112), 3, False),
    (lambda: er_exact_degree(257, 301, 17, seed=113), 8, False),
    (lambda: er_exact_degree(1000, 1000, 32, seed=114), 32, False),
    (lambda: rmat(11, 8, seed=115), 64, True),
    (lambda: er_exact_degree(500, 700, 40, seed=116), 128, False),
    (lambda: rmat(10, 16, seed=117), 256, True),
    (lambda: er_exact_degree(130, 90, 20, seed=118), 96, False),
    (lambda: er_exact_degree(64, 64, 64, seed=119), 1024, False),
    (lambda: er_exact_degree(80, 70, 12, seed=120), 512, False),   # the widest fp64 rows
]


def _dtypes_for(r):
    out = [torch.float32, torch.float64]
    if r % 8 == 0:
        out.append(torch.bfloat16)
    if r > 512 and r % 2 == 0:
        out.remove(torch.float64)
    return out


@pytest.mark.parametrize("k", range(len(FWD_SHAPES)))
def test_forward_parity(k):
    build, r, split = FWD_SHAPES[k]
    S32 = build()
    for dtype in _dtypes_for(r):
        S = S32
        if dtype == torch.float64:
            S = CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx, S32.val.astype(np.float64))
        A, B = _inputs(S, r, 1000 + k, dtype)
        log(f"forward case={k} m={S.m} n={S.n} nnz={S.nnz} r={r} dtype={dtype} split={split}")
        P = _pattern(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
        if split:
            assert P.schedules["csr"] is not None
        Ad, Bd = _to_dev(A, dtype), _to_dev(B, dtype)
        Ar, Br = _ref_inputs(A, dtype), _ref_inputs(B, dtype)
        tol = TOL[dtype]
        ref, mag = ref_fusedmm_a(S, A, B)
        refq, magq = ref_fusedmm_a(S, Ar, Br)
        for fused in (True, False):
            Cg, _ = F.fusedmm_a_raw(P, Ad, Bd, fused=fused)
            gate(f"FusedMMA fused={fused}", host(Cg), ref, mag, tol)
            if dtype == torch.bfloat16:
                gate(f"FusedMMA bf16-rounded fused={fused}", host(Cg), refq, magq, TOL_F32)
        ref, mag = ref_fusedmm_b(S, A, B)
        refq, magq = ref_fusedmm_b(S, Ar, Br)
        for fused in (True, False):
            Cg, _ = F.fusedmm_b_raw(P, Ad, Bd, fused=fused)
            gate(f"FusedMMB fused={fused}", host(Cg), ref, mag, tol)
            if dtype == torch.bfloat16:
                gate(f"FusedMMB bf16-rounded fused={fused}", host(Cg), refq, magq, TOL_F32)
        ref, mag = ref_sddmm(S, A, B)
        gate("SDDMM csr", host(F.sddmm_raw(P, Ad, Bd)), ref, mag, tol)
        # SDDMM on the transposed copy gives the same values in CSC order
        Rt = host(F.sddmm_raw(P, Ad, Bd, orient=C.FMM_CSC))
        perm = P.perm.cpu().numpy()
        gate("SDDMM csc", Rt, ref[perm], mag[perm], tol)
        # SpMMs with S's own values
        refa = oracle.spmm_a(S, S.val, B)
        maga = oracle.spmm_a(oracle.absolute(S), np.abs(S.val), np.abs(B))
        gate("SpMMA", host(F.spmm_a_raw(P, Bd)), refa, maga, tol)
        refb = oracle.spmm_b(S, S.val, A)
        magb = oracle.spmm_b(oracle.absolute(S), np.abs(S.val), np.abs(A))
        gate("SpMMB", host(F.spmm_b_raw(P, Ad)), refb, magb, tol)


# r = 1, 32, 64 (split), 256 (split), 96 (idle lanes), 1024 (widest fp32/bf16 rows), 512 (widest fp64)
@pytest.mark.parametrize("k", [0, 3, 4, 6, 7, 8, 9])
def test_backward_parity(k):
    build, r, split = FWD_SHAPES[k]
    S32 = build()
    for dtype in _dtypes_for(r):
        S = S32
        if dtype == torch.float64:
            S = CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx, S32.val.astype(np.float64))
        A, B = _inputs(S, r, 2000 + k, dtype)
        npdt = np.float64 if dtype == torch.float64 else np.float32
        Ga = dense_normal(S.m, r, 3000 + k, dtype=npdt)
        Gb = dense_normal(S.n, r, 4000 + k, dtype=npdt)
        log(f"backward case={k} nnz={S.nnz} r={r} dtype={dtype} split={split}")
        P = _pattern(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
        Ad, Bd = _to_dev(A, dtype), _to_dev(B, dtype)
        odt = torch.float64 if dtype == torch.float64 else torch.float32
        Gad, Gbd = dev(Ga, odt), dev(Gb, odt)
        tol = TOL[dtype]
        dA, dB, mA, mB = ref_fusedmm_a_backward(S, A, B, Ga)
        for fused in (True, False):
            R_ws = None
            if not fused:
                _, R_ws = F.fusedmm_a_raw(P, Ad, Bd, fused=False)
            gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, Gad, fused=fused, R_ws=R_ws)
            gate(f"FusedMMA dA fused={fused}", host(gA), dA, mA, tol)
            gate(f"FusedMMA dB fused={fused}", host(gB), dB, mB, tol)
        dA, dB, mA, mB = ref_fusedmm_b_backward(S, A, B, Gb)
        for fused in (True, False):
            R_ws = None
            if not fused:
                _, R_ws = F.fusedmm_b_raw(P, Ad, Bd, fused=False)
            gA, gB = F.fusedmm_b_backward_raw(P, Ad, Bd, Gbd, fused=fused, R_ws=R_ws)
            gate(f"FusedMMB dA fused={fused}", host(gA), dA, mA, tol)
            gate(f"FusedMMB dB fused={fused}", host(gB), dB, mB, tol)


def test_autograd_functions_fp32():
    S = er_exact_degree(200, 150, 12, seed=131)
    r = 16
    A, B = _inputs(S, r, 132, torch.float32)
    Ga = dense_normal(S.m, r, 133)
    log("autograd fp32")
    P = _pattern(S)
    At = dev(A).requires_grad_(True)
    Bt = dev(B).requires_grad_(True)
    out = F.fusedmm_a(P, At, Bt)
    (out * dev(Ga)).sum().backward()
    dA, dB, mA, mB = ref_fusedmm_a_backward(S, A, B, Ga)
    gate("autograd dA", host(At.grad), dA, mA, TOL_F32)
    gate("autograd dB", host(Bt.grad), dB, mB, TOL_F32)
    # SDDMM and the SpMMs through autograd
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    dR = np.random.default_rng(134).standard_normal(S.nnz).astype(np.float32)
    At.grad = None
    Bt.grad = None
    F.sddmm(P, At, Bt).mul(dev(dR)).sum().backward()
    eA, eB = oracle.sddmm_backward(S, A, B, dR)
    mA2, mB2 = oracle.sddmm_backward(oracle.absolute(S), np.abs(A), np.abs(B), np.abs(dR))
    gate("sddmm dA", host(At.grad), eA, mA2, TOL_F32)
    gate("sddmm dB", host(Bt.grad), eB, mB2, TOL_F32)
    w = np.random.default_rng(135).standard_normal(S.nnz).astype(np.float32)
    wt = dev(w).requires_grad_(True)
    Bt.grad = None
    Gc = dense_normal(S.m, r, 136)
    (F.spmm_a(P, Bt, wt) * dev(Gc)).sum().backward()
    ew, eB = oracle.spmm_a_backward(S, w, B, Gc)
    mw, mB3 = oracle.spmm_a_backward(oracle.absolute(S), np.abs(w), np.abs(B), np.abs(Gc))
    gate("spmm_a dw", host(wt.grad), ew, mw, TOL_F32)
    gate("spmm_a dB", host(Bt.grad), eB, mB3, TOL_F32)
    wt.grad = None
    At.grad = None
    Gd = dense_normal(S.n, r, 137)
    (F.spmm_b(P, At, wt) * dev(Gd)).sum().backward()
    ew, eA = oracle.spmm_b_backward(S, w, A, Gd)
    mw, mA3 = oracle.spmm_b_backward(oracle.absolute(S), np.abs(w), np.abs(A), np.abs(Gd))
    gate("spmm_b dw", host(wt.grad), ew, mw, TOL_F32)
    gate("spmm_b dA", host(At.grad), eA, mA3, TOL_F32)


def test_fd_case_fp64_and_gradcheck():
    w = workload("fd256_d8_r8", dtype=np.float64)
    S, A, B, G = w["S"], w["A"], w["B"], w["G"]
    log("fd256 fp64 backward + gradcheck")
    P = _pattern(S, val_dtype=torch.float64)
    dA, dB, mA, mB = ref_fusedmm_a_backward(S, A, B, G)
    gA, gB = F.fusedmm_a_backward_raw(P, dev(A), dev(B), dev(G))
    gate("fd256 dA", host(gA), dA, mA, TOL_F64)
    gate("fd256 dB", host(gB), dB, mB, TOL_F64)
    small = tiny_case(12, 10, 3, 0.4, seed=141)
    Ps = _pattern(small["S"], val_dtype=torch.float64)
    At = dev(small["A"]).requires_grad_(True)
    Bt = dev(small["B"]).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: F.fusedmm_a(Ps, a, b), (At, Bt), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda a, b: F.fusedmm_b(Ps, a, b), (At, Bt), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda a, b: F.sddmm(Ps, a, b), (At, Bt), eps=1e-6, atol=1e-8)


def test_invariants_bit_exact():
    S = rmat(11, 8, seed=151)
    r = 32
    A, B = _inputs(S, r, 152, torch.float32)
    log("invariants")
    P = _pattern(S)
    Ad, Bd = dev(A), dev(B)
    C1, _ = F.fusedmm_a_raw(P, Ad, Bd)
    C2, _ = F.fusedmm_a_raw(P, Ad, Bd)
    assert torch.equal(C1, C2)  # run-to-run repeatable
    # FusedMMB(S, A, B) == FusedMMA(S^T, B, A): same arrays, same kernel
    colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
    ST = CsrPattern(S.n, S.m, colptr, rowidx, valT)
    PT = _pattern(ST)
    Cb, _ = F.fusedmm_b_raw(P, Ad, Bd)
    CaT, _ = F.fusedmm_a_raw(PT, Bd, Ad)
    assert torch.equal(Cb, CaT)
    # permuting rows of S and A permutes rows of C exactly
    q = np.random.default_rng(153).permutation(S.m)
    lens = np.diff(S.rowptr)
    rp = np.concatenate([[0], np.cumsum(lens[q])]).astype(np.int32)
    ci = np.concatenate([S.colidx[S.rowptr[i]:S.rowptr[i + 1]] for i in q]).astype(np.int32)
    vv = np.concatenate([S.val[S.rowptr[i]:S.rowptr[i + 1]] for i in q])
    PP = _pattern(CsrPattern(S.m, S.n, rp, ci, vv))
    Cp, _ = F.fusedmm_a_raw(PP, dev(A[q]), Bd)
    assert torch.equal(Cp, C1[torch.from_numpy(q).cuda()])
    # zero-valued entries keep the pattern: R is stored as 0 there
    v0 = S.val.copy()
    v0[::5] = 0
    P0 = _pattern(CsrPattern(S.m, S.n, S.rowptr, S.colidx, v0))
    R0 = F.sddmm_raw(P0, Ad, Bd).cpu().numpy()
    assert R0.shape[0] == S.nnz and np.all(R0[::5] == 0)
    # power-of-two scaling is exact
    C4, _ = F.fusedmm_a_raw(P, Ad, 2 * Bd)
    assert torch.equal(C4, 4 * C1)


def test_empty_rows_and_columns_are_zero():
    rowptr = np.array([0, 0, 2, 2, 3], np.int32)
    colidx = np.array([1, 3, 1], np.int32)
    val = np.array([0.5, 2.0, 1.5], np.float32)
    S = CsrPattern(4, 5, rowptr, colidx, val)
    A, B = _inputs(S, 8, 161, torch.float32)
    log("empty rows/cols")
    P = _pattern(S)
    Cg = host(F.fusedmm_a_raw(P, dev(A), dev(B))[0])
    assert np.all(Cg[0] == 0) and np.all(Cg[2] == 0)
    Cb = host(F.fusedmm_b_raw(P, dev(A), dev(B))[0])
    assert np.all(Cb[0] == 0) and np.all(Cb[2] == 0) and np.all(Cb[4] == 0)
    ref, mag = ref_fusedmm_a(S, A, B)
    gate("tiny C", Cg, ref, mag, TOL_F32)


def test_shape_overrides_agree():
    S = er_exact_degree(777, 500, 13, seed=171)
    r = 128
    A, B = _inputs(S, r, 172, torch.float32)
    log("shape overrides")
    P = _pattern(S)
    Ad, Bd = dev(A), dev(B)
    ref, mag = ref_fusedmm_a(S, A, B)
    try:
        for lanes, nv in [(32, 1), (16, 2), (64, 1), (32, 2), (64, 2)]:
            F.set_tuning(lanes, nv)
            Cg, _ = F.fusedmm_a_raw(P, Ad, Bd)
            gate(f"lanes={lanes} nv={nv}", host(Cg), ref, mag, TOL_F32)
    finally:
        F.set_tuning(0, 0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float64])
def test_batch_variants_parity(dtype):
    S32 = rmat(11, 8, seed=181)
    S = S32 if dtype != torch.float64 else CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx,
                                                        S32.val.astype(np.float64))
    r = 64
    A, B = _inputs(S, r, 182, dtype)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    Ga, Gb = dense_normal(S.m, r, 183, dtype=npdt), dense_normal(S.n, r, 184, dtype=npdt)
    odt = torch.float64 if dtype == torch.float64 else torch.float32
    P = _pattern(S, long_len=64, chunk=32)
    Ad, Bd = _to_dev(A, dtype), _to_dev(B, dtype)
    tol = TOL[dtype]
    ref, mag = ref_fusedmm_a(S, A, B)
    refb, magb = ref_fusedmm_b(S, A, B)
    dA, dB, mA, mB = ref_fusedmm_a_backward(S, A, B, Ga)
    eA, eB, nA, nB = ref_fusedmm_b_backward(S, A, B, Gb)
    Rr, Rm = ref_sddmm(S, A, B)
    for v in (1, 2, 3):
        log(f"variant {v} dtype={dtype}")
        P.set_variant(v, v)
        for fused in (True, False):
            Cg, R_ws = F.fusedmm_a_raw(P, Ad, Bd, fused=fused)
            gate(f"v{v} FusedMMA fused={fused}", host(Cg), ref, mag, tol)
            gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, dev(Ga, odt), fused=fused, R_ws=R_ws)
            gate(f"v{v} dA fused={fused}", host(gA), dA, mA, tol)
            gate(f"v{v} dB fused={fused}", host(gB), dB, mB, tol)
            Cb, Rb = F.fusedmm_b_raw(P, Ad, Bd, fused=fused)
            gate(f"v{v} FusedMMB fused={fused}", host(Cb), refb, magb, tol)
            gA, gB = F.fusedmm_b_backward_raw(P, Ad, Bd, dev(Gb, odt), fused=fused, R_ws=Rb)
            gate(f"v{v} B dA fused={fused}", host(gA), eA, nA, tol)
            gate(f"v{v} B dB fused={fused}", host(gB), eB, nB, tol)
        gate(f"v{v} SDDMM", host(F.sddmm_raw(P, Ad, Bd)), Rr, Rm, tol)
    P.set_variant(0, 0)
    got = P.autotune(Ad, Bd, dev(Ga, odt), form="a")
    assert got["csr"] in (1, 2, 3) and got["csc"] in (1, 2, 3)
    Cg, _ = F.fusedmm_a_raw(P, Ad, Bd)
    gate("autotuned FusedMMA", host(Cg), ref, mag, tol)
    got = P.autotune(Ad, Bd, dev(Gb, odt), form="b")
    assert got["csr"] in (1, 2, 3) and got["csc"] in (1, 2, 3)


@pytest.mark.parametrize("m,n", [(5, 4), (0, 3), (3, 0), (0, 0)])
def test_patterns_without_entries(m, n):
    """nnz = 0 (and zero-size sides): every output is exactly zero, SDDMM is empty,
    and the adjoint calls run, for fused and unfused forms."""
    r = 8
    S = CsrPattern(m, n, np.zeros(m + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    A, B = _inputs(S, r, 191, torch.float32)
    log(f"no entries m={m} n={n}")
    P = _pattern(S)
    assert P.colptr.cpu().numpy().tolist() == [0] * (n + 1)
    Ad, Bd = dev(A), dev(B)
    for fused in (True, False):
        Ca, R = F.fusedmm_a_raw(P, Ad, Bd, fused=fused)
        Cb, _ = F.fusedmm_b_raw(P, Ad, Bd, fused=fused)
        assert tuple(Ca.shape) == (m, r) and tuple(Cb.shape) == (n, r)
        assert not host(Ca).any() and not host(Cb).any()
        gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, dev(dense_normal(m, r, 192)), fused=fused, R_ws=R)
        assert not host(gA).any() and not host(gB).any()
    assert F.sddmm_raw(P, Ad, Bd).numel() == 0
    assert not host(F.spmm_a_raw(P, Bd)).any() and not host(F.spmm_b_raw(P, Ad)).any()


def _order_ref(ptr, long_len):
    lens = np.diff(np.asarray(ptr, np.int64))
    key = np.where(lens > long_len, 1024, 1023 - np.minimum(lens, 1023))
    return np.argsort(key, kind="stable")


@pytest.mark.parametrize("case", ["er300x200_d9", "rmat10", "tiny_dense"])
def test_line_order_exact(case):
    """fmm_line_order: lines up to long_len by decreasing length, then the split ones,
    ties in index order (a stable sort, so the permutation is unique)."""
    S = dict(CASES)[case]()
    log(f"line order {case}")
    for ll in (16, 1 << 30):
        P = _pattern(S, long_len=ll, chunk=min(ll, 16), line_order=True)
        colptr = oracle.csr_to_csc(S)[0]
        assert np.array_equal(P.orders["csr"].cpu().numpy()[:S.m], _order_ref(S.rowptr, ll))
        assert np.array_equal(P.orders["csc"].cpu().numpy()[:S.n], _order_ref(colptr, ll))
    # lengths of 1023 and more sort as equal
    rp = np.array([0, 1500, 1503, 2603, 2603], np.int32)
    ci = np.concatenate([np.arange(1500), np.arange(3), np.arange(1100)]).astype(np.int32)
    S2 = CsrPattern(4, 2000, rp, ci, np.ones(len(ci), np.float32))
    P2 = _pattern(S2, split=False, line_order=True)
    assert P2.orders["csr"].cpu().numpy().tolist() == [0, 2, 1, 3]


def test_line_order_gives_identical_results():
    """The order only moves lines between lane groups: every output is bit-identical."""
    S = rmat(11, 8, seed=195)
    r = 64
    A, B = _inputs(S, r, 196, torch.float32)
    G = dense_normal(S.m, r, 197)
    Gb = dense_normal(S.n, r, 198)
    log("line order identical results")
    Po = _pattern(S, long_len=64, chunk=32, line_order=True)
    Pn = _pattern(S, long_len=64, chunk=32, line_order=False)
    assert Po.csr.order and not Pn.csr.order
    for dtype in (torch.float32, torch.bfloat16):
        Ad, Bd = _to_dev(A, dtype), _to_dev(B, dtype)
        for fused in (True, False):
            outs = []
            for P in (Po, Pn):
                Ca, Ra = F.fusedmm_a_raw(P, Ad, Bd, fused=fused)
                Cb, _ = F.fusedmm_b_raw(P, Ad, Bd, fused=fused)
                gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, dev(G), fused=fused, R_ws=None if fused else Ra)
                hA, hB = F.fusedmm_b_backward_raw(P, Ad, Bd, dev(Gb), fused=fused,
                                                  R_ws=None if fused else F.fusedmm_b_raw(P, Ad, Bd, fused=False)[1])
                outs.append([Ca, Cb, gA, gB, hA, hB, F.sddmm_raw(P, Ad, Bd), F.spmm_a_raw(P, Bd),
                             F.spmm_b_raw(P, Ad)])
            for x, y in zip(*outs):
                assert torch.equal(x, y)
    a1 = dev(dense_normal(1, r, 199, sigma=r ** -0.5)[0])
    a2 = dev(dense_normal(1, r, 200, sigma=r ** -0.5)[0])
    Hd = dev(B)
    assert torch.equal(F.gat_forward(Po, Hd, a1, a2), F.gat_forward(Pn, Hd, a1, a2))


def _hints_ref(S, orient, top):
    """Gather hints by their definition, on the host: entry p is hot when its minor line
    is as long as the top-th longest minor line (every line, for top >= the count)."""
    if orient == C.FMM_CSR:
        idx = np.asarray(S.colidx, np.int64)
        lens = np.bincount(idx, minlength=S.n)
    else:
        ST = oracle.transpose(S)
        idx = np.asarray(ST.colidx, np.int64)
        lens = np.diff(np.asarray(S.rowptr, np.int64))
    if top <= 0:
        return np.zeros(idx.size, np.uint8)
    if top >= lens.size:
        return np.ones(idx.size, np.uint8)
    thr = max(1, int(np.sort(lens)[::-1][top - 1]))
    return (lens[idx] >= thr).astype(np.uint8)


def test_gather_hints_exact_and_results_unchanged():
    """fmm_gather_hints marks exactly the entries of the top minor lines (bit-exact against
    the host definition, both orientations, with ties, none and all), and hints change
    only cache policy: every output is bit-identical with and without them."""
    S = rmat(11, 8, seed=205)
    r = 64
    A, B = _inputs(S, r, 206, torch.float32)
    G = dense_normal(S.m, r, 207)
    Gb = dense_normal(S.n, r, 208)
    log("gather hints")
    Ph = _pattern(S, long_len=64, chunk=32, line_order=True)
    Pn = _pattern(S, long_len=64, chunk=32, line_order=True)
    for orient in (C.FMM_CSR, C.FMM_CSC):
        for top in (1, 37, 300, S.n + 5):
            Ph.set_gather_hints(orient, top)
            got = Ph._hints[orient][1][:S.nnz].cpu().numpy()
            assert np.array_equal(got, _hints_ref(S, orient, top)), (orient, top)
        Ph.set_gather_hints(orient, 200)
    assert Ph.csr.hot and Ph.csc.hot and not Pn.csr.hot
    assert Ph.gather_hints == {"csr": 200, "csc": 200}
    for dtype in (torch.float32, torch.bfloat16):
        Ad, Bd = _to_dev(A, dtype), _to_dev(B, dtype)
        for fused in (True, False):
            outs = []
            for P in (Ph, Pn):
                Ca, Ra = F.fusedmm_a_raw(P, Ad, Bd, fused=fused)
                Cb, _ = F.fusedmm_b_raw(P, Ad, Bd, fused=fused)
                gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, dev(G), fused=fused, R_ws=None if fused else Ra)
                hA, hB = F.fusedmm_b_backward_raw(P, Ad, Bd, dev(Gb), fused=fused,
                                                  R_ws=None if fused else F.fusedmm_b_raw(P, Ad, Bd, fused=False)[1])
                outs.append([Ca, Cb, gA, gB, hA, hB, F.sddmm_raw(P, Ad, Bd), F.spmm_a_raw(P, Bd),
                             F.spmm_b_raw(P, Ad)])
            for x, y in zip(*outs):
                assert torch.equal(x, y)
    # the fp64 path and the autotuner with hints
    A64, B64 = dev(np.asarray(A, np.float64)), dev(np.asarray(B, np.float64))
    S64 = type(S)(S.m, S.n, S.rowptr, S.colidx, np.asarray(S.val, np.float64))
    P64 = F.Pattern.from_csr(S64, long_len=64, chunk=32)
    want, _ = F.fusedmm_a_raw(P64, A64, B64)
    P64.set_gather_hints(C.FMM_CSR, 100)
    assert torch.equal(F.fusedmm_a_raw(P64, A64, B64)[0], want)
    Pn.autotune(_to_dev(A, torch.float32), _to_dev(B, torch.float32), dev(G), form="a")
    assert set(Pn.tuning["csr"]) == {"variant", "long_len", "line_order", "gather_hints"}
    ref, mag = ref_fusedmm_a(S, A, B)
    gate("autotuned with hints", host(F.fusedmm_a_raw(Pn, _to_dev(A, torch.float32), _to_dev(B, torch.float32))[0]),
         ref, mag, TOL_F32)
