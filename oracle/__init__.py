"""FP64 CPU oracle for the local FusedMM path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import it, and it imports nothing from them.

The loops live in ``fmm_oracle.c`` (plain double-precision definitions of SDDMM,
SpMMA, SpMMB and the CSR->CSC transpose).  This module assembles the paper's
composite operations from them, exactly as the paper defines them (Section II):

    FusedMMA(S, A, B) = SpMMA(SDDMM(A, B, S), B)
    FusedMMB(S, A, B) = SpMMB(SDDMM(A, B, S), A)

and the adjoints, which the paper does not give.  They are derived here from
R = S * P with P = A B^T (the derivation is repeated in each docstring).  It also
holds the graph-attention variant of the sampled product (Section VI-E).

Every input is promoted exactly to float64 before use.  A "pattern" argument is
any object with attributes ``m, n, rowptr, colidx, val`` (canonical CSR).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from types import SimpleNamespace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
# Two builds of the same source.  "default" is the one every parity check uses.  "native"
# adds -O3 and the host's own instruction set, for timing the oracle on the host's cores.
# Both keep FMA contraction off and never reassociate (no -ffast-math), so every product
# and sum is rounded once, as written, and the two builds give bit-identical results.
_BUILDS = {
    "default": ("liboracle.so", ["-O2"]),
    "native": ("liboracle_native.so", ["-O3", "-march=native"]),
}
_LIB_PATH = os.path.join(_HERE, _BUILDS["default"][0])
_libs = {}
_which = "default"
_lock = threading.Lock()


def build(force: bool = False, native: bool = False) -> str:
    """Compile fmm_oracle.c with gcc (no FMA contraction): liboracle.so, or with
    ``native`` liboracle_native.so (-O3 -march=native, for timing on this host)."""
    name, opt = _BUILDS["native" if native else "default"]
    path = os.path.join(_HERE, name)
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *opt, "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def select_build(which: str) -> None:
    """Route every later oracle call to the "default" or the "native" build.  The native
    build is compiled here, on first use, for this host's CPU."""
    global _which
    if which not in _BUILDS:
        raise ValueError(which)
    if which == "native":
        build(force="native" not in _libs, native=True)
    with _lock:
        _which = which


def build_flags(which: str = None) -> str:
    """The gcc optimisation flags of a build (for reports)."""
    return " ".join(_BUILDS[which or _which][1] + ["-ffp-contract=off", "-fopenmp"])


def _load():
    with _lock:
        lib = _libs.get(_which)
        if lib is None:
            path = build(native=_which == "native")
            lib = ctypes.CDLL(path)
            i64, p = ctypes.c_int64, ctypes.c_void_p
            lib.oracle_sddmm.argtypes = [i64, i64, p, p, p, p, p, p, p, i64]
            lib.oracle_spmm_a.argtypes = [i64, i64, p, p, p, p, p, p, i64]
            lib.oracle_spmm_b.argtypes = [i64, i64, i64, p, p, p, p, p]
            lib.oracle_csr_to_csc.argtypes = [i64, i64, p, p, p, p, p, p, p]
            lib.oracle_num_threads.restype = ctypes.c_int
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            lib.oracle_set_threads.restype = None
            lib.oracle_gat_scores.argtypes = [i64, i64, p, p, p, p, p]
            lib.oracle_gat_scores.restype = None
            lib.oracle_gat_edges.argtypes = [i64, p, p, p, p, p, ctypes.c_double, ctypes.c_int, p]
            lib.oracle_gat_edges.restype = None
            for f in ("oracle_sddmm", "oracle_spmm_a", "oracle_spmm_b", "oracle_csr_to_csc"):
                getattr(lib, f).restype = None
            _libs[_which] = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _rows(rows):
    return None if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the OpenMP routines (timing at a fixed thread count)."""
    _load().oracle_set_threads(int(n))


# ----------------------------------------------------------------------------------
# The three primitives (Section II) and the transpose (Section IV-B)
# ----------------------------------------------------------------------------------

def sddmm(S, A, B, val="S", rows=None, out=None):
    """R[p] = val[p] * <A_i:, B_j:> at each stored entry p = (i, j) (Eq. (1)).

    ``val="S"`` uses S's values, ``val=None`` the pattern alone (all ones), or an
    explicit array.  With ``rows`` only those rows' entries are computed (others 0).
    """
    lib = _load()
    A, B = _f64(A), _f64(B)
    r = A.shape[1]
    assert A.shape == (S.m, r) and B.shape == (S.n, r)
    v = _f64(S.val) if isinstance(val, str) else (None if val is None else _f64(val))
    R = np.zeros(S.colidx.shape[0], dtype=np.float64) if out is None else out
    rp, ci, rw = _i32(S.rowptr), _i32(S.colidx), _rows(rows)
    lib.oracle_sddmm(S.m, r, _ptr(rp), _ptr(ci), _ptr(v), _ptr(A), _ptr(B), _ptr(R),
                     _ptr(rw), 0 if rw is None else rw.shape[0])
    return R


def spmm_a(S, w, B, rows=None):
    """SpMMA: C = W . B where W has S's pattern and stored values ``w`` (Section II)."""
    lib = _load()
    B, w = _f64(B), _f64(w)
    r = B.shape[1]
    assert B.shape[0] == S.n and w.shape[0] == S.colidx.shape[0]
    rw = _rows(rows)
    cnt = S.m if rw is None else rw.shape[0]
    C = np.empty((cnt, r), dtype=np.float64)
    rp, ci = _i32(S.rowptr), _i32(S.colidx)
    lib.oracle_spmm_a(S.m, r, _ptr(rp), _ptr(ci), _ptr(w), _ptr(B), _ptr(C),
                      _ptr(rw), 0 if rw is None else rw.shape[0])
    return C


def spmm_b(S, w, A):
    """SpMMB: C' = W^T . A (n x r), W with S's pattern and stored values ``w`` (Section II)."""
    lib = _load()
    A, w = _f64(A), _f64(w)
    r = A.shape[1]
    assert A.shape[0] == S.m and w.shape[0] == S.colidx.shape[0]
    C = np.empty((S.n, r), dtype=np.float64)
    rp, ci = _i32(S.rowptr), _i32(S.colidx)
    lib.oracle_spmm_b(S.m, S.n, r, _ptr(rp), _ptr(ci), _ptr(w), _ptr(A), _ptr(C))
    return C


def csr_to_csc(S):
    """Stored transposed copy of S (Section IV-B): (colptr, rowidx, valT, perm),
    rows ascending inside each column, perm[q] = CSR position of CSC entry q.
    valT keeps the dtype of S.val."""
    lib = _load()
    nnz = S.colidx.shape[0]
    colptr = np.empty(S.n + 1, dtype=np.int32)
    rowidx = np.empty(nnz, dtype=np.int32)
    perm = np.empty(nnz, dtype=np.int32)
    v = _f64(S.val)
    valT = np.empty(nnz, dtype=np.float64)
    rp, ci = _i32(S.rowptr), _i32(S.colidx)
    lib.oracle_csr_to_csc(S.m, S.n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(colptr), _ptr(rowidx),
                          _ptr(valT), _ptr(perm))
    return colptr, rowidx, valT.astype(np.asarray(S.val).dtype), perm


def transpose(S):
    """S^T as a pattern object (n x m CSR), built from :func:`csr_to_csc`."""
    colptr, rowidx, valT, perm = csr_to_csc(S)
    return SimpleNamespace(m=S.n, n=S.m, rowptr=colptr, colidx=rowidx, val=valT, perm=perm)


def absolute(S):
    """|S|: same pattern, absolute stored values (for magnitude companions)."""
    return SimpleNamespace(m=S.m, n=S.n, rowptr=S.rowptr, colidx=S.colidx,
                           val=np.abs(_f64(S.val)))


# ----------------------------------------------------------------------------------
# Composite operations (Section II) and their adjoints
# ----------------------------------------------------------------------------------

def fusedmm_a(S, A, B, rows=None):
    """FusedMMA(S, A, B) = SpMMA(SDDMM(A, B, S), B); m x r (or the listed rows)."""
    R = sddmm(S, A, B, rows=rows)
    return spmm_a(S, R, B, rows=rows)


def fusedmm_b(S, A, B):
    """FusedMMB(S, A, B) = SpMMB(SDDMM(A, B, S), A); n x r."""
    R = sddmm(S, A, B)
    return spmm_b(S, R, A)


def fusedmm_a_backward(S, A, B, dC):
    """Adjoint of C = FusedMMA(S, A, B) = R B with R = S * (A B^T), S's values fixed.

    With upstream gradient dC (m x r): dL/dR_ij = <dC_i:, B_j:>, so the gradient
    reaching P = A B^T is dP = S * (dC B^T) = SDDMM(dC, B, S).  Then
      dA = dP B                         = SpMMA(dP, B)
      dB = dP^T A + R^T dC              = SpMMB(dP, A) + SpMMB(R, dC)
    (B enters twice: through the sampled product and as the SpMM operand).
    Returns (dA, dB).
    """
    R = sddmm(S, A, B)
    dP = sddmm(S, dC, B)
    dA = spmm_a(S, dP, B)
    dB = spmm_b(S, dP, A) + spmm_b(S, R, dC)
    return dA, dB


def fusedmm_b_backward(S, A, B, dC):
    """Adjoint of C' = FusedMMB(S, A, B) = R^T A with R = S * (A B^T).

    With upstream gradient dC (n x r): dL/dR_ij = <A_i:, dC_j:>, so
    dP = S * (A dC^T) = SDDMM(A, dC, S), and
      dA = dP B + R dC                  = SpMMA(dP, B) + SpMMA(R, dC)
      dB = dP^T A                       = SpMMB(dP, A)
    Returns (dA, dB).
    """
    R = sddmm(S, A, B)
    dP = sddmm(S, A, dC)
    dA = spmm_a(S, dP, B) + spmm_a(S, R, dC)
    dB = spmm_b(S, dP, A)
    return dA, dB


def fusedmm_a_backward_values(S, A, B, dC, rows=None):
    """Gradient of L with respect to S's stored values for C = FusedMMA(S, A, B), the
    adjoint with learned edge values.  C_i = sum_j S_ij P_ij B_j with P = A B^T, so
    dL/dS_ij = P_ij <dC_i:, B_j:>: the pattern's SDDMM of A, B times that of dC, B (CSR
    order; with ``rows`` only those rows' entries, others 0)."""
    return sddmm(S, A, B, val=None, rows=rows) * sddmm(S, dC, B, val=None, rows=rows)


def fusedmm_b_backward_values(S, A, B, dC, rows=None):
    """Gradient with respect to S's stored values for C' = FusedMMB(S, A, B):
    C'_j = sum_i S_ij P_ij A_i, so dL/dS_ij = P_ij <A_i:, dC_j:> (CSR order)."""
    return sddmm(S, A, B, val=None, rows=rows) * sddmm(S, A, dC, val=None, rows=rows)


def sddmm_backward(S, A, B, dR):
    """Adjoint of R = SDDMM(A, B, S) (stored values R[p]) w.r.t. A and B:
    dA = (S * dR) B = SpMMA(S*dR, B), dB = (S * dR)^T A = SpMMB(S*dR, A)."""
    w = _f64(S.val) * _f64(dR)
    return spmm_a(S, w, B), spmm_b(S, w, A)


def spmm_a_backward(S, w, B, dC):
    """Adjoint of C = W B (W: S's pattern with stored values w):
    dw[p] = <dC_i:, B_j:> (an SDDMM with unit values), dB = W^T dC = SpMMB(w, dC)."""
    return sddmm(S, dC, B, val=None), spmm_b(S, w, dC)


def spmm_b_backward(S, w, A, dC):
    """Adjoint of C' = W^T A: dw[p] = <A_i:, dC_j:>, dA = W dC' = SpMMA(w, dC')."""
    return sddmm(S, A, dC, val=None), spmm_a(S, w, dC)


# ----------------------------------------------------------------------------------
# Row- and column-sampled forms for large inputs (rows are independent)
# ----------------------------------------------------------------------------------

def fusedmm_a_rows(S, A, B, rows):
    """Rows ``rows`` of FusedMMA(S, A, B)."""
    return fusedmm_a(S, A, B, rows=rows)


def fusedmm_b_cols(ST, A, B, cols):
    """Columns ``cols`` of FusedMMB(S, A, B), given ST = transpose(S):
    FusedMMB(S, A, B)_j = sum_i S_ij <A_i, B_j> A_i = FusedMMA(S^T, B, A)_j."""
    return fusedmm_a(ST, B, A, rows=cols)


def fusedmm_a_backward_sampled(S, ST, A, B, dC, rows, cols):
    """Rows ``rows`` of dA and rows ``cols`` of dB for the FusedMMA adjoint.
    dA_i = sum_j dP_ij B_j (row form); dB_j = sum_i S_ij(<dC_i,B_j> A_i + <A_i,B_j> dC_i),
    computed on S^T as SpMMA(S^T * (B dC^T), A) + SpMMA(S^T * (B A^T), dC)."""
    dP = sddmm(S, dC, B, rows=rows)
    dA = spmm_a(S, dP, B, rows=rows)
    dPT = sddmm(ST, B, dC, rows=cols)
    RT = sddmm(ST, B, A, rows=cols)
    dB = spmm_a(ST, dPT, A, rows=cols) + spmm_a(ST, RT, dC, rows=cols)
    return dA, dB


def fusedmm_b_backward_sampled(S, ST, A, B, dC, rows, cols):
    """Rows ``rows`` of dA and rows ``cols`` of dB for the FusedMMB adjoint (dC is n x r).
    dA_i = sum_j S_ij(<A_i,dC_j> B_j + <A_i,B_j> dC_j); dB_j = sum_i S_ij <A_i,dC_j> A_i."""
    dP = sddmm(S, A, dC, rows=rows)
    R = sddmm(S, A, B, rows=rows)
    dA = spmm_a(S, dP, B, rows=rows) + spmm_a(S, R, dC, rows=rows)
    dPT = sddmm(ST, dC, A, rows=cols)
    dB = spmm_a(ST, dPT, A, rows=cols)
    return dA, dB


class _Rows:
    """Rows of an array, passed through an elementwise map when taken."""

    def __init__(self, X, f):
        self.X, self.f = X, f

    def __getitem__(self, idx):
        x = self.X[idx]
        return x if self.f is None else self.f(x)


def restrict_rows(S, rows):
    """The stored entries of rows ``rows`` of S as a pattern of their own: row t of the
    result is row rows[t] of S, and the columns those rows touch are renumbered 0..k-1 in
    ascending order (so each row stays canonical).  Returns (pattern, cols) with cols[c]
    the original index of new column c.  Index bookkeeping only: with A[rows] and B[cols],
    every row of a row-form output (FusedMMA, SDDMM, SpMMA, the adjoint's dA) is the same
    sum over the same terms in the same order as on S, since rows are independent."""
    rows = np.asarray(rows, dtype=np.int64)
    rp = np.asarray(S.rowptr, dtype=np.int64)
    lens = rp[rows + 1] - rp[rows]
    ends = np.cumsum(lens)
    pos = np.repeat(rp[rows] - ends + lens, lens) + np.arange(int(ends[-1]) if rows.size else 0)
    col = np.asarray(S.colidx, dtype=np.int64)[pos]
    cols, newcol = np.unique(col, return_inverse=True)
    sub = SimpleNamespace(m=int(rows.size), n=int(cols.size),
                          rowptr=np.concatenate([[0], np.cumsum(lens)]).astype(np.int32),
                          colidx=newcol.astype(np.int32).reshape(-1), val=np.asarray(S.val)[pos])
    return sub, cols


def fusedmm_a_outputs_sampled(S, ST, A, B, dC, rows, cols, prep=None):
    """Rows ``rows`` of C = FusedMMA(S, A, B) and of its adjoint's dA, and rows ``cols`` of
    the adjoint's dB, without touching (or converting) any other row of A, B or dC: each is
    computed on the sub-pattern that holds exactly the entries it sums (rows of S for C and
    dA, rows of ST = S^T for dB; see restrict_rows).  The arithmetic is that of
    fusedmm_a and fusedmm_a_backward_sampled.  ``prep`` = (fA, fB, fdC), elementwise maps
    applied to the rows taken from A, B and dC before use (e.g. bf16_round, np.abs).
    Returns (C_rows, dA_rows, dB_cols)."""
    rows, cols = np.asarray(rows, np.int64), np.asarray(cols, np.int64)
    fA, fB, fG = prep if prep is not None else (None, None, None)
    A = _Rows(A, fA)
    B = _Rows(B, fB)
    dC = _Rows(dC, fG)
    none = np.zeros(0, np.int64)
    Sr, cr = restrict_rows(S, rows)            # row t of Sr is row rows[t] of S
    Ar, Br, Gr = A[rows], B[cr], dC[rows]
    C = fusedmm_a(Sr, Ar, Br)
    dA, _ = fusedmm_a_backward_sampled(Sr, transpose(Sr), Ar, Br, Gr, np.arange(Sr.m), none)
    Tc, rc = restrict_rows(ST, cols)          # column cols[t] of S as row t of Tc, its rows renumbered
    Sc = transpose(Tc)                         # S restricted to rows rc and columns cols
    _, dB = fusedmm_a_backward_sampled(Sc, Tc, A[rc], B[cols], dC[rc], none, np.arange(Tc.m))
    return C, dA, dB


# ----------------------------------------------------------------------------------
# bfloat16 storage rounding (round to nearest, ties to even)
# ----------------------------------------------------------------------------------

def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even) and return them
    as float32.  bfloat16 keeps the top 16 bits of an IEEE binary32; the discarded
    low half decides the rounding.  NaNs stay NaN."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    rounded = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = rounded.view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


# ----------------------------------------------------------------------------------
# Graph attention (Section VI-E): S' = LeakyReLU(S * (H ._GAT H^T)), optionally
# row-softmax normalised, then the aggregation S' . H
# ----------------------------------------------------------------------------------

def gat_scores(H, a1, a2):
    """s = H a1, t = H a2: the two halves of a^T (H_i || H_j) = s_i + t_j."""
    lib = _load()
    H, a1, a2 = _f64(H), _f64(a1), _f64(a2)
    n, r = H.shape
    assert a1.shape == (r,) and a2.shape == (r,)
    s = np.empty(n, dtype=np.float64)
    t = np.empty(n, dtype=np.float64)
    lib.oracle_gat_scores(n, r, _ptr(H), _ptr(a1), _ptr(a2), _ptr(s), _ptr(t))
    return s, t


def gat_edges(S, s, t, slope=0.2, softmax=True, use_val=True):
    """Edge weights in CSR order: LeakyReLU(S_ij (s_i + t_j)), row-softmaxed if asked."""
    lib = _load()
    s, t = _f64(s), _f64(t)
    v = _f64(S.val) if use_val and S.val is not None else None
    w = np.empty(S.colidx.shape[0], dtype=np.float64)
    rp, ci = _i32(S.rowptr), _i32(S.colidx)
    lib.oracle_gat_edges(S.m, _ptr(rp), _ptr(ci), _ptr(v), _ptr(s), _ptr(t), float(slope), int(bool(softmax)),
                         _ptr(w))
    return w


def gat_forward(S, H, a1, a2, slope=0.2, softmax=True, use_val=True, rows=None):
    """One attention head: out = S' . H with S' the (row-softmaxed) LeakyReLU edge values.
    H is n x r with n = S.m = S.n (a square graph)."""
    s, t = gat_scores(H, a1, a2)
    w = gat_edges(S, s, t, slope, softmax, use_val)
    return spmm_a(S, w, H, rows=rows)


def gat_backward(S, H, a1, a2, dO, slope=0.2, softmax=True, use_val=True):
    """Adjoint of the attention head out = W H (the paper gives the forward only; this is
    the chain rule through its definition, step by step).  With upstream gradient dO:

      x_ij = S_ij (s_i + t_j), e = LeakyReLU(x), w = e or its row softmax,
      dw_ij = <dO_i, H_j>                                 (an SDDMM on the pattern)
      de_ij = dw_ij, or with the softmax  w_ij (dw_ij - sum_k w_ik dw_ik)
      dx_ij = de_ij * (1 if x_ij > 0 else slope)          (LeakyReLU's derivative)
      dS_ij = dx_ij (s_i + t_j);   ds_i = sum_j dx_ij S_ij;   dt_j = sum_i dx_ij S_ij
      dH    = W^T dO + ds a1^T + dt a2^T;   da1 = H^T ds;   da2 = H^T dt

    Returns (dH, da1, da2, dS); dS is None without stored values (use_val False)."""
    H, dO = _f64(H), _f64(dO)
    a1, a2 = _f64(a1), _f64(a2)
    n = H.shape[0]
    s, t = gat_scores(H, a1, a2)
    rows = np.repeat(np.arange(S.m), np.diff(np.asarray(S.rowptr, np.int64)))
    cols = np.asarray(S.colidx, np.int64)
    v = _f64(S.val) if use_val and S.val is not None else np.ones(cols.shape[0])
    score = s[rows] + t[cols]
    x = v * score
    w = gat_edges(S, s, t, slope, softmax, use_val)
    dw = sddmm(S, dO, H, val=None)
    # np.add.at adds the terms one at a time in stored order (unbuffered), like a loop
    if softmax:
        D = np.zeros(S.m)
        np.add.at(D, rows, w * dw)
        de = w * (dw - D[rows])
    else:
        de = dw
    dx = de * np.where(x > 0, 1.0, slope)
    g = dx * v
    ds = np.zeros(n)
    dt = np.zeros(n)
    np.add.at(ds, rows, g)
    np.add.at(dt, cols, g)
    dH = spmm_b(S, w, dO) + np.outer(ds, a1) + np.outer(dt, a2)
    da1 = H.T @ ds
    da2 = H.T @ dt
    dS = dx * score if use_val and S.val is not None else None
    return dH, da1, da2, dS


# ----------------------------------------------------------------------------------
# Alternating least squares (Section VI-E): batched CG on the per-line normal equations
# ----------------------------------------------------------------------------------


def gram_apply(S, X, F):
    """Per line i of S's pattern: sum_j <X_i, F_j> F_j (S's values ignored)."""
    return spmm_a(S, sddmm(S, X, F, val=None), F)


def _rowdot(X, Y):
    return np.einsum("ij,ij->i", X, Y)


def cg_lines(S, F, rhs, lam, iters, X0):
    """Conjugate gradients, run for every line of S at once, on
    (sum_{j in line} F_j F_j^T + lam I) x = rhs_line, starting from X0.  Each line runs the
    textbook recurrence (residual r, direction p, alpha = r.r / p.Mp, beta = r'.r' / r.r);
    a line whose residual or curvature is zero keeps its iterate."""
    X = _f64(X0).copy()
    rhs = _f64(rhs)
    F = _f64(F)
    R = rhs - (gram_apply(S, X, F) + lam * X)
    P = R.copy()
    rr = _rowdot(R, R)
    for _ in range(iters):
        MP = gram_apply(S, P, F) + lam * P
        pq = _rowdot(P, MP)
        ok = (rr > 0) & (pq > 0)
        alpha = np.where(ok, rr / np.where(ok, pq, 1.0), 0.0)
        X += alpha[:, None] * P
        R -= alpha[:, None] * MP
        rrn = _rowdot(R, R)
        beta = np.where(rr > 0, rrn / np.where(rr > 0, rr, 1.0), 0.0)
        P = R + beta[:, None] * P
        rr = rrn
    return X


def als_residual(S, A, B):
    """sum over stored entries of (S_ij - <A_i, B_j>)^2, S's values being the observations."""
    pred = sddmm(S, A, B, val=None)
    return float(np.sum((_f64(S.val) - pred) ** 2))
