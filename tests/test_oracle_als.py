"""Pins for the ALS oracle (Section VI-E): the per-line Gram operator against the dense
masked formula, CG run to convergence against numpy's direct solve of each line's normal
equations, and the residual against a dense computation."""
import numpy as np

import oracle
from workloads import er_exact_degree, rmat, tiny_case, dense_normal


def _mask(S):
    M = np.zeros((S.m, S.n))
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    M[rows, S.colidx] = 1.0
    return M


def test_gram_apply_dense():
    case = tiny_case(19, 14, 5, 0.4, seed=500)
    S, X, F = case["S"], case["A"], case["B"]
    M = _mask(S)
    ref = (M * (X @ F.T)) @ F
    assert np.max(np.abs(oracle.gram_apply(S, X, F) - ref)) <= 1e-12 * (1 + np.abs(ref).max())


def test_cg_converges_to_direct_solve():
    S = er_exact_degree(60, 80, 9, seed=501, val_dtype=np.float64)
    r, lam = 6, 0.3
    F = dense_normal(80, r, 502, dtype=np.float64)
    rhs = dense_normal(60, r, 503, dtype=np.float64)
    X = oracle.cg_lines(S, F, rhs, lam, 40, np.zeros((60, r)))
    for i in range(60):
        Fi = F[S.colidx[S.rowptr[i]:S.rowptr[i + 1]]]
        x = np.linalg.solve(Fi.T @ Fi + lam * np.eye(r), rhs[i])
        assert np.max(np.abs(X[i] - x)) <= 1e-9 * (1 + np.abs(x).max())


def test_cg_columns_via_transpose_and_empty_lines():
    S = rmat(8, 4, seed=504, val_dtype=np.float64)  # has empty rows and columns
    ST = oracle.transpose(S)
    r = 4
    A = dense_normal(S.m, r, 505, dtype=np.float64)
    rhs = dense_normal(S.n, r, 506, dtype=np.float64)
    Y0 = dense_normal(S.n, r, 507, dtype=np.float64)
    Y = oracle.cg_lines(ST, A, rhs, 0.0, 30, Y0)
    empty = np.flatnonzero(np.diff(ST.rowptr) == 0)
    assert np.array_equal(Y[empty], Y0[empty])  # lambda = 0, no entries: M = 0, iterate kept
    for j in np.flatnonzero(np.diff(ST.rowptr) >= 2 * r)[:20]:
        Aj = A[ST.colidx[ST.rowptr[j]:ST.rowptr[j + 1]]]
        y = np.linalg.solve(Aj.T @ Aj, rhs[j])
        assert np.max(np.abs(Y[j] - y)) <= 1e-7 * (1 + np.abs(y).max())


def test_residual_dense():
    case = tiny_case(11, 13, 4, 0.5, seed=508)
    S, A, B = case["S"], case["A"], case["B"]
    M = _mask(S)
    D = np.zeros((S.m, S.n))
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    D[rows, S.colidx] = S.val
    ref = np.sum((M * (D - A @ B.T)) ** 2)
    assert abs(oracle.als_residual(S, A, B) - ref) <= 1e-12 * (1 + ref)
