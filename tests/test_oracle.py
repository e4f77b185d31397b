"""Pins for the FP64 oracle, independent of the oracle's own loops.

Each test checks the oracle against something the paper or mathematics fixes:
dense brute force with numpy matrix products, closed forms (identity pattern,
all-ones pattern -> dense GEMM), exact invariants (permutation, power-of-two
scaling, zero-valued entries), a hand-worked integer example, library routines
(scipy's CSC conversion, torch's bfloat16 rounding, torch CPU autograd on the
dense formulation) and central finite differences, which are exact up to
rounding here because the loss is a polynomial of degree <= 2 in every factor.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from tests import golden_io
from workloads import er_exact_degree, tiny_case, rmat, dense_normal


def dense_of(S):
    D = np.zeros((S.m, S.n))
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    D[rows, S.colidx] = S.val
    return D


def mask_of(S):
    D = np.zeros((S.m, S.n))
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    D[rows, S.colidx] = 1.0
    return D


def stored(S, Dense):
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    return Dense[rows, S.colidx]


def close(a, b, scale, tol=1e-12):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    if a.size:
        assert np.max(np.abs(a - b)) <= tol * max(1.0, scale), np.max(np.abs(a - b))


SHAPES = [(1, 1), (2, 3), (3, 2), (7, 7), (33, 17), (64, 64), (5, 64)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("r", [1, 3, 8, 32])
@pytest.mark.parametrize("density", [0.0, 0.1, 0.5, 1.0])
def test_dense_bruteforce(m, n, r, density):
    case = tiny_case(m, n, r, density, seed=m * 1000 + n * 10 + r)
    S, A, B = case["S"], case["A"], case["B"]
    Sd = dense_of(S)
    P = A @ B.T
    Rd = Sd * P
    scale = np.abs(Sd).sum() * (np.abs(A).max(initial=0) * np.abs(B).max(initial=0) + 1) ** 2 * (r + 1)
    R = oracle.sddmm(S, A, B)
    close(R, stored(S, Rd), scale)
    close(oracle.fusedmm_a(S, A, B), Rd @ B, scale)
    close(oracle.fusedmm_b(S, A, B), Rd.T @ A, scale)
    close(oracle.spmm_a(S, S.val, B), Sd @ B, scale)
    close(oracle.spmm_b(S, S.val, A), Sd.T @ A, scale)


def test_golden_hand_example():
    g = golden_io.load("fusedmm_2x3.txt")
    m, n = int(g["m"]), int(g["n"])
    from types import SimpleNamespace
    S = SimpleNamespace(m=m, n=n, rowptr=g["rowptr"].astype(np.int32),
                        colidx=g["colidx"].astype(np.int32), val=g["val"])
    A, B = g["A"], g["B"]
    assert np.array_equal(oracle.sddmm(S, A, B), g["R"])
    assert np.array_equal(oracle.fusedmm_a(S, A, B), g["C"])
    assert np.array_equal(oracle.fusedmm_b(S, A, B), g["Cb"])
    dA, dB = oracle.fusedmm_a_backward(S, A, B, g["G"])
    assert np.array_equal(dA, g["dA"]) and np.array_equal(dB, g["dB"])
    dA, dB = oracle.fusedmm_b_backward(S, A, B, g["Gb"])
    assert np.array_equal(dA, g["dAb"]) and np.array_equal(dB, g["dBb"])
    colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
    assert np.array_equal(colptr, g["colptr"]) and np.array_equal(rowidx, g["rowidx"])
    assert np.array_equal(perm, g["perm"]) and np.array_equal(valT, g["valT"])


def test_all_ones_pattern_is_dense_gemm():
    m, n, r = 19, 23, 5
    rng = np.random.default_rng(0)
    A, B = rng.standard_normal((m, r)), rng.standard_normal((n, r))
    from types import SimpleNamespace
    S = SimpleNamespace(m=m, n=n, rowptr=(np.arange(m + 1) * n).astype(np.int32),
                        colidx=np.tile(np.arange(n), m).astype(np.int32), val=np.ones(m * n))
    close(oracle.sddmm(S, A, B), (A @ B.T).reshape(-1), 100)
    close(oracle.fusedmm_a(S, A, B), (A @ B.T) @ B, 1e3)
    close(oracle.fusedmm_b(S, A, B), (B @ A.T) @ A, 1e3)


def test_identity_pattern_closed_form():
    n, r = 40, 7
    rng = np.random.default_rng(1)
    A, B, s = rng.standard_normal((n, r)), rng.standard_normal((n, r)), rng.random(n)
    from types import SimpleNamespace
    S = SimpleNamespace(m=n, n=n, rowptr=np.arange(n + 1, dtype=np.int32),
                        colidx=np.arange(n, dtype=np.int32), val=s)
    d = np.einsum("ik,ik->i", A, B)
    close(oracle.sddmm(S, A, B), s * d, 10)
    close(oracle.fusedmm_a(S, A, B), (s * d)[:, None] * B, 100)
    close(oracle.fusedmm_b(S, A, B), (s * d)[:, None] * A, 100)


def test_row_permutation_is_exact():
    S = er_exact_degree(300, 200, 9, seed=3, val_dtype=np.float64)
    A, B = dense_normal(300, 16, 4, dtype=np.float64), dense_normal(200, 16, 5, dtype=np.float64)
    C = oracle.fusedmm_a(S, A, B)
    perm = np.random.default_rng(6).permutation(300)
    lens = np.diff(S.rowptr)
    rowptr = np.concatenate([[0], np.cumsum(lens[perm])]).astype(np.int32)
    colidx = np.concatenate([S.colidx[S.rowptr[i]:S.rowptr[i + 1]] for i in perm]).astype(np.int32)
    val = np.concatenate([S.val[S.rowptr[i]:S.rowptr[i + 1]] for i in perm])
    from types import SimpleNamespace
    SP = SimpleNamespace(m=300, n=200, rowptr=rowptr, colidx=colidx, val=val)
    assert np.array_equal(oracle.fusedmm_a(SP, A[perm], B), C[perm])


def test_column_permutation_within_rounding():
    S = er_exact_degree(120, 90, 11, seed=7, val_dtype=np.float64)
    A, B = dense_normal(120, 8, 8, dtype=np.float64), dense_normal(90, 8, 9, dtype=np.float64)
    q = np.random.default_rng(10).permutation(90)  # new column index of old column c is q[c]
    rows = np.repeat(np.arange(120), np.diff(S.rowptr))
    newc = q[S.colidx]
    order = np.lexsort((newc, rows))
    from types import SimpleNamespace
    SP = SimpleNamespace(m=120, n=90, rowptr=S.rowptr, colidx=newc[order].astype(np.int32),
                         val=S.val[order])
    Bp = np.empty_like(B)
    Bp[q] = B
    C, Cp = oracle.fusedmm_a(S, A, B), oracle.fusedmm_a(SP, A, Bp)
    close(C, Cp, np.abs(C).max(), tol=1e-13)


def test_zero_valued_entries_keep_pattern():
    S = er_exact_degree(50, 60, 6, seed=11, val_dtype=np.float64)
    A, B = dense_normal(50, 4, 12, dtype=np.float64), dense_normal(60, 4, 13, dtype=np.float64)
    val = S.val.copy()
    zero = np.zeros_like(val, dtype=bool)
    zero[::3] = True
    val[zero] = 0.0
    from types import SimpleNamespace
    SZ = SimpleNamespace(m=50, n=60, rowptr=S.rowptr, colidx=S.colidx, val=val)
    R = oracle.sddmm(SZ, A, B)
    assert R.shape[0] == S.nnz and np.all(R[zero] == 0)
    # dropping those entries from the pattern changes nothing else
    keep = ~zero
    rows = np.repeat(np.arange(50), np.diff(S.rowptr))
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=50))]).astype(np.int32)
    SD = SimpleNamespace(m=50, n=60, rowptr=rp, colidx=S.colidx[keep], val=val[keep])
    assert np.array_equal(oracle.fusedmm_a(SZ, A, B), oracle.fusedmm_a(SD, A, B))
    assert np.array_equal(oracle.fusedmm_b(SZ, A, B), oracle.fusedmm_b(SD, A, B))


def test_power_of_two_scaling_is_exact():
    S = er_exact_degree(64, 64, 8, seed=14, val_dtype=np.float64)
    A, B = dense_normal(64, 8, 15, dtype=np.float64), dense_normal(64, 8, 16, dtype=np.float64)
    C = oracle.fusedmm_a(S, A, B)
    from types import SimpleNamespace
    S2 = SimpleNamespace(m=64, n=64, rowptr=S.rowptr, colidx=S.colidx, val=2 * S.val)
    assert np.array_equal(oracle.fusedmm_a(S, A, 2 * B), 4 * C)
    assert np.array_equal(oracle.fusedmm_a(S2, A, B), 2 * C)
    assert np.array_equal(oracle.fusedmm_a(S, 0.5 * A, B), 0.5 * C)


def test_linearity_in_values_and_A():
    S = er_exact_degree(40, 30, 5, seed=17, val_dtype=np.float64)
    A1, A2 = dense_normal(40, 6, 18, dtype=np.float64), dense_normal(40, 6, 19, dtype=np.float64)
    B = dense_normal(30, 6, 20, dtype=np.float64)
    C = oracle.fusedmm_a(S, A1 + A2, B)
    close(C, oracle.fusedmm_a(S, A1, B) + oracle.fusedmm_a(S, A2, B), np.abs(C).max() + 1, 1e-13)


def test_fusedmm_b_is_fusedmm_a_on_transpose():
    S = rmat(9, 8, seed=21, val_dtype=np.float64)
    A, B = dense_normal(S.m, 12, 22, dtype=np.float64), dense_normal(S.n, 12, 23, dtype=np.float64)
    ST = oracle.transpose(S)
    # same products, same ascending-row order inside each column: bitwise equal
    assert np.array_equal(oracle.fusedmm_b(S, A, B), oracle.fusedmm_a(ST, B, A))
    cols = np.array([0, 5, 77, S.n - 1])
    assert np.array_equal(oracle.fusedmm_b_cols(ST, A, B, cols), oracle.fusedmm_b(S, A, B)[cols])


def test_csr_to_csc_matches_scipy_and_round_trips():
    for S in (rmat(10, 8, seed=24), er_exact_degree(77, 130, 13, seed=25), tiny_case(9, 4, 2, 0.5, 26)["S"]):
        colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
        M = sp.csr_matrix((np.arange(S.nnz, dtype=np.float64) + 1, S.colidx, S.rowptr), shape=(S.m, S.n))
        Mc = M.tocsc()
        Mc.sort_indices()
        assert np.array_equal(colptr, Mc.indptr) and np.array_equal(rowidx, Mc.indices)
        assert np.array_equal(perm, Mc.data.astype(np.int64) - 1)
        assert np.array_equal(valT, np.asarray(S.val)[perm])
        # round trip: transposing the transpose gives back the CSR arrays
        from types import SimpleNamespace
        T = SimpleNamespace(m=S.n, n=S.m, rowptr=colptr, colidx=rowidx, val=valT)
        rp2, ci2, v2, perm2 = oracle.csr_to_csc(T)
        assert np.array_equal(rp2, S.rowptr) and np.array_equal(ci2, S.colidx)
        assert np.array_equal(v2, S.val) and np.array_equal(perm[perm2], np.arange(S.nnz))


def test_csr_to_csc_dense_bruteforce_tiny():
    for seed in range(5):
        S = tiny_case(6, 5, 1, 0.4, seed)["S"]
        colptr, rowidx, valT, perm = oracle.csr_to_csc(S)
        D = dense_of(S)
        exp_rows, exp_vals = [], []
        for j in range(S.n):
            for i in range(S.m):
                if mask_of(S)[i, j]:
                    exp_rows.append(i)
                    exp_vals.append(D[i, j])
        assert list(rowidx) == exp_rows and np.array_equal(valT, exp_vals)
        assert list(np.diff(colptr)) == [int(mask_of(S)[:, j].sum()) for j in range(S.n)]


def _loss_a(S, A, B, G):
    return float((oracle.fusedmm_a(S, A, B) * G).sum())


def _loss_b(S, A, B, G):
    return float((oracle.fusedmm_b(S, A, B) * G).sum())


@pytest.mark.parametrize("variant", ["a", "b"])
def test_backward_central_differences(variant):
    # 256 x 256, 8 per row, r = 8, fp64; loss = sum(C * G) is linear in A and
    # quadratic in B, so central differences are exact up to rounding.
    S = er_exact_degree(256, 256, 8, seed=27, val_dtype=np.float64)
    A, B = dense_normal(256, 8, 28, dtype=np.float64), dense_normal(256, 8, 29, dtype=np.float64)
    G = dense_normal(256, 8, 30, dtype=np.float64)
    loss = _loss_a if variant == "a" else _loss_b
    bwd = oracle.fusedmm_a_backward if variant == "a" else oracle.fusedmm_b_backward
    dA, dB = bwd(S, A, B, G)
    h = 2.0 ** -8
    rng = np.random.default_rng(31)
    for X, dX in ((A, dA), (B, dB)):
        idx = rng.choice(X.size, 300, replace=False)
        for e in idx:
            i, k = divmod(int(e), X.shape[1])
            old = X[i, k]
            X[i, k] = old + h
            lp = loss(S, A, B, G)
            X[i, k] = old - h
            lm = loss(S, A, B, G)
            X[i, k] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - dX[i, k]) <= 1e-8 * max(1.0, abs(dX[i, k])), (i, k, fd, dX[i, k])


def test_backward_full_fd_tiny():
    case = tiny_case(6, 5, 3, 0.5, seed=32)
    S, A, B = case["S"], case["A"], case["B"]
    for variant, G in (("a", case["G"]), ("b", np.random.default_rng(33).standard_normal((5, 3)))):
        loss = _loss_a if variant == "a" else _loss_b
        dA, dB = (oracle.fusedmm_a_backward if variant == "a" else oracle.fusedmm_b_backward)(S, A, B, G)
        h = 2.0 ** -6
        for X, dX in ((A, dA), (B, dB)):
            for i in range(X.shape[0]):
                for k in range(X.shape[1]):
                    old = X[i, k]
                    X[i, k] = old + h
                    lp = loss(S, A, B, G)
                    X[i, k] = old - h
                    lm = loss(S, A, B, G)
                    X[i, k] = old
                    assert abs((lp - lm) / (2 * h) - dX[i, k]) <= 1e-10 * max(1, abs(dX[i, k]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_vs_dense_torch_autograd(seed):
    case = tiny_case(13, 11, 5, 0.3, seed=40 + seed)
    S, A, B, G = case["S"], case["A"], case["B"], case["G"]
    Gb = np.random.default_rng(seed).standard_normal((11, 5))
    Sd = torch.tensor(dense_of(S))
    for variant in ("a", "b"):
        At = torch.tensor(A, requires_grad=True)
        Bt = torch.tensor(B, requires_grad=True)
        Rt = Sd * (At @ Bt.T)
        if variant == "a":
            C, Gt = Rt @ Bt, torch.tensor(G)
            dA, dB = oracle.fusedmm_a_backward(S, A, B, G)
        else:
            C, Gt = Rt.T @ At, torch.tensor(Gb)
            dA, dB = oracle.fusedmm_b_backward(S, A, B, Gb)
        (C * Gt).sum().backward()
        close(dA, At.grad.numpy(), 100)
        close(dB, Bt.grad.numpy(), 100)


def test_primitive_adjoints_vs_dense_torch_autograd():
    case = tiny_case(9, 7, 4, 0.4, seed=50)
    S, A, B = case["S"], case["A"], case["B"]
    rng = np.random.default_rng(51)
    Sd, M = torch.tensor(dense_of(S)), torch.tensor(mask_of(S))
    dR = rng.standard_normal(S.nnz)
    At, Bt = torch.tensor(A, requires_grad=True), torch.tensor(B, requires_grad=True)
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    R = (Sd * (At @ Bt.T))[rows, S.colidx]
    (R * torch.tensor(dR)).sum().backward()
    dA, dB = oracle.sddmm_backward(S, A, B, dR)
    close(dA, At.grad.numpy(), 100)
    close(dB, Bt.grad.numpy(), 100)
    # SpMMA / SpMMB with learnable stored values w
    w = rng.standard_normal(S.nnz)
    for variant in ("a", "b"):
        wt = torch.tensor(w, requires_grad=True)
        W = torch.zeros(S.m, S.n, dtype=torch.float64).index_put((torch.tensor(rows), torch.tensor(S.colidx.astype(np.int64))), wt)
        Xt = torch.tensor(B if variant == "a" else A, requires_grad=True)
        C = W @ Xt if variant == "a" else W.T @ Xt
        Gt = torch.tensor(rng.standard_normal(tuple(C.shape)))
        (C * Gt).sum().backward()
        if variant == "a":
            dw, dX = oracle.spmm_a_backward(S, w, B, Gt.numpy())
        else:
            dw, dX = oracle.spmm_b_backward(S, w, A, Gt.numpy())
        close(dw, wt.grad.numpy(), 100)
        close(dX, Xt.grad.numpy(), 100)


def test_backward_identities():
    S = rmat(8, 6, seed=60, val_dtype=np.float64)
    A, B = dense_normal(S.m, 6, 61, dtype=np.float64), dense_normal(S.n, 6, 62, dtype=np.float64)
    # with dC := A the FusedMMA adjoint's dB equals 2 * FusedMMB(S, A, B), exactly
    _, dB = oracle.fusedmm_a_backward(S, A, B, A)
    assert np.array_equal(dB, 2 * oracle.fusedmm_b(S, A, B))
    # dA of FusedMMA is FusedMMA(S, dC, B)
    G = dense_normal(S.m, 6, 63, dtype=np.float64)
    dA, _ = oracle.fusedmm_a_backward(S, A, B, G)
    assert np.array_equal(dA, oracle.fusedmm_a(S, G, B))


def test_sampled_forms_match_full():
    S = rmat(9, 8, seed=64, val_dtype=np.float64)
    ST = oracle.transpose(S)
    A, B = dense_normal(S.m, 5, 65, dtype=np.float64), dense_normal(S.n, 5, 66, dtype=np.float64)
    Ga, Gb = dense_normal(S.m, 5, 67, dtype=np.float64), dense_normal(S.n, 5, 68, dtype=np.float64)
    rows = np.array([3, 0, 511, 200, 17])
    cols = np.array([1, 400, 2, 511])
    dA, dB = oracle.fusedmm_a_backward(S, A, B, Ga)
    sA, sB = oracle.fusedmm_a_backward_sampled(S, ST, A, B, Ga, rows, cols)
    close(sA, dA[rows], 1e3, 1e-13)
    close(sB, dB[cols], 1e3, 1e-13)
    dA, dB = oracle.fusedmm_b_backward(S, A, B, Gb)
    sA, sB = oracle.fusedmm_b_backward_sampled(S, ST, A, B, Gb, rows, cols)
    close(sA, dA[rows], 1e3, 1e-13)
    close(sB, dB[cols], 1e3, 1e-13)
    assert np.array_equal(oracle.fusedmm_a_rows(S, A, B, rows), oracle.fusedmm_a(S, A, B)[rows])


def test_restricted_samples_match_full():
    # the sampled outputs computed on restricted patterns equal the full computation bit for
    # bit (same terms, same order), for float32 inputs, with empty and repeated lines
    S = rmat(10, 8, seed=71)
    ST = oracle.transpose(S)
    r = 16
    A, B, G = dense_normal(S.m, r, 72), dense_normal(S.n, r, 73), dense_normal(S.m, r, 74)
    lens_r, lens_c = np.diff(S.rowptr), np.diff(ST.rowptr)
    rows = np.array([int(np.argmax(lens_r)), int(np.flatnonzero(lens_r == 0)[0]), 0, 1023, 5, 5])
    cols = np.array([int(np.argmax(lens_c)), int(np.flatnonzero(lens_c == 0)[0]), 3, 1023, 3])
    C, dA, dB = oracle.fusedmm_a_outputs_sampled(S, ST, A, B, G, rows, cols)
    fA, fB = oracle.fusedmm_a_backward(S, A, B, G)
    assert np.array_equal(C, oracle.fusedmm_a(S, A, B)[rows])
    assert np.array_equal(dA, fA[rows])
    assert np.array_equal(dB, fB[cols])
    sub, cmap = oracle.restrict_rows(S, rows)
    assert sub.m == rows.size and np.all(np.diff(cmap) > 0)
    for t, i in enumerate(rows):
        got = cmap[sub.colidx[sub.rowptr[t]:sub.rowptr[t + 1]]]
        assert np.array_equal(got, S.colidx[S.rowptr[i]:S.rowptr[i + 1]])


def test_native_build_is_bit_identical():
    # the -O3 -march=native build (timed on the host) computes exactly what the parity
    # build computes: contraction stays off and nothing is reassociated
    case = tiny_case(40, 30, 24, 0.3, seed=75)
    S, A, B, G = case["S"], case["A"], case["B"], case["G"]
    ref = (oracle.fusedmm_a(S, A, B),) + oracle.fusedmm_a_backward(S, A, B, G) + oracle.csr_to_csc(S)
    try:
        oracle.select_build("native")
        got = (oracle.fusedmm_a(S, A, B),) + oracle.fusedmm_a_backward(S, A, B, G) + oracle.csr_to_csc(S)
    finally:
        oracle.select_build("default")
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(70)
    x = np.concatenate([
        rng.standard_normal(10000).astype(np.float32),
        (rng.standard_normal(1000) * 1e-40).astype(np.float32),  # subnormals
        np.array([0.0, -0.0, np.inf, -np.inf, 3.4e38, -3.4e38, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8,
                  1.0 + 2 ** -9, 65504.0], dtype=np.float32),
    ])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(oracle.bf16_round(np.array([np.nan], np.float32))[0])


# ------------------------------------------------------------ gradient w.r.t. S's values

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_value_gradient_vs_dense_torch_autograd(seed):
    """dL/dS at the stored entries, against torch autograd through the dense masked
    products (FusedMMA: C = (S*(A B^T)) B; FusedMMB: C' = (S*(A B^T))^T A)."""
    case = tiny_case(13, 11, 5, 0.3, seed=80 + seed)
    S, A, B, G = case["S"], case["A"], case["B"], case["G"]
    Gb = np.random.default_rng(90 + seed).standard_normal((11, 5))
    rows = torch.tensor(np.repeat(np.arange(S.m), np.diff(S.rowptr)))
    cols = torch.tensor(S.colidx.astype(np.int64))
    for variant in ("a", "b"):
        st = torch.tensor(np.asarray(S.val, np.float64), requires_grad=True)
        Sd = torch.zeros(S.m, S.n, dtype=torch.float64).index_put((rows, cols), st)
        At, Bt = torch.tensor(A), torch.tensor(B)
        R = Sd * (At @ Bt.T)
        if variant == "a":
            (R @ Bt * torch.tensor(G)).sum().backward()
            ds = oracle.fusedmm_a_backward_values(S, A, B, G)
        else:
            (R.T @ At * torch.tensor(Gb)).sum().backward()
            ds = oracle.fusedmm_b_backward_values(S, A, B, Gb)
        close(ds, st.grad.numpy(), 100)


def test_value_gradient_central_differences():
    # L = sum(C * G) is linear in S's values, so central differences are exact up to rounding
    S = er_exact_degree(256, 256, 8, seed=84, val_dtype=np.float64)
    A, B = dense_normal(256, 8, 85, dtype=np.float64), dense_normal(256, 8, 86, dtype=np.float64)
    G = dense_normal(256, 8, 87, dtype=np.float64)
    for variant in ("a", "b"):
        fwd = oracle.fusedmm_a if variant == "a" else oracle.fusedmm_b
        ds = (oracle.fusedmm_a_backward_values if variant == "a" else oracle.fusedmm_b_backward_values)(S, A, B, G)
        h = 0.5
        rng = np.random.default_rng(88)
        for p in rng.choice(S.nnz, 200, replace=False):
            old = S.val[p]
            S.val[p] = old + h
            lp = float((fwd(S, A, B) * G).sum())
            S.val[p] = old - h
            lm = float((fwd(S, A, B) * G).sum())
            S.val[p] = old
            assert abs((lp - lm) / (2 * h) - ds[p]) <= 1e-10 * max(1.0, abs(ds[p]))


def test_value_gradient_identities():
    """sum_p S_p dS_p = <C, dC> (C is linear in S), and the rows form matches the full one."""
    S = rmat(9, 8, seed=89, val_dtype=np.float64)
    r = 6
    A, B = dense_normal(S.m, r, 90, dtype=np.float64), dense_normal(S.n, r, 91, dtype=np.float64)
    G, Gb = dense_normal(S.m, r, 92, dtype=np.float64), dense_normal(S.n, r, 93, dtype=np.float64)
    da = oracle.fusedmm_a_backward_values(S, A, B, G)
    db = oracle.fusedmm_b_backward_values(S, A, B, Gb)
    ca, cb = float((oracle.fusedmm_a(S, A, B) * G).sum()), float((oracle.fusedmm_b(S, A, B) * Gb).sum())
    assert abs(float(np.dot(S.val, da)) - ca) <= 1e-10 * max(1.0, float(np.abs(S.val) @ np.abs(da)))
    assert abs(float(np.dot(S.val, db)) - cb) <= 1e-10 * max(1.0, float(np.abs(S.val) @ np.abs(db)))
    rows = np.array([0, 5, 17, S.m - 1])
    part = oracle.fusedmm_a_backward_values(S, A, B, G, rows=rows)
    keep = np.zeros(S.nnz, bool)
    for i in rows:
        keep[S.rowptr[i]:S.rowptr[i + 1]] = True
    assert np.array_equal(part[keep], da[keep]) and not part[~keep].any()
