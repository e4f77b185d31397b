"""Pins for the graph-attention oracle (Section VI-E): dense brute force in numpy,
torch's LeakyReLU and softmax on the dense masked matrix, and closed forms."""
import numpy as np
import pytest
import torch

import oracle
from workloads import er_exact_degree, tiny_case, rmat, dense_normal


def _dense(S):
    D = np.zeros((S.m, S.n))
    M = np.zeros((S.m, S.n), dtype=bool)
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    D[rows, S.colidx] = S.val
    M[rows, S.colidx] = True
    return D, M


@pytest.mark.parametrize("softmax", [True, False])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gat_dense_bruteforce_numpy(softmax, seed):
    case = tiny_case(23, 23, 6, 0.3, seed=300 + seed)
    S, H = case["S"], case["A"]
    rng = np.random.default_rng(seed)
    a1, a2 = rng.standard_normal(6), rng.standard_normal(6)
    D, M = _dense(S)
    s, t = H @ a1, H @ a2
    X = D * (s[:, None] + t[None, :])
    E = np.where(X >= 0, X, 0.2 * X)
    if softmax:
        Em = np.where(M, E, -np.inf)
        mx = np.max(Em, axis=1, keepdims=True)
        mx = np.where(np.isfinite(mx), mx, 0)
        P = np.where(M, np.exp(Em - mx), 0)
        den = P.sum(axis=1, keepdims=True)
        W = np.where(den > 0, P / np.where(den > 0, den, 1), 0)
    else:
        W = np.where(M, E, 0)
    got = oracle.gat_forward(S, H, a1, a2, slope=0.2, softmax=softmax)
    assert np.max(np.abs(got - W @ H)) <= 1e-12 * (1 + np.abs(W @ H).max())


def test_gat_vs_torch_leaky_relu_and_softmax():
    case = tiny_case(17, 17, 5, 0.4, seed=310)
    S, H = case["S"], case["A"]
    rng = np.random.default_rng(311)
    a1, a2 = rng.standard_normal(5), rng.standard_normal(5)
    D, M = _dense(S)
    Ht = torch.tensor(H)
    s = Ht @ torch.tensor(a1)
    t = Ht @ torch.tensor(a2)
    E = torch.nn.functional.leaky_relu(torch.tensor(D) * (s[:, None] + t[None, :]), negative_slope=0.3)
    E = E.masked_fill(~torch.tensor(M), float("-inf"))
    W = torch.softmax(E, dim=1)
    W = torch.nan_to_num(W, nan=0.0)  # rows without entries
    ref = (W @ Ht).numpy()
    got = oracle.gat_forward(S, H, a1, a2, slope=0.3, softmax=True)
    assert np.max(np.abs(got - ref)) <= 1e-12 * (1 + np.abs(ref).max())


def test_gat_zero_attention_is_neighbour_mean():
    S = er_exact_degree(200, 200, 7, seed=312, val_dtype=np.float64)
    H = dense_normal(200, 9, 313, dtype=np.float64)
    z = np.zeros(9)
    got = oracle.gat_forward(S, H, z, z, softmax=True)
    ref = np.stack([H[S.colidx[S.rowptr[i]:S.rowptr[i + 1]]].mean(axis=0) for i in range(200)])
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_gat_single_neighbour_copies_row_and_weights_sum_to_one():
    n = 50
    perm = np.random.default_rng(314).permutation(n)
    from types import SimpleNamespace
    S = SimpleNamespace(m=n, n=n, rowptr=np.arange(n + 1, dtype=np.int32), colidx=perm.astype(np.int32),
                        val=np.ones(n))
    H = dense_normal(n, 4, 315, dtype=np.float64)
    a1, a2 = dense_normal(1, 4, 316, dtype=np.float64)[0], dense_normal(1, 4, 317, dtype=np.float64)[0]
    assert np.array_equal(oracle.gat_forward(S, H, a1, a2, softmax=True), H[perm])
    S2 = rmat(9, 8, seed=318, val_dtype=np.float64)
    H2 = dense_normal(S2.m, 4, 319, dtype=np.float64)
    s, t = oracle.gat_scores(H2, a1, a2)
    w = oracle.gat_edges(S2, s, t, softmax=True)
    sums = np.add.reduceat(w, S2.rowptr[:-1][np.diff(S2.rowptr) > 0])
    assert np.allclose(sums, 1.0, atol=1e-14, rtol=0)


# ------------------------------------------------------------ adjoint of the attention head

def _torch_head(S, H, a1, a2, vals, slope, softmax):
    """The head through torch on the dense masked matrix (autograd reference)."""
    rows = torch.tensor(np.repeat(np.arange(S.m), np.diff(S.rowptr)))
    cols = torch.tensor(S.colidx.astype(np.int64))
    M = torch.zeros(S.m, S.n, dtype=torch.bool)
    M[rows, cols] = True
    D = torch.zeros(S.m, S.n, dtype=torch.float64).index_put((rows, cols), vals)
    s, t = H @ a1, H @ a2
    E = torch.nn.functional.leaky_relu(D * (s[:, None] + t[None, :]), negative_slope=slope)
    if softmax:
        W = torch.nan_to_num(torch.softmax(E.masked_fill(~M, float("-inf")), dim=1), nan=0.0)
    else:
        W = E * M
    return W @ H


@pytest.mark.parametrize("softmax", [True, False])
@pytest.mark.parametrize("seed", [0, 1])
def test_gat_backward_vs_torch_autograd(softmax, seed):
    case = tiny_case(19, 19, 6, 0.35, seed=320 + seed)
    S, H = case["S"], case["A"]
    rng = np.random.default_rng(330 + seed)
    a1, a2 = rng.standard_normal(6), rng.standard_normal(6)
    dO = rng.standard_normal((19, 6))
    Ht = torch.tensor(H, requires_grad=True)
    a1t, a2t = torch.tensor(a1, requires_grad=True), torch.tensor(a2, requires_grad=True)
    vt = torch.tensor(np.asarray(S.val, np.float64), requires_grad=True)
    (_torch_head(S, Ht, a1t, a2t, vt, 0.2, softmax) * torch.tensor(dO)).sum().backward()
    dH, da1, da2, dS = oracle.gat_backward(S, H, a1, a2, dO, slope=0.2, softmax=softmax)
    for got, ref in ((dH, Ht.grad), (da1, a1t.grad), (da2, a2t.grad), (dS, vt.grad)):
        ref = ref.numpy()
        assert np.max(np.abs(got - ref)) <= 1e-11 * (1 + np.abs(ref).max())


def test_gat_backward_central_differences():
    S = er_exact_degree(40, 40, 5, seed=340, val_dtype=np.float64)
    rng = np.random.default_rng(341)
    H = rng.standard_normal((40, 4))
    a1, a2 = rng.standard_normal(4) * 0.5, rng.standard_normal(4) * 0.5
    dO = rng.standard_normal((40, 4))
    dH, da1, da2, dS = oracle.gat_backward(S, H, a1, a2, dO, slope=0.2, softmax=True)

    def loss():
        return float((oracle.gat_forward(S, H, a1, a2, slope=0.2, softmax=True) * dO).sum())

    h = 1e-6
    for X, dX in ((H, dH), (a1, da1), (a2, da2), (S.val, dS)):
        flat = X.reshape(-1)
        for k in rng.choice(flat.size, min(40, flat.size), replace=False):
            old = flat[k]
            flat[k] = old + h
            lp = loss()
            flat[k] = old - h
            lm = loss()
            flat[k] = old
            assert abs((lp - lm) / (2 * h) - dX.reshape(-1)[k]) <= 1e-6 * max(1.0, abs(dX.reshape(-1)[k]))


def test_gat_backward_softmax_rows_are_shift_invariant():
    """With the softmax and every stored value 1, a row's scores all carry the same s_i,
    which the softmax cancels while LeakyReLU stays on one branch: the output does not
    depend on s, so the gradient through it vanishes (da1 = 0 up to rounding).  Positive
    H and a2 shifted down keep every x_ij = s_i + t_j negative, with t still spread."""
    S = rmat(7, 6, seed=350)
    S1 = type(S)(S.m, S.n, S.rowptr, S.colidx, np.ones(S.nnz))
    rng = np.random.default_rng(351)
    H = rng.random((S.n, 5)) + 0.1
    a1 = 0.02 * rng.standard_normal(5)
    a2 = 0.02 * rng.standard_normal(5) - 1.5
    s, t = H @ a1, H @ a2
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    assert np.all(s[rows] + t[S.colidx] < 0) and np.ptp(t) > 1.0
    dO = rng.standard_normal((S.m, 5))
    _, da1, da2, _ = oracle.gat_backward(S1, H, a1, a2, dO, slope=0.2, softmax=True)
    assert np.max(np.abs(da1)) <= 1e-12 * (1 + np.abs(da2).max() + np.abs(H).sum())
    assert np.max(np.abs(da2)) > 1e-3


@pytest.mark.parametrize("softmax", [True, False])
def test_gat_adjoint_magnitudes_bound_rounding_sized_perturbations(softmax):
    """The attention adjoint's magnitude companions bound its first-order sensitivity:
    relative perturbations of size delta in every input (H, a1, a2, dO, the stored
    values) move each output by at most a small multiple of delta times its companion,
    element by element.  And a relative error of 1e-3 planted in an ordinary element of
    dH fails the 1e-5 componentwise gate (which a gate scaled by the hub rows would
    let through)."""
    from tests.gat_gate import gat_backward_magnitudes, kink_free
    from tests.gates import componentwise_error

    S0 = rmat(9, 8, seed=660, val_dtype=np.float64)
    r = 16
    H = dense_normal(S0.n, r, 661, dtype=np.float64)
    a1 = dense_normal(1, r, 662, sigma=r ** -0.5, dtype=np.float64)[0]
    a2 = dense_normal(1, r, 663, sigma=r ** -0.5, dtype=np.float64)[0]
    dO = dense_normal(S0.m, r, 664, dtype=np.float64)
    S, _ = kink_free(S0, H, a1, a2, margin=1e-3)
    ref = oracle.gat_backward(S, H, a1, a2, dO, softmax=softmax)
    mag = gat_backward_magnitudes(S, H, a1, a2, dO, softmax=softmax)
    rng = np.random.default_rng(665)
    delta = 1e-8

    def jig(x):
        return x * (1.0 + delta * rng.uniform(-1.0, 1.0, np.shape(x)))

    worst = 0.0
    for _ in range(4):
        Sp = type(S)(S.m, S.n, S.rowptr, S.colidx, jig(S.val))
        got = oracle.gat_backward(Sp, jig(H), jig(a1), jig(a2), jig(dO), softmax=softmax)
        for g, e, mg in zip(got, ref, mag):
            worst = max(worst, componentwise_error(g, e, mg) / delta)
    assert worst <= 4.0, worst
    # a planted error in an ordinary row (one of the lower half by max |dH|, at its
    # best-conditioned element) is found
    dH, dHm = ref[0], mag[0]
    low = np.argsort(np.abs(dH).max(axis=1))[: S.n // 2]
    ratio = np.where(dH[low] != 0, dHm[low] / np.maximum(np.abs(dH[low]), 1e-300), np.inf)
    t, k = np.unravel_index(int(np.argmin(ratio)), ratio.shape)
    j = int(low[t])
    bad = dH.copy()
    bad[j, k] *= 1.0 + 1e-3
    assert componentwise_error(bad, dH, dHm) > 1e-5
    assert np.abs(bad - dH).max() <= 1e-5 * np.abs(dH).max()  # the max-norm gate would pass it


def test_kink_free_zeroes_only_near_kink_entries():
    from tests.gat_gate import kink_free

    S = rmat(10, 8, seed=670)
    r = 8
    H = dense_normal(S.n, r, 671)
    a1 = dense_normal(1, r, 672, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 673, sigma=r ** -0.5)[0]
    K, k = kink_free(S, H, a1, a2, margin=1e-2)
    s, t = oracle.gat_scores(H, a1, a2)
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    score = s[rows] + t[S.colidx]
    changed = K.val != S.val
    assert k == int(changed.sum()) > 0 and np.all(K.val[changed] == 0)
    assert np.array_equal(K.rowptr, S.rowptr) and np.array_equal(K.colidx, S.colidx)
    assert np.abs(score[changed]).max() < np.abs(score[~changed]).max()
