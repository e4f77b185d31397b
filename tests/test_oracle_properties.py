"""Property-based pins for the FP64 oracle (hypothesis, derandomized so every run checks
the same cases): on random small patterns, empty ones included, the oracle agrees with
dense brute force for FusedMMA and FusedMMB (Section II); its CSR -> CSC conversion is
the dense transpose and round-trips; and its adjoint satisfies the directional
derivative identity <dA, V> + <dB, W> = d/dt <G, FusedMM(S, A + tV, B + tW)> at t = 0,
where the five-point central difference is exact up to rounding (the loss is a
polynomial of degree <= 3 in t: linear in A, quadratic in B)."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from workloads import CsrPattern

SETTINGS = settings(max_examples=200, deadline=None, derandomize=True)


@st.composite
def problems(draw):
    m = draw(st.integers(1, 9))
    n = draw(st.integers(1, 9))
    r = draw(st.integers(1, 5))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    density = draw(st.sampled_from([0.0, 0.2, 0.5, 1.0]))
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)  # row-major order: CSR with increasing columns per row
    rowptr = np.zeros(m + 1, np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    val = rng.uniform(-1.0, 1.0, rows.size)
    S = CsrPattern(m, n, rowptr, cols.astype(np.int32), val)
    A = rng.standard_normal((m, r))
    B = rng.standard_normal((n, r))
    G = rng.standard_normal((m, r))
    return S, A, B, G, rng


def _dense(S):
    D = np.zeros((S.m, S.n))
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    D[rows, S.colidx] = S.val
    return D


def _close(got, want, tol=1e-11):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    assert got.shape == want.shape
    if got.size:
        scale = max(1.0, float(np.abs(want).max()))
        assert float(np.abs(got - want).max()) <= tol * scale


@SETTINGS
@given(problems())
def test_fusedmm_matches_dense_bruteforce(p):
    S, A, B, _, _ = p
    R = _dense(S) * (A @ B.T)  # the sampled product, zero off the pattern
    _close(oracle.fusedmm_a(S, A, B), R @ B)
    _close(oracle.fusedmm_b(S, A, B), R.T @ A)


@SETTINGS
@given(problems())
def test_transpose_is_dense_transpose_and_round_trips(p):
    S, _, _, _, _ = p
    ST = oracle.transpose(S)
    assert (ST.m, ST.n) == (S.n, S.m)
    _close(_dense(ST), _dense(S).T, tol=0.0)
    back = oracle.transpose(ST)
    assert np.array_equal(back.rowptr, S.rowptr) and np.array_equal(back.colidx, S.colidx)
    assert np.array_equal(back.val, S.val)


@SETTINGS
@given(problems())
def test_adjoint_directional_derivative(p):
    S, A, B, G, rng = p
    V, W = rng.standard_normal(A.shape), rng.standard_normal(B.shape)
    Gb = rng.standard_normal((S.n, A.shape[1]))
    for fwd, bwd, Gf in ((oracle.fusedmm_a, oracle.fusedmm_a_backward, G),
                         (oracle.fusedmm_b, oracle.fusedmm_b_backward, Gb)):
        dA, dB = bwd(S, A, B, Gf)
        lhs = float(np.sum(dA * V) + np.sum(dB * W))

        def loss(t):
            return float(np.sum(Gf * fwd(S, A + t * V, B + t * W)))
        h = 0.5  # d/dt at 0 from values at +-h and +-2h: the five-point stencil, exact for cubics
        rhs = (8 * (loss(h) - loss(-h)) - (loss(2 * h) - loss(-2 * h))) / (12 * h)
        assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs), abs(rhs)), fwd.__name__


@SETTINGS
@given(problems())
def test_value_gradient_is_exact_difference(p):
    """<G, FusedMMA(S, A, B)> is linear in S's stored values, so <dS, D> equals the plain
    difference of the loss along D (and the same for FusedMMB with an n x r gradient)."""
    S, A, B, G, rng = p
    D = rng.standard_normal(S.val.shape)
    Sd = CsrPattern(S.m, S.n, S.rowptr, S.colidx, S.val + D)
    for form, fwd, grad, Gf in (("a", oracle.fusedmm_a, oracle.fusedmm_a_backward_values, G),
                                ("b", oracle.fusedmm_b, oracle.fusedmm_b_backward_values,
                                 rng.standard_normal((S.n, A.shape[1])))):
        dS = grad(S, A, B, Gf)
        lhs = float(np.sum(dS * D))
        rhs = float(np.sum(Gf * fwd(Sd, A, B)) - np.sum(Gf * fwd(S, A, B)))
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs), abs(rhs)), form


@SETTINGS
@given(problems())
def test_primitive_adjoints_are_transposes(p):
    """Each primitive is linear in every argument, so its adjoint is exact against the
    forward along random directions (the dot-product test <y, J x> = <J^T y, x>)."""
    S, A, B, G, rng = p
    r = A.shape[1]
    nnz = S.val.shape[0]
    dR = rng.standard_normal(nnz)
    w = rng.standard_normal(nnz)
    Gb = rng.standard_normal((S.n, r))
    V, W, dw = rng.standard_normal(A.shape), rng.standard_normal(B.shape), rng.standard_normal(nnz)

    def check(lhs, rhs):
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs), abs(rhs))
    # SDDMM: bilinear in (A, B); the loss <dR, R> is quadratic, so a central difference is exact
    gA, gB = oracle.sddmm_backward(S, A, B, dR)

    def sd(t):
        return float(np.sum(dR * oracle.sddmm(S, A + t * V, B + t * W)))
    check(float(np.sum(gA * V) + np.sum(gB * W)), (sd(0.5) - sd(-0.5)) / 1.0)
    # SpMMA: C = W(w) B, linear in w and in B
    gw, gB = oracle.spmm_a_backward(S, w, B, G)
    check(float(np.sum(gw * dw)), float(np.sum(G * oracle.spmm_a(S, dw, B))))
    check(float(np.sum(gB * W)), float(np.sum(G * oracle.spmm_a(S, w, W))))
    # SpMMB: C' = W(w)^T A, linear in w and in A
    gw, gA = oracle.spmm_b_backward(S, w, A, Gb)
    check(float(np.sum(gw * dw)), float(np.sum(Gb * oracle.spmm_b(S, dw, A))))
    check(float(np.sum(gA * V)), float(np.sum(Gb * oracle.spmm_b(S, w, V))))


@st.composite
def attention_problems(draw):
    n = draw(st.integers(1, 7))
    r = draw(st.integers(1, 4))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    density = draw(st.sampled_from([0.3, 0.6, 1.0]))
    softmax = draw(st.booleans())
    rng = np.random.default_rng(seed)
    rows, cols = np.nonzero(rng.random((n, n)) < density)
    rowptr = np.cumsum(np.concatenate([[0], np.bincount(rows, minlength=n)])).astype(np.int32)
    S = CsrPattern(n, n, rowptr, cols.astype(np.int32), rng.uniform(0.5, 1.5, rows.size))
    return S, rng.standard_normal((n, r)), rng.standard_normal(r), rng.standard_normal(r), \
        rng.standard_normal((n, r)), softmax, rng


@SETTINGS
@given(attention_problems())
def test_attention_adjoint_directional_derivative(p):
    """The attention head's adjoint (dH, da1, da2, dS) against a five-point central
    difference of <dO, out> along random directions in H, a1, a2 and S's values.  The head
    is smooth away from LeakyReLU's kink, so examples with a score within reach of 0 are
    skipped."""
    from hypothesis import assume

    S, H, a1, a2, dO, softmax, rng = p
    h = 1e-3
    V, u1, u2 = rng.standard_normal(H.shape), rng.standard_normal(a1.shape), rng.standard_normal(a2.shape)
    dv = rng.standard_normal(S.val.shape)
    s, t = oracle.gat_scores(H, a1, a2)
    rows = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    x = S.val * (s[rows] + t[S.colidx])
    assume(x.size == 0 or np.min(np.abs(x)) > 0.05)
    dH, da1, da2, dS = oracle.gat_backward(S, H, a1, a2, dO, softmax=softmax)
    lhs = float(np.sum(dH * V) + np.sum(da1 * u1) + np.sum(da2 * u2) + np.sum(dS * dv))

    def loss(e):
        St = CsrPattern(S.m, S.n, S.rowptr, S.colidx, S.val + e * dv)
        return float(np.sum(dO * oracle.gat_forward(St, H + e * V, a1 + e * u1, a2 + e * u2, softmax=softmax)))
    rhs = (8 * (loss(h) - loss(-h)) - (loss(2 * h) - loss(-2 * h))) / (12 * h)
    assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(lhs)), (lhs, rhs)
