"""Seeded synthetic inputs: determinism and structural properties."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

from workloads import batch_er, content_hash, dense_normal, er_exact_degree, rmat, workload


def _canonical(S):
    rp = S.rowptr.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == S.nnz and np.all(np.diff(rp) >= 0)
    assert S.colidx.dtype == np.int32 and S.rowptr.dtype == np.int32
    if S.nnz:
        assert S.colidx.min() >= 0 and S.colidx.max() < S.n
    rows = np.repeat(np.arange(S.m), np.diff(rp))
    same = rows[1:] == rows[:-1]
    assert np.all(np.diff(S.colidx.astype(np.int64))[same] > 0)  # strictly increasing in a row


def test_er_exact_degree_structure_and_determinism():
    for (m, n, d) in [(1000, 5000, 32), (64, 64, 64), (50, 40, 30), (10, 1, 1), (7, 9, 0)]:
        S = er_exact_degree(m, n, d, seed=9)
        _canonical(S)
        assert np.all(np.diff(S.rowptr) == d)
        assert S.val.dtype == np.float32 and np.all((S.val >= 0) & (S.val < 1))
        S2 = er_exact_degree(m, n, d, seed=9)
        assert content_hash(S.rowptr, S.colidx, S.val) == content_hash(S2.rowptr, S2.colidx, S2.val)
    S3 = er_exact_degree(1000, 5000, 32, seed=10)
    assert not np.array_equal(S3.colidx, er_exact_degree(1000, 5000, 32, seed=9).colidx)


def test_er_columns_roughly_uniform():
    S = er_exact_degree(4096, 256, 32, seed=1)
    counts = np.bincount(S.colidx, minlength=256)
    exp = S.nnz / 256
    assert np.abs(counts - exp).max() < 6 * np.sqrt(exp)


def test_rmat_structure():
    S = rmat(12, 16, seed=3)
    _canonical(S)
    assert S.m == S.n == 4096
    assert S.nnz <= 16 * 4096 and S.nnz > 0.75 * 16 * 4096
    lens = S.row_lengths()
    assert S.meta["empty_rows"] == int((lens == 0).sum()) and S.meta["max_row"] == int(lens.max())
    assert lens.max() > 20 * lens.mean()  # skewed
    S2 = rmat(12, 16, seed=3)
    assert content_hash(S.rowptr, S.colidx, S.val) == content_hash(S2.rowptr, S2.colidx, S2.val)


def test_batch_ranges():
    gs = batch_er(12, 8, seed=5, nmin=64, nmax=1024, dmin=8, dmax=64)
    for g in gs:
        S = g["S"]
        _canonical(S)
        assert 64 <= S.m <= 1024 and S.m == S.n
        d = np.diff(S.rowptr)
        assert np.all(d == d[0]) and 8 <= d[0] <= 64
        assert g["A"].shape == (S.m, 8) and g["B"].shape == (S.n, 8)


def test_dense_normal_sigma_and_workload_shapes():
    x = dense_normal(2000, 64, 1, sigma=256 ** -0.25)
    assert abs(x.std() - 0.25) < 0.01 and x.dtype == np.float32
    w = workload("er4096_d32_r32")
    assert w["S"].nnz == 131072 and w["A"].shape == (4096, 32) and w["B"].shape == (4096, 32)
    w = workload("fd256_d8_r8", dtype=np.float64)
    assert w["S"].nnz == 2048 and w["A"].dtype == np.float64 and w["S"].val.dtype == np.float64


_PROPS = settings(max_examples=80, deadline=None, derandomize=True)


@_PROPS
@given(st.integers(1, 40), st.integers(1, 60), st.data())
def test_er_exact_degree_properties(m, n, data):
    """Any (m, n, d <= n, seed): exactly d distinct, strictly increasing, in-range columns
    per row, values in [0, 1), and the same seed gives the same matrix."""
    d = data.draw(st.integers(0, n))
    seed = data.draw(st.integers(0, 2 ** 31 - 1))
    S = er_exact_degree(m, n, d, seed=seed)
    assert np.array_equal(np.diff(S.rowptr), np.full(m, d))
    cols = S.colidx.reshape(m, d) if d else np.zeros((m, 0), np.int32)
    assert (np.diff(cols, axis=1) > 0).all() and ((cols >= 0) & (cols < n)).all()
    assert ((S.val >= 0) & (S.val < 1)).all()
    T = er_exact_degree(m, n, d, seed=seed)
    assert np.array_equal(T.colidx, S.colidx) and np.array_equal(T.val, S.val)


@_PROPS
@given(st.integers(1, 9), st.integers(1, 8), st.integers(0, 2 ** 31 - 1))
def test_rmat_properties(scale, ef, seed):
    """Any small R-MAT: a canonical CSR (strictly increasing columns, no duplicates) on
    2**scale vertices with at most ef * 2**scale entries."""
    S = rmat(scale, ef, seed=seed)
    n = 1 << scale
    assert S.m == S.n == n and S.rowptr[0] == 0 and S.rowptr[-1] == S.colidx.size <= ef * n
    assert (np.diff(S.rowptr) >= 0).all() and ((S.colidx >= 0) & (S.colidx < n)).all()
    for i in range(n):
        row = S.colidx[S.rowptr[i]:S.rowptr[i + 1]]
        assert (np.diff(row) > 0).all()


def test_workload_cache_gives_the_same_arrays(tmp_path, monkeypatch):
    from workloads import workload

    fresh = workload("er4096_d32_r32")
    monkeypatch.setenv("FMM_WORKLOAD_CACHE", str(tmp_path))
    first, again = workload("er4096_d32_r32"), workload("er4096_d32_r32")  # writes, then maps
    for w in (first, again):
        for k in ("rowptr", "colidx", "val"):
            assert np.array_equal(np.asarray(getattr(w["S"], k)), np.asarray(getattr(fresh["S"], k)))
        for k in "ABG":
            assert w[k].dtype == fresh[k].dtype and np.array_equal(w[k], fresh[k])
        assert w["r"] == fresh["r"] and w["S"].m == fresh["S"].m and w["S"].nnz == fresh["S"].nnz
