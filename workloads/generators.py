"""Seeded generators for the sparse patterns and dense factors of the FusedMM workloads.

The paper evaluates on Erdos-Renyi matrices with a fixed number of nonzeros per
row (Section VI-B, weak scaling setup 1) and on power-law real-world graphs
(Section VI-D, Table 5).  The real-world matrices are replaced here by R-MAT
graphs, whose skewed degree distribution stands in for theirs.  Every array is
drawn from numpy's PCG64 with an explicit seed, so a run is reproducible.

Conventions shared by every generator:
  * CSR with int32 ``rowptr[m+1]`` and ``colidx[nnz]``; the columns of a row are
    strictly increasing (no duplicates), which is the canonical form the kernels
    and the oracle both assume.
  * ``val`` holds the values of S in CSR order.
  * dense factors are row-major ``(rows, r)`` arrays.
"""

from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class CsrPattern:
    """A sparse matrix S (m x n) in canonical CSR form."""

    m: int
    n: int
    rowptr: np.ndarray  # int32 [m+1]
    colidx: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float32 or float64 [nnz]
    meta: Dict[str, object] = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colidx.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def _rowptr_from_sorted_rows(rows: np.ndarray, m: int) -> np.ndarray:
    counts = np.bincount(rows, minlength=m).astype(np.int64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return rowptr.astype(np.int32)


def _distinct_sorted_columns(rng: np.random.Generator, m: int, n: int, d: int) -> np.ndarray:
    """(m, d) int32 array: each row holds d distinct columns of [0, n), ascending,
    every d-subset equally likely."""
    if d > n:
        raise ValueError(f"cannot place {d} distinct columns in {n}")
    if d == 0 or m == 0:
        return np.zeros((m, d), dtype=np.int32)
    if m * n <= (1 << 22) or 4 * d > n:
        # small or dense rows: rank random keys and keep the d smallest
        out = np.empty((m, d), dtype=np.int32)
        step = max(1, (1 << 22) // n)
        for r0 in range(0, m, step):
            keys = rng.random((min(step, m - r0), n))
            sel = np.argpartition(keys, d - 1, axis=1)[:, :d] if d < n else np.argsort(keys, axis=1)
            out[r0:r0 + sel.shape[0]] = np.sort(sel, axis=1)
        return out
    # sparse rows: draw with replacement, redraw the rows that collided
    cols = rng.integers(0, n, size=(m, d), dtype=np.int32)
    cols.sort(axis=1)
    bad = np.flatnonzero((np.diff(cols, axis=1) == 0).any(axis=1))
    while bad.size:
        redo = rng.integers(0, n, size=(bad.size, d), dtype=np.int32)
        redo.sort(axis=1)
        cols[bad] = redo
        still = (np.diff(redo, axis=1) == 0).any(axis=1)
        bad = bad[still]
    return cols


def er_exact_degree(m: int, n: int, d: int, seed: int, val_dtype=np.float32) -> CsrPattern:
    """Erdos-Renyi-style S with exactly ``d`` distinct uniform columns per row and
    values U(0,1): the matrices of the paper's weak-scaling runs (Section VI-B)."""
    rng = np.random.default_rng(seed)
    cols = _distinct_sorted_columns(rng, m, n, d)
    rowptr = (np.arange(m + 1, dtype=np.int64) * d).astype(np.int32)
    val = rng.random(m * d, dtype=np.float64).astype(val_dtype)
    return CsrPattern(m, n, rowptr, cols.reshape(-1), val,
                      meta={"kind": "er", "d": d, "seed": seed})


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, val_dtype=np.float32) -> CsrPattern:
    """R-MAT graph on 2**scale vertices with edge_factor * 2**scale generated edges.

    Each edge descends ``scale`` levels of the recursive quadrant split with
    probabilities (a, b, c, 1-a-b-c), with no noise.  Self-loops are kept, edges are
    directed, and a seeded random vertex relabelling is applied (the paper permutes
    rows and columns to balance load, Section VI); duplicate edges are then removed,
    and values U(0,1) are drawn in CSR order.
    """
    n = 1 << scale
    E = edge_factor * n
    rng = np.random.default_rng(seed)
    rows = np.zeros(E, dtype=np.int64)
    cols = np.zeros(E, dtype=np.int64)
    ab, abc = a + b, a + b + c
    chunk = 1 << 23
    for e0 in range(0, E, chunk):
        e1 = min(E, e0 + chunk)
        rr = np.zeros(e1 - e0, dtype=np.int64)
        cc = np.zeros(e1 - e0, dtype=np.int64)
        for level in range(scale):
            u = rng.random(e1 - e0, dtype=np.float64)
            rbit = u >= ab
            cbit = ((u >= a) & (u < ab)) | (u >= abc)
            rr = (rr << 1) | rbit
            cc = (cc << 1) | cbit
        rows[e0:e1] = rr
        cols[e0:e1] = cc
    relabel = rng.permutation(n).astype(np.int64)
    key = (relabel[rows] << scale) | relabel[cols]
    del rows, cols
    key = np.unique(key)
    rr = (key >> scale).astype(np.int64)
    cc = (key & (n - 1)).astype(np.int32)
    rowptr = _rowptr_from_sorted_rows(rr, n)
    val = rng.random(cc.shape[0], dtype=np.float64).astype(val_dtype)
    lens = np.diff(rowptr.astype(np.int64))
    meta = {"kind": "rmat", "scale": scale, "edge_factor": edge_factor, "seed": seed,
            "abcd": (a, b, c, 1.0 - a - b - c), "generated_edges": E,
            "empty_rows": int((lens == 0).sum()), "max_row": int(lens.max(initial=0))}
    return CsrPattern(n, n, rowptr, cc, val, meta=meta)


def dense_normal(rows: int, r: int, seed: int, sigma: float = 1.0, dtype=np.float32) -> np.ndarray:
    """Row-major (rows, r) matrix with entries N(0, sigma^2)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((rows, r), dtype=np.float32 if dtype == np.float32 else np.float64)
    if sigma != 1.0:
        x *= np.asarray(sigma, dtype=x.dtype)
    return np.ascontiguousarray(x.astype(dtype, copy=False))


def batch_er(nbatch: int, r: int, seed: int, nmin: int = 1024, nmax: int = 65536,
             dmin: int = 8, dmax: int = 64) -> List[dict]:
    """``nbatch`` independent square ER graphs: n_g log-uniform on [nmin, nmax]
    (rounded), degree d_g uniform on {dmin..dmax}, each with its own A_g, B_g, G_g."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), nbatch))).astype(np.int64)
    ds = rng.integers(dmin, dmax + 1, size=nbatch)
    child = rng.integers(0, 2**62, size=(nbatch, 4))
    out = []
    for g in range(nbatch):
        n, d = int(ns[g]), int(ds[g])
        S = er_exact_degree(n, n, d, seed=int(child[g, 0]))
        out.append({
            "S": S,
            "A": dense_normal(n, r, int(child[g, 1])),
            "B": dense_normal(n, r, int(child[g, 2])),
            "G": dense_normal(n, r, int(child[g, 3])),
        })
    return out


def tiny_case(m: int, n: int, r: int, density: float, seed: int, dtype=np.float64) -> dict:
    """Small random S of roughly the given density (each entry kept independently),
    with A (m x r), B (n x r) N(0,1) and G (m x r) N(0,1), for brute-force checks."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    rowptr = _rowptr_from_sorted_rows(rows.astype(np.int64), m) if m else np.zeros(1, np.int32)
    val = rng.random(rows.shape[0]).astype(dtype)
    S = CsrPattern(m, n, rowptr, cols.astype(np.int32), val,
                   meta={"kind": "tiny", "density": density, "seed": seed})
    A = rng.standard_normal((m, r)).astype(dtype)
    B = rng.standard_normal((n, r)).astype(dtype)
    G = rng.standard_normal((m, r)).astype(dtype)
    return {"S": S, "A": A, "B": B, "G": G}


# The paper-shaped workloads, named by what they are.  Seeds are fixed per workload.
WORKLOADS = {
    # ER 4096 x 4096, 32 per row, r = 32 fp32: the small case checked in full.
    "er4096_d32_r32": dict(kind="er", m=4096, n=4096, d=32, r=32, seed=1, sigma=1.0),
    # ER 2^20 x 2^20, 32 per row, r = 128 fp32 (paper: 32 nonzeros per row, Section VI-B).
    "er1m_d32_r128": dict(kind="er", m=1 << 20, n=1 << 20, d=32, r=128, seed=2, sigma=1.0),
    # R-MAT scale 22, edge factor 16, r = 256, factors N(0, variance 1/sqrt(r)).
    "rmat22_ef16_r256": dict(kind="rmat", scale=22, ef=16, r=256, seed=3, sigma=256 ** -0.25),
    # R-MAT scale 20, edge factor 16, r = 64 fp32, used for the adjoint.
    "rmat20_ef16_r64": dict(kind="rmat", scale=20, ef=16, r=64, seed=4, sigma=1.0),
    # finite-difference case: 256 x 256, 8 per row, r = 8, fp64.
    "fd256_d8_r8": dict(kind="er", m=256, n=256, d=8, r=8, seed=6, sigma=1.0),
}


def workload(name: str, dtype=np.float32, scale_override: Optional[int] = None) -> dict:
    """Pattern S plus dense A (m x r), B (n x r) and upstream gradient G (m x r).

    With the environment variable FMM_WORKLOAD_CACHE naming a directory, the arrays are
    saved there on first use and memory-mapped on later calls (profiling runs that start
    many processes on one workload); the arrays are the same either way."""
    cache = os.environ.get("FMM_WORKLOAD_CACHE")
    if cache and scale_override is None:
        d = os.path.join(cache, f"{name}_{np.dtype(dtype).name}")
        keys = ("rowptr", "colidx", "val", "A", "B", "G")
        if os.path.exists(os.path.join(d, "done")):
            with open(os.path.join(d, "meta.json")) as fh:
                meta = json.load(fh)
            arr = {k: np.load(os.path.join(d, k + ".npy"), mmap_mode="r") for k in keys}
            S = CsrPattern(meta["m"], meta["n"], arr["rowptr"], arr["colidx"], arr["val"], meta=meta["meta"])
            return {"name": name, "S": S, "A": arr["A"], "B": arr["B"], "G": arr["G"], "r": meta["r"],
                    "sigma": meta["sigma"]}
        w = _generate(name, dtype)
        os.makedirs(d, exist_ok=True)
        S = w["S"]
        for k, a in zip(keys, (S.rowptr, S.colidx, S.val, w["A"], w["B"], w["G"])):
            np.save(os.path.join(d, k + ".npy"), np.ascontiguousarray(a))
        with open(os.path.join(d, "meta.json"), "w") as fh:
            json.dump({"m": S.m, "n": S.n, "r": w["r"], "sigma": w["sigma"], "meta": S.meta}, fh)
        open(os.path.join(d, "done"), "w").close()
        return w
    return _generate(name, dtype, scale_override)


def _generate(name: str, dtype=np.float32, scale_override: Optional[int] = None) -> dict:
    w = dict(WORKLOADS[name])
    seed = w["seed"]
    if w["kind"] == "er":
        S = er_exact_degree(w["m"], w["n"], w["d"], seed=seed,
                            val_dtype=np.float64 if dtype == np.float64 else np.float32)
    else:
        scale = scale_override if scale_override is not None else w["scale"]
        S = rmat(scale, w["ef"], seed=seed,
                 val_dtype=np.float64 if dtype == np.float64 else np.float32)
    r = w["r"]
    A = dense_normal(S.m, r, seed * 1000 + 1, sigma=w["sigma"], dtype=dtype)
    B = dense_normal(S.n, r, seed * 1000 + 2, sigma=w["sigma"], dtype=dtype)
    G = dense_normal(S.m, r, seed * 1000 + 3, dtype=dtype)
    return {"name": name, "S": S, "A": A, "B": B, "G": G, "r": r, "sigma": w["sigma"]}


def content_hash(*arrays: np.ndarray) -> str:
    """SHA-256 over dtype, shape and bytes of each array in order."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
