"""Componentwise gate for the adjoint of the graph-attention head (Section VI-E).

The adjoint's outputs are sums of signed terms, so each output gets a magnitude
companion: the same chain-rule steps as oracle.gat_backward, taken on absolute values
with every difference turned into a sum, plus the first-order sensitivity of the
weights to rounding in the scores.  With x_ij = S_ij (s_i + t_j) the scores carry an
error of order u * xbar_ij, xbar_ij = |S_ij| (sbar_i + tbar_j), sbar = |H||a1|,
tbar = |H||a2|; a softmax weight w_ij = exp(e_ij) / sum_k exp(e_ik) then moves by at
most w_ij (xbar_ij + sum_k w_ik xbar_ik) times that order (its derivative is
w_ij (delta_jk - w_ik)).  The companions:

    wbar_ij  = w_ij (1 + xbar_ij + Xbar_i), Xbar_i = sum_k w_ik xbar_ik   (softmax)
             = xbar_ij                                                    (no softmax: w = e)
    dwbar_ij = <|dO_i|, |H_j|>
    debar_ij = wbar_ij |dw_ij - D_i| + w_ij (dwbar_ij + Dbar_i),
               Dbar_i = sum_k (wbar_ik |dw_ik| + w_ik dwbar_ik)           (softmax)
             = dwbar_ij                                                   (no softmax)
    dxbar    = debar                                  (LeakyReLU's slope is at most 1)
    dSbar_ij = dxbar_ij (sbar_i + tbar_j)
    gbar_ij  = dxbar_ij |S_ij|,  dsbar_i = sum_j gbar_ij,  dtbar_j = sum_i gbar_ij
    dHbar    = (W + Wbar)^T |dO| + dsbar |a1|^T + dtbar |a2|^T
    da1bar   = |H|^T dsbar,  da2bar = |H|^T dtbar

These are first-order bounds: de = w (dw - D) moves by dw (dw - D) + w (ddw - dD), and
D = sum_k w_ik dw_ik by sum_k (dw_ik dw_ik + w_ik ddw_ik), with the exact dw and D of
the oracle in place of the perturbed ones.

LeakyReLU's derivative jumps at x = 0, and an entry whose x lies within rounding
distance of 0 may take either branch in float32; kink_free() gives such entries the
stored value 0 (kept in the pattern), so that x is exactly 0 on every path and both
sides take the same branch.
"""
import numpy as np

import oracle


def _rows_of(S):
    return np.repeat(np.arange(S.m), np.diff(np.asarray(S.rowptr, np.int64)))


def kink_free(S, H, a1, a2, margin=1e-5):
    """S with the stored value 0 at every entry whose score s_i + t_j is within
    margin * (sbar_i + tbar_j) of 0 (the pattern and every other value unchanged);
    returns (pattern, number of entries zeroed)."""
    from workloads import CsrPattern

    s, t = oracle.gat_scores(H, a1, a2)
    sb, tb = oracle.gat_scores(np.abs(np.asarray(H, np.float64)), np.abs(a1), np.abs(a2))
    rows, cols = _rows_of(S), np.asarray(S.colidx, np.int64)
    near = np.abs(s[rows] + t[cols]) <= margin * (sb[rows] + tb[cols])
    val = np.array(S.val, copy=True)
    val[near] = 0
    return CsrPattern(S.m, S.n, S.rowptr, S.colidx, val), int(near.sum())


def gat_backward_magnitudes(S, H, a1, a2, dO, slope=0.2, softmax=True):
    """Magnitude companions (dH, da1, da2, dS) of oracle.gat_backward's outputs."""
    H, dO = np.asarray(H, np.float64), np.asarray(dO, np.float64)
    a1, a2 = np.asarray(a1, np.float64), np.asarray(a2, np.float64)
    rows, cols = _rows_of(S), np.asarray(S.colidx, np.int64)
    v = np.abs(np.asarray(S.val, np.float64))
    s, t = oracle.gat_scores(H, a1, a2)
    sb, tb = oracle.gat_scores(np.abs(H), np.abs(a1), np.abs(a2))
    xbar = v * (sb[rows] + tb[cols])
    dwbar = oracle.sddmm(S, np.abs(dO), np.abs(H), val=None)
    if softmax:
        w = oracle.gat_edges(S, s, t, slope, True)
        dw = oracle.sddmm(S, dO, H, val=None)
        Xbar = np.zeros(S.m)
        np.add.at(Xbar, rows, w * xbar)
        wbar = w * (1.0 + xbar + Xbar[rows])
        D, Dbar = np.zeros(S.m), np.zeros(S.m)
        np.add.at(D, rows, w * dw)
        np.add.at(Dbar, rows, wbar * np.abs(dw) + w * dwbar)
        debar = wbar * np.abs(dw - D[rows]) + w * (dwbar + Dbar[rows])
        wsum = w + wbar
    else:
        wbar = xbar
        debar = dwbar
        wsum = wbar
    gbar = debar * v
    dsb, dtb = np.zeros(S.n), np.zeros(S.n)
    np.add.at(dsb, rows, gbar)
    np.add.at(dtb, cols, gbar)
    dH = oracle.spmm_b(S, wsum, np.abs(dO)) + np.outer(dsb, np.abs(a1)) + np.outer(dtb, np.abs(a2))
    return dH, np.abs(H).T @ dsb, np.abs(H).T @ dtb, debar * (sb[rows] + tb[cols])
