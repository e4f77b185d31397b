"""Componentwise error gate shared by the parity tests.

err(X) = max_e |X_gpu[e] - X_ref[e]| / Xm[e], where Xm is the reference computed
on absolute values of every input (the magnitude companion).  For a dot product
the textbook bound |fl(x.y) - x.y| <= gamma_r |x|.|y| makes this the quantity
rounding error is bounded by; where Xm[e] == 0 the GPU value must be exactly 0.
"""
import numpy as np

TOL_F32 = 1e-5
TOL_BF16 = 2e-2
TOL_F64 = 1e-12


def componentwise_error(x, ref, mag):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mag = np.asarray(mag, dtype=np.float64)
    assert x.shape == ref.shape == mag.shape, (x.shape, ref.shape, mag.shape)
    if x.size == 0:
        return 0.0
    zero = mag == 0
    if np.any(x[zero] != 0):
        return float("inf")
    if not np.all(np.isfinite(x)):
        return float("inf")
    diff = np.abs(x - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(zero, 0.0, diff / np.where(zero, 1.0, mag))
    return float(rel.max())


def normwise_error(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))
