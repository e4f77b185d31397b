"""Shared helpers for the GPU parity tests: device upload, oracle references with
their magnitude companions, and the componentwise gate."""
import sys

import numpy as np
import torch

import oracle
from tests.gates import componentwise_error, normwise_error


def log(msg):
    """Name the case on stdout before a GPU step, so a failed run still says which."""
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu").to(torch.float64).numpy()


def gate(name, got, ref, mag, tol):
    err = componentwise_error(got, ref, mag)
    nerr = normwise_error(got, ref)
    assert err <= tol, f"{name}: componentwise error {err:.3e} > {tol:.1e} (normwise {nerr:.3e})"
    return err


def abs_pattern(S):
    return oracle.absolute(S)


def ref_fusedmm_a(S, A, B, rows=None):
    """Oracle FusedMMA and its magnitude companion (the same definition on |.|)."""
    ref = oracle.fusedmm_a(S, A, B, rows=rows)
    mag = oracle.fusedmm_a(oracle.absolute(S), np.abs(A), np.abs(B), rows=rows)
    return ref, mag


def ref_fusedmm_b(S, A, B, ST=None, cols=None):
    if cols is None:
        ref = oracle.fusedmm_b(S, A, B)
        mag = oracle.fusedmm_b(oracle.absolute(S), np.abs(A), np.abs(B))
        return ref, mag
    ref = oracle.fusedmm_b_cols(ST, A, B, cols)
    mag = oracle.fusedmm_b_cols(oracle.absolute(ST), np.abs(A), np.abs(B), cols)
    return ref, mag


def ref_sddmm(S, A, B):
    return oracle.sddmm(S, A, B), oracle.sddmm(oracle.absolute(S), np.abs(A), np.abs(B))


def ref_fusedmm_a_backward(S, A, B, dC):
    dA, dB = oracle.fusedmm_a_backward(S, A, B, dC)
    mA, mB = oracle.fusedmm_a_backward(oracle.absolute(S), np.abs(A), np.abs(B), np.abs(dC))
    return dA, dB, mA, mB


def ref_fusedmm_b_backward(S, A, B, dC):
    dA, dB = oracle.fusedmm_b_backward(S, A, B, dC)
    mA, mB = oracle.fusedmm_b_backward(oracle.absolute(S), np.abs(A), np.abs(B), np.abs(dC))
    return dA, dB, mA, mB
