"""GPU parity at full workload size under every launch configuration the benchmark's
autotuner can choose: batch depth (deep, medium, shallow) x split threshold (none, 256,
128, 64) x line order (off, on), set on both orientations, and then the configuration
the autotuner itself picks.  Outputs are checked on seeded samples of rows (FusedMMA,
dA) and columns (dB), which the oracle computes exactly."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from paper_2203_07673_amd import _capi as CA
from tests.gates import TOL_BF16, TOL_F32
from tests.gpu_helpers import dev, gate, host, log
from tests.test_gpu_full import _f64, _sample_lines
from workloads import workload

pytestmark = pytest.mark.gpu

NO_SPLIT = 1 << 30
VARIANTS = (CA.FMM_VARIANT_DEEP, CA.FMM_VARIANT_MEDIUM, CA.FMM_VARIANT_SHALLOW)


def _configure(P, variant, long_len, order):
    for o in (CA.FMM_CSR, CA.FMM_CSC):
        P.set_split(o, long_len if long_len is not None else NO_SPLIT)
        P.set_line_order(o, order)
    P.set_variant(variant, variant)


def _check_all(name, w, dtypes, k):
    S = w["S"]
    log(f"{name}: m={S.m} nnz={S.nnz} r={w['r']}")
    P = F.Pattern.from_csr(S)
    ST = oracle.transpose(S)
    rows = _sample_lines(S.rowptr, k, 11)
    cols = _sample_lines(ST.rowptr, k, 12)
    A64, B64, G64 = _f64(w["A"]), _f64(w["B"]), _f64(w["G"])
    Ad32, Bd32, Gd = dev(w["A"]), dev(w["B"]), dev(w["G"])
    eC = oracle.fusedmm_a_rows(S, A64, B64, rows)
    mC = oracle.fusedmm_a_rows(oracle.absolute(S), np.abs(A64), np.abs(B64), rows)
    eA, eB = oracle.fusedmm_a_backward_sampled(S, ST, A64, B64, G64, rows, cols)
    mA, mB = oracle.fusedmm_a_backward_sampled(oracle.absolute(S), oracle.absolute(ST), np.abs(A64), np.abs(B64),
                                               np.abs(G64), rows, cols)
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()

    def check(tag, Ad, Bd, tol):
        Cg, _ = F.fusedmm_a_raw(P, Ad, Bd)
        gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, Gd)
        gate(f"{tag} C", host(Cg[ri]), eC, mC, tol)
        gate(f"{tag} dA", host(gA[ri]), eA, mA, tol)
        gate(f"{tag} dB", host(gB[ci]), eB, mB, tol)

    for dtype in dtypes:
        Ad, Bd, tol = (F.to_bf16(Ad32), F.to_bf16(Bd32), TOL_BF16) if dtype == torch.bfloat16 else \
            (Ad32, Bd32, TOL_F32)
        for variant in VARIANTS:
            for long_len in (None, 256, 128, 64):
                for order in (False, True):
                    tag = f"{name} {dtype} variant={variant} long_len={long_len} order={order}"
                    log(tag)
                    _configure(P, variant, long_len, order)
                    check(tag, Ad, Bd, tol)
        log(f"{name} {dtype}: autotune")
        P.autotune(Ad, Bd, Gd, form="a")
        log(f"{name} {dtype}: tuned {P.tuning}")
        check(f"{name} {dtype} autotuned", Ad, Bd, tol)


@pytest.mark.timeout(900)
def test_er1m_every_tuning_sampled():
    _check_all("er1m", workload("er1m_d32_r128"), (torch.float32, torch.bfloat16), k=512)


@pytest.mark.timeout(900)
def test_rmat20_r64_every_tuning_sampled():
    _check_all("rmat20", workload("rmat20_ef16_r64"), (torch.float32, torch.bfloat16), k=512)


def test_apply_tuning_restores_an_autotuned_configuration():
    """A tuning saved as JSON and applied to a fresh pattern of the same matrix gives the
    same configuration and the same results, bit for bit."""
    import json

    from workloads import dense_normal, rmat

    S = rmat(12, 8, seed=700)
    r = 64
    A, B, G = dev(dense_normal(S.m, r, 701)), dev(dense_normal(S.n, r, 702)), dev(dense_normal(S.m, r, 703))
    log("apply_tuning")
    P = F.Pattern.from_csr(S)
    P.autotune(A, B, G, form="a")
    saved = json.loads(json.dumps(P.tuning))
    Q = F.Pattern.from_csr(S)
    Q.apply_tuning(saved)
    assert Q.tuning == P.tuning
    out = {name: (F.fusedmm_a_raw(X, A, B)[0],) + F.fusedmm_a_backward_raw(X, A, B, G)
           for name, X in (("tuned", P), ("restored", Q))}
    assert all(torch.equal(x, y) for x, y in zip(out["tuned"], out["restored"]))
