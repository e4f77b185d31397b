"""GPU parity at the paper-shaped workload sizes, on sampled outputs.

Rows of FusedMMA (and columns of FusedMMB) are independent, so checking a seeded
sample of them against the oracle is exact for those outputs.  Samples include the
longest lines (the split-chunk path on R-MAT), empty lines and random ones.  Calls
run in the Pattern's default configuration (default shapes and split schedule);
test_gpu_tuning_full.py repeats the check under every configuration the benchmark's
autotuner can choose.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from tests.gates import TOL_BF16, TOL_F32
from tests.gpu_helpers import dev, gate, host, log
from workloads import workload

# Configurations the benchmark's autotuner chose for R-MAT scale 22, r = 256 on MI355X
# (batch depth class, split threshold, line order and gather hints per orientation), for
# float32 and for bfloat16 storage.  The adjoint test runs under these and under the autotuner's own pick.
RMAT22_BENCH_TUNING = {
    "f32": {"csr": {"variant": 2, "long_len": 256, "line_order": False, "gather_hints": 32768},
            "csc": {"variant": 3, "long_len": 256, "line_order": False, "gather_hints": 32768}},
    "bf16": {"csr": {"variant": 3, "long_len": 256, "line_order": True, "gather_hints": None},
             "csc": {"variant": 2, "long_len": 256, "line_order": False, "gather_hints": 65536}},
}

pytestmark = pytest.mark.gpu


def _sample_lines(ptr, k, seed):
    lens = np.diff(ptr.astype(np.int64))
    rng = np.random.default_rng(seed)
    rand = rng.choice(lens.shape[0], size=min(k, lens.shape[0]), replace=False)
    longest = np.argsort(lens)[-16:]
    empty = np.flatnonzero(lens == 0)[:8]
    return np.unique(np.concatenate([rand, longest, empty])).astype(np.int64)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _refs_rows(S, A, B, rows):
    ref = oracle.fusedmm_a_rows(S, A, B, rows)
    mag = oracle.fusedmm_a_rows(oracle.absolute(S), np.abs(A), np.abs(B), rows)
    return ref, mag


def _refs_cols(ST, A, B, cols):
    ref = oracle.fusedmm_b_cols(ST, A, B, cols)
    mag = oracle.fusedmm_b_cols(oracle.absolute(ST), np.abs(A), np.abs(B), cols)
    return ref, mag


def _check_forward(name, w, dtypes, k=2048):
    S = w["S"]
    log(f"{name}: m={S.m} nnz={S.nnz} r={w['r']} building pattern")
    P = F.Pattern.from_csr(S)
    ST = oracle.transpose(S)
    rows = _sample_lines(S.rowptr, k, 1)
    cols = _sample_lines(ST.rowptr, k, 2)
    A64, B64 = _f64(w["A"]), _f64(w["B"])
    Ad32, Bd32 = dev(w["A"]), dev(w["B"])
    for dtype in dtypes:
        if dtype == torch.bfloat16:
            Ad, Bd, tol = F.to_bf16(Ad32), F.to_bf16(Bd32), TOL_BF16
        else:
            Ad, Bd, tol = Ad32, Bd32, TOL_F32
        ref, mag = _refs_rows(S, A64, B64, rows)
        refb, magb = _refs_cols(ST, A64, B64, cols)
        for fused in (True, False):
            log(f"{name}: FusedMMA dtype={dtype} fused={fused}")
            Cg, _ = F.fusedmm_a_raw(P, Ad, Bd, fused=fused)
            gate(f"{name} FusedMMA {dtype} fused={fused}", host(Cg[torch.from_numpy(rows).cuda()]), ref, mag, tol)
            del Cg
            log(f"{name}: FusedMMB dtype={dtype} fused={fused}")
            Cb, _ = F.fusedmm_b_raw(P, Ad, Bd, fused=fused)
            gate(f"{name} FusedMMB {dtype} fused={fused}", host(Cb[torch.from_numpy(cols).cuda()]), refb, magb, tol)
            del Cb
            torch.cuda.empty_cache()
    return P, ST, rows, cols


@pytest.mark.timeout(600)
def test_er4096_unfused_sequence_full():
    # SDDMM then SpMM (unfused FusedMMA), checked on every output
    w = workload("er4096_d32_r32")
    S, A, B = w["S"], w["A"], w["B"]
    log("er4096 full")
    P = F.Pattern.from_csr(S)
    R = host(F.sddmm_raw(P, dev(A), dev(B)))
    Rref = oracle.sddmm(S, A, B)
    Rmag = oracle.sddmm(oracle.absolute(S), np.abs(A), np.abs(B))
    gate("er4096 R", R, Rref, Rmag, TOL_F32)
    for fused in (False, True):
        Cg, _ = F.fusedmm_a_raw(P, dev(A), dev(B), fused=fused)
        ref = oracle.fusedmm_a(S, A, B)
        mag = oracle.fusedmm_a(oracle.absolute(S), np.abs(A), np.abs(B))
        gate(f"er4096 C fused={fused}", host(Cg), ref, mag, TOL_F32)


@pytest.mark.timeout(600)
def test_er1m_forward_and_adjoint_sampled():
    w = workload("er1m_d32_r128")
    P, ST, rows, cols = _check_forward("er1m", w, (torch.float32, torch.bfloat16))
    S = w["S"]
    A64, B64, G64 = _f64(w["A"]), _f64(w["B"]), _f64(w["G"])
    Ad, Bd, Gd = dev(w["A"]), dev(w["B"]), dev(w["G"])
    eA, eB = oracle.fusedmm_a_backward_sampled(S, ST, A64, B64, G64, rows, cols)
    mA, mB = oracle.fusedmm_a_backward_sampled(oracle.absolute(S), oracle.absolute(ST), np.abs(A64), np.abs(B64),
                                               np.abs(G64), rows, cols)
    for fused in (True, False):
        log(f"er1m adjoint fused={fused}")
        R_ws = F.fusedmm_a_raw(P, Ad, Bd, fused=False)[1] if not fused else None
        gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, Gd, fused=fused, R_ws=R_ws)
        gate(f"er1m dA fused={fused}", host(gA[torch.from_numpy(rows).cuda()]), eA, mA, TOL_F32)
        gate(f"er1m dB fused={fused}", host(gB[torch.from_numpy(cols).cuda()]), eB, mB, TOL_F32)
        del gA, gB, R_ws


@pytest.mark.timeout(900)
def test_rmat22_r256_forward_sampled():
    w = workload("rmat22_ef16_r256")
    S = w["S"]
    assert S.meta["max_row"] > 10000 and S.meta["empty_rows"] > S.m // 3
    P, ST, rows, cols = _check_forward("rmat22", w, (torch.bfloat16, torch.float32), k=1024)
    assert P.schedules["csr"] is not None and P.schedules["csc"] is not None


@pytest.mark.timeout(600)
def test_rmat20_r64_adjoint_sampled():
    w = workload("rmat20_ef16_r64")
    S = w["S"]
    log(f"rmat20: nnz={S.nnz}")
    P = F.Pattern.from_csr(S)
    ST = oracle.transpose(S)
    rows = _sample_lines(S.rowptr, 2048, 3)
    cols = _sample_lines(ST.rowptr, 2048, 4)
    A64, B64, G64 = _f64(w["A"]), _f64(w["B"]), _f64(w["G"])
    Ad, Bd, Gd = dev(w["A"]), dev(w["B"]), dev(w["G"])
    eA, eB = oracle.fusedmm_a_backward_sampled(S, ST, A64, B64, G64, rows, cols)
    mA, mB = oracle.fusedmm_a_backward_sampled(oracle.absolute(S), oracle.absolute(ST), np.abs(A64), np.abs(B64),
                                               np.abs(G64), rows, cols)
    At = Ad.clone().requires_grad_(True)
    Bt = Bd.clone().requires_grad_(True)
    log("rmat20 autograd fwd+bwd")
    (F.fusedmm_a(P, At, Bt) * Gd).sum().backward()
    gate("rmat20 dA", host(At.grad[torch.from_numpy(rows).cuda()]), eA, mA, TOL_F32)
    gate("rmat20 dB", host(Bt.grad[torch.from_numpy(cols).cuda()]), eB, mB, TOL_F32)
    # FusedMMB adjoint at the same size (upstream gradient n x r)
    Gb64 = _f64(w["G"])  # square graph: reuse G as an n x r gradient
    eA, eB = oracle.fusedmm_b_backward_sampled(S, ST, A64, B64, Gb64, rows, cols)
    mA, mB = oracle.fusedmm_b_backward_sampled(oracle.absolute(S), oracle.absolute(ST), np.abs(A64), np.abs(B64),
                                               np.abs(Gb64), rows, cols)
    log("rmat20 FusedMMB adjoint")
    gA, gB = F.fusedmm_b_backward_raw(P, Ad, Bd, Gd)
    gate("rmat20 B dA", host(gA[torch.from_numpy(rows).cuda()]), eA, mA, TOL_F32)
    gate("rmat20 B dB", host(gB[torch.from_numpy(cols).cuda()]), eB, mB, TOL_F32)


@pytest.mark.timeout(1200)
def test_rmat22_r256_adjoint_sampled():
    """The adjoint at the bench's own workload: dA on sampled rows and dB on sampled columns
    (random ones, the 16 longest, which the split schedule cuts into chunks, and empty
    ones), with float32 storage, bfloat16 storage, and bfloat16 storage with a bfloat16
    upstream gradient, under the bench's tuning and the autotuner's pick."""
    w = workload("rmat22_ef16_r256")
    S = w["S"]
    log(f"rmat22 adjoint: nnz={S.nnz} building pattern")
    P = F.Pattern.from_csr(S)
    ST = oracle.transpose(S)
    rows = _sample_lines(S.rowptr, 1024, 21)
    cols = _sample_lines(ST.rowptr, 1024, 22)
    lens_c = np.diff(ST.rowptr.astype(np.int64))
    assert lens_c[cols].max() == lens_c.max() > 50000 and (lens_c[cols] == 0).any()
    A, B, G = w["A"], w["B"], w["G"]
    rnd, ab = oracle.bf16_round, np.abs
    rab = lambda x: np.abs(oracle.bf16_round(x))  # noqa: E731
    SA, STA = oracle.absolute(S), oracle.absolute(ST)

    def refs(prep, prep_mag):
        return (oracle.fusedmm_a_outputs_sampled(S, ST, A, B, G, rows, cols, prep=prep),
                oracle.fusedmm_a_outputs_sampled(SA, STA, A, B, G, rows, cols, prep=prep_mag))

    log("rmat22 adjoint: oracle references")
    ref32 = refs(None, (ab, ab, ab))
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    Ad32, Bd32, Gd = dev(A), dev(B), dev(G)
    Ad16, Bd16 = F.to_bf16(Ad32), F.to_bf16(Bd32)
    Gd16 = F.to_bf16(Gd)
    cases = (("f32", Ad32, Bd32, Gd, TOL_F32, None),
             ("bf16", Ad16, Bd16, Gd, TOL_BF16, ((rnd, rnd, None), (rab, rab, ab))),
             ("bf16_dc_bf16", Ad16, Bd16, Gd16, TOL_BF16, ((rnd, rnd, rnd), (rab, rab, rab))))
    for tag, Ad, Bd, Gi, tol, rounded in cases:
        refq = refs(*rounded) if rounded else None
        for how in ("bench tuning", "autotuned"):
            if how == "bench tuning":
                P.apply_tuning(RMAT22_BENCH_TUNING["f32" if tag == "f32" else "bf16"])
            else:
                log(f"rmat22 adjoint {tag}: autotune")
                P.autotune(Ad, Bd, Gd, form="a")
            log(f"rmat22 adjoint {tag} {how}: {P.tuning}")
            Cg, _ = F.fusedmm_a_raw(P, Ad, Bd)
            gA, gB = F.fusedmm_a_backward_raw(P, Ad, Bd, Gi)
            got = (host(Cg[ri]), host(gA[ri]), host(gB[ci]))
            del Cg, gA, gB
            for name, x, e, mg in zip(("C", "dA", "dB"), got, ref32[0], ref32[1]):
                gate(f"rmat22 {tag} {how} {name}", x, e, mg, tol)
            if refq is not None:
                for name, x, e, mg in zip(("C", "dA", "dB"), got, refq[0], refq[1]):
                    gate(f"rmat22 {tag} {how} {name} (rounded inputs)", x, e, mg, TOL_F32)
            torch.cuda.empty_cache()
