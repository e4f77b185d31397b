"""GPU parity of the gradient with respect to S's stored values (learned edge values)
against the FP64 oracle: the fused one-pass kernel (alone and together with the row
pass dA / dB), the unfused two-SDDMM form, the autograd path and an FP64 gradcheck."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from tests.gates import TOL_BF16, TOL_F32, TOL_F64
from tests.gpu_helpers import dev, gate, host, log, ref_fusedmm_a_backward, ref_fusedmm_b_backward
from workloads import CsrPattern, dense_normal, er_exact_degree, rmat, tiny_case

pytestmark = pytest.mark.gpu

TOL = {torch.float32: TOL_F32, torch.bfloat16: TOL_BF16, torch.float64: TOL_F64}

CASES = [
    # (name, pattern builder, r, split)
    ("er_r8", lambda: er_exact_degree(300, 200, 9, seed=501), 8, False),
    ("rmat11_r64_split", lambda: rmat(11, 8, seed=502), 64, True),
    ("er_r128", lambda: er_exact_degree(700, 900, 33, seed=503), 128, False),
    ("rmat10_r256_split", lambda: rmat(10, 16, seed=504), 256, True),
    ("er_r3_scalar", lambda: er_exact_degree(150, 170, 5, seed=505), 3, False),
]


def _refs(S, A, B, G, form):
    fn = oracle.fusedmm_a_backward_values if form == "a" else oracle.fusedmm_b_backward_values
    return fn(S, A, B, G), fn(S, np.abs(A), np.abs(B), np.abs(G))


@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_value_gradient_parity(case):
    _, build, r, split = [c for c in CASES if c[0] == case][0]
    S32 = build()
    for dtype in (torch.float32, torch.bfloat16, torch.float64):
        if dtype == torch.bfloat16 and r % 8:
            continue
        npdt = np.float64 if dtype == torch.float64 else np.float32
        S = S32 if dtype != torch.float64 else CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx,
                                                            S32.val.astype(np.float64))
        A, B = dense_normal(S.m, r, 510, dtype=npdt), dense_normal(S.n, r, 511, dtype=npdt)
        Ga, Gb = dense_normal(S.m, r, 512, dtype=npdt), dense_normal(S.n, r, 513, dtype=npdt)
        odt = torch.float64 if dtype == torch.float64 else torch.float32
        P = F.Pattern.from_csr(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
        Ad = F.to_bf16(dev(A)) if dtype == torch.bfloat16 else dev(A, dtype)
        Bd = F.to_bf16(dev(B)) if dtype == torch.bfloat16 else dev(B, dtype)
        Aq = oracle.bf16_round(A) if dtype == torch.bfloat16 else A
        Bq = oracle.bf16_round(B) if dtype == torch.bfloat16 else B
        for form, G in (("a", Ga), ("b", Gb)):
            Gd = dev(G, odt)
            ref, mag = _refs(S, A, B, G, form)
            refq, magq = _refs(S, Aq, Bq, G, form)
            if form == "a":
                rows_ref = ref_fusedmm_a_backward(S, A, B, G)[0::2]           # dA and its companion
                rows_refq = ref_fusedmm_a_backward(S, Aq, Bq, G)[0::2]
            else:
                rows_ref = ref_fusedmm_b_backward(S, A, B, G)[1::2]           # dB and its companion
                rows_refq = ref_fusedmm_b_backward(S, Aq, Bq, G)[1::2]
            raw = F.fusedmm_a_backward_values_raw if form == "a" else F.fusedmm_b_backward_values_raw
            for fused, with_rows in ((True, False), (True, True), (False, False)):
                log(f"values {case} {dtype} form={form} fused={fused} rows={with_rows}")
                kw = {"want_dA": with_rows} if form == "a" else {"want_dB": with_rows}
                dS, X = raw(P, Ad, Bd, Gd, fused=fused, **kw)
                gate(f"{case} dS form={form} fused={fused}", host(dS), ref, mag, TOL[dtype])
                if dtype == torch.bfloat16:
                    gate(f"{case} dS bf16-rounded form={form}", host(dS), refq, magq, TOL_F32)
                if with_rows:
                    gate(f"{case} rows form={form}", host(X), rows_ref[0], rows_ref[1], TOL[dtype])
                    if dtype == torch.bfloat16:
                        gate(f"{case} rows bf16-rounded form={form}", host(X), rows_refq[0], rows_refq[1], TOL_F32)


def test_value_gradient_no_entries_and_errors():
    S = CsrPattern(4, 3, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    P = F.Pattern.from_csr(S)
    log("values: no entries")
    dS, dA = F.fusedmm_a_backward_values_raw(P, dev(dense_normal(4, 8, 1)), dev(dense_normal(3, 8, 2)),
                                             dev(dense_normal(4, 8, 3)), want_dA=True)
    assert dS.numel() == 0 and not host(dA).any()
    S2 = er_exact_degree(50, 40, 4, seed=520)
    P2 = F.Pattern.from_csr(S2)
    A, B, G = dev(dense_normal(50, 8, 4)), dev(dense_normal(40, 8, 5)), dev(dense_normal(50, 8, 6))
    with pytest.raises(F.FmmError):  # the unfused form writes dS only
        F.fusedmm_a_backward_values_raw(P2, A, B, G, want_dA=True, fused=False)
    with pytest.raises(ValueError):
        P2.with_values(torch.ones(3, device="cuda"))


@pytest.mark.parametrize("form", ["a", "b"])
@pytest.mark.parametrize("fused", [True, False])
def test_learned_values_autograd(form, fused):
    S = rmat(10, 8, seed=530)
    r = 32
    A, B = dense_normal(S.m, r, 531), dense_normal(S.n, r, 532)
    G = dense_normal(S.m if form == "a" else S.n, r, 533)
    s = np.random.default_rng(534).random(S.nnz, dtype=np.float32) + 0.5
    log(f"learned values autograd form={form} fused={fused}")
    P = F.Pattern.from_csr(S, long_len=64, chunk=32)
    At, Bt, st = dev(A).requires_grad_(True), dev(B).requires_grad_(True), dev(s).requires_grad_(True)
    fn = F.fusedmm_a if form == "a" else F.fusedmm_b
    out = fn(P, At, Bt, fused=fused, values=st)
    Sv = CsrPattern(S.m, S.n, S.rowptr, S.colidx, s)
    ref_out = (oracle.fusedmm_a if form == "a" else oracle.fusedmm_b)(Sv, A, B)
    mag_out = (oracle.fusedmm_a if form == "a" else oracle.fusedmm_b)(oracle.absolute(Sv), np.abs(A), np.abs(B))
    gate("forward with values", host(out), ref_out, mag_out, TOL_F32)
    (out * dev(G)).sum().backward()
    ref_s, mag_s = _refs(S, A, B, G, form)
    gate("values grad", host(st.grad), ref_s, mag_s, TOL_F32)
    dA, dB, mA, mB = (ref_fusedmm_a_backward if form == "a" else ref_fusedmm_b_backward)(Sv, A, B, G)
    gate("A grad", host(At.grad), dA, mA, TOL_F32)
    gate("B grad", host(Bt.grad), dB, mB, TOL_F32)
    # only the values require a gradient
    st.grad = None
    out = fn(P, dev(A), dev(B), fused=fused, values=st)
    (out * dev(G)).sum().backward()
    gate("values grad alone", host(st.grad), ref_s, mag_s, TOL_F32)


def test_learned_values_gradcheck_fp64():
    small = tiny_case(12, 10, 3, 0.4, seed=540)
    S = small["S"]
    log("learned values gradcheck fp64")
    P = F.Pattern.from_csr(S, val_dtype=torch.float64)
    At = dev(small["A"]).requires_grad_(True)
    Bt = dev(small["B"]).requires_grad_(True)
    st = dev(np.asarray(S.val, np.float64)).requires_grad_(True)
    for fused in (True, False):
        assert torch.autograd.gradcheck(lambda a, b, v: F.fusedmm_a(P, a, b, fused=fused, values=v), (At, Bt, st),
                                        eps=1e-6, atol=1e-8)
        assert torch.autograd.gradcheck(lambda a, b, v: F.fusedmm_b(P, a, b, fused=fused, values=v), (At, Bt, st),
                                        eps=1e-6, atol=1e-8)


def test_with_values_keeps_the_original_pattern_intact():
    """Tuning a values view must not touch the pattern it came from (their descriptors
    point at their own schedule and order tensors)."""
    S = rmat(10, 8, seed=550)
    P = F.Pattern.from_csr(S, long_len=64, chunk=32, line_order=True)
    A, B = dev(dense_normal(S.m, 16, 551)), dev(dense_normal(S.n, 16, 552))
    log("with_values independence")
    before = F.fusedmm_a_raw(P, A, B)[0].clone()
    Q = P.with_values(P.val.clone())
    Q.set_line_order(0, False)
    Q.set_line_order(1, False)
    Q.set_split(1, 16)
    torch.cuda.synchronize()
    assert P.orders["csr"] is not None and P.orders["csc"] is not None and P.splits["csc"] == 64
    assert torch.equal(F.fusedmm_a_raw(P, A, B)[0], before)
    # same values and CSR schedule, order off: the order never changes a line's arithmetic
    assert torch.equal(F.fusedmm_a_raw(Q, A, B)[0], before)


@pytest.mark.parametrize("r,dtype", [(1024, torch.float32), (512, torch.float64), (1024, torch.bfloat16)])
def test_value_gradient_widest_rows(r, dtype):
    S32 = er_exact_degree(96, 80, 7, seed=560)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    S = S32 if dtype != torch.float64 else CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx, S32.val.astype(np.float64))
    A, B, G = dense_normal(S.m, r, 561, dtype=npdt), dense_normal(S.n, r, 562, dtype=npdt), dense_normal(S.m, r, 563,
                                                                                                          dtype=npdt)
    log(f"values widest r={r} {dtype}")
    P = F.Pattern.from_csr(S)
    odt = torch.float64 if dtype == torch.float64 else torch.float32
    Ad = F.to_bf16(dev(A)) if dtype == torch.bfloat16 else dev(A, dtype)
    Bd = F.to_bf16(dev(B)) if dtype == torch.bfloat16 else dev(B, dtype)
    dS, dA = F.fusedmm_a_backward_values_raw(P, Ad, Bd, dev(G, odt), want_dA=True)
    Aq = oracle.bf16_round(A) if dtype == torch.bfloat16 else A
    Bq = oracle.bf16_round(B) if dtype == torch.bfloat16 else B
    ref, mag = _refs(S, Aq, Bq, G, "a")
    gate(f"widest dS r={r}", host(dS), ref, mag, TOL_F64 if dtype == torch.float64 else TOL_F32)
    eA, _, mA, _ = ref_fusedmm_a_backward(S, Aq, Bq, G)
    gate(f"widest dA r={r}", host(dA), eA, mA, TOL_F64 if dtype == torch.float64 else TOL_F32)
