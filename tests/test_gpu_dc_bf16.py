"""GPU parity of the adjoints with a bfloat16 upstream gradient (FMM_DC_BF16), against
the FP64 oracle: within the bf16-storage gate on the original float32 A, B, dC, and
within the float32 gate on the bf16-rounded ones (so the only extra error is the
rounding of dC).  Results repeat bit for bit, also when one output is computed alone.
The float32-dC call on the rounded dC meets the same float32 gate; the two differ in
rounding only, since a dot product of two bfloat16 vectors (here <dC_i, B_j>) takes the
bf16 dot instruction, which a float32 dC cannot."""
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from tests.gates import TOL_BF16, TOL_F32
from tests.gpu_helpers import dev, gate, host, log, ref_fusedmm_a_backward, ref_fusedmm_b_backward
from workloads import dense_normal, er_exact_degree, rmat

pytestmark = pytest.mark.gpu

CASES = [
    # (name, pattern builder, r, split)
    ("er_r64", lambda: er_exact_degree(300, 200, 9, seed=601), 64, False),
    ("rmat11_r64_split", lambda: rmat(11, 8, seed=602), 64, True),
    ("er_r128", lambda: er_exact_degree(700, 900, 33, seed=603), 128, False),
    ("rmat10_r256_split", lambda: rmat(10, 16, seed=604), 256, True),
    ("er_r1024", lambda: er_exact_degree(96, 80, 7, seed=605), 1024, False),
    ("er_r8", lambda: er_exact_degree(150, 170, 5, seed=606), 8, False),
]


@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_bf16_upstream_gradient_parity(case):
    _, build, r, split = [c for c in CASES if c[0] == case][0]
    S = build()
    P = F.Pattern.from_csr(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
    A, B = dense_normal(S.m, r, 610), dense_normal(S.n, r, 611)
    Ad, Bd = F.to_bf16(dev(A)), F.to_bf16(dev(B))
    Aq, Bq = oracle.bf16_round(A), oracle.bf16_round(B)
    for form in ("a", "b"):
        G = dense_normal(S.m if form == "a" else S.n, r, 612)
        G16 = F.to_bf16(dev(G))
        Gq = oracle.bf16_round(G)
        raw = F.fusedmm_a_backward_raw if form == "a" else F.fusedmm_b_backward_raw
        ref = ref_fusedmm_a_backward if form == "a" else ref_fusedmm_b_backward
        log(f"dC bf16 {case} form={form}")
        dA, dB = raw(P, Ad, Bd, G16)
        eA, eB, mA, mB = ref(S, A, B, G)
        gate(f"{case} {form} dA", host(dA), eA, mA, TOL_BF16)
        gate(f"{case} {form} dB", host(dB), eB, mB, TOL_BF16)
        qA, qB, qmA, qmB = ref(S, Aq, Bq, Gq)
        gate(f"{case} {form} dA rounded inputs", host(dA), qA, qmA, TOL_F32)
        gate(f"{case} {form} dB rounded inputs", host(dB), qB, qmB, TOL_F32)
        rA, rB = raw(P, Ad, Bd, G16)
        assert torch.equal(dA, rA) and torch.equal(dB, rB)
        # the float32-dC call on the rounded gradient: the same gate
        fA, fB = raw(P, Ad, Bd, G16.float())
        gate(f"{case} {form} dA float32 dC, rounded inputs", host(fA), qA, qmA, TOL_F32)
        gate(f"{case} {form} dB float32 dC, rounded inputs", host(fB), qB, qmB, TOL_F32)
        # one output at a time gives the same bits
        oA, _ = raw(P, Ad, Bd, G16, need=(True, False))
        _, oB = raw(P, Ad, Bd, G16, need=(False, True))
        assert torch.equal(oA, dA) and torch.equal(oB, dB)


def test_bf16_upstream_gradient_errors():
    S = er_exact_degree(50, 40, 4, seed=620)
    P = F.Pattern.from_csr(S)
    A, B, G = dev(dense_normal(50, 16, 1)), dev(dense_normal(40, 16, 2)), dev(dense_normal(50, 16, 3))
    log("dC bf16 errors")
    with pytest.raises(TypeError):  # float32 A and B take a float32 dC only
        F.fusedmm_a_backward_raw(P, A, B, F.to_bf16(G))
    with pytest.raises(ValueError):  # the unfused adjoint reads dC as float32
        F.fusedmm_a_backward_raw(P, F.to_bf16(A), F.to_bf16(B), F.to_bf16(G), fused=False)
    with pytest.raises(TypeError):
        F.fusedmm_b_backward_raw(P, F.to_bf16(A), F.to_bf16(B), dev(dense_normal(40, 16, 4), torch.float64))
    with pytest.raises(TypeError):  # the autotuner reads dC as float32
        P.autotune(F.to_bf16(A), F.to_bf16(B), F.to_bf16(G))
    with pytest.raises(ValueError):  # and checks its shape before any launch
        P.autotune(A, B, G[:10])


def test_bf16_upstream_gradient_autograd():
    """fusedmm_a/b(..., grad_bf16=True): the backward hands the fused adjoint the upstream
    gradient rounded to bfloat16 (the engine then casts the float32 gradients to the
    bfloat16 leaves' dtype)."""
    S = rmat(10, 8, seed=630)
    r = 64
    P = F.Pattern.from_csr(S, long_len=64, chunk=32)
    A16, B16 = F.to_bf16(dev(dense_normal(S.m, r, 631))), F.to_bf16(dev(dense_normal(S.n, r, 632)))
    for form, fn, raw, rows in (("a", F.fusedmm_a, F.fusedmm_a_backward_raw, S.m),
                                ("b", F.fusedmm_b, F.fusedmm_b_backward_raw, S.n)):
        log(f"dC bf16 autograd form={form}")
        G = dev(dense_normal(rows, r, 633))
        for grad_bf16 in (True, False):
            At, Bt = A16.clone().requires_grad_(True), B16.clone().requires_grad_(True)
            (fn(P, At, Bt, grad_bf16=grad_bf16) * G).sum().backward()
            eA, eB = raw(P, A16, B16, F.to_bf16(G) if grad_bf16 else G)
            assert At.grad.dtype == torch.bfloat16
            assert torch.equal(At.grad, eA.to(torch.bfloat16)) and torch.equal(Bt.grad, eB.to(torch.bfloat16))


def test_raw_calls_check_caller_buffers():
    """Caller-supplied outputs of the wrong shape, dtype or size are refused before any
    launch."""
    S = er_exact_degree(60, 50, 5, seed=640)
    P = F.Pattern.from_csr(S)
    A, B, G = dev(dense_normal(60, 16, 1)), dev(dense_normal(50, 16, 2)), dev(dense_normal(60, 16, 3))
    log("caller buffers")
    with pytest.raises(ValueError):
        F.fusedmm_a_raw(P, A, B, out=torch.empty(59, 16, device="cuda"))
    with pytest.raises(TypeError):
        F.fusedmm_b_raw(P, A, B, out=torch.empty(50, 16, device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        F.fusedmm_a_raw(P, A, B, fused=False, R_ws=torch.empty(S.nnz - 1, device="cuda"))
    with pytest.raises(ValueError):
        F.fusedmm_a_backward_raw(P, A, B, G, dB=torch.empty(50, 8, device="cuda"))
    with pytest.raises(ValueError):
        F.sddmm_raw(P, A, B, out=torch.empty(S.nnz // 2, device="cuda"))
    with pytest.raises(ValueError):
        F.spmm_a_raw(P, B, w=torch.ones(3, device="cuda"))
    with pytest.raises(TypeError):
        F.fusedmm_a_backward_values_raw(P, A, B, G.double())
    with pytest.raises(ValueError):
        F.fusedmm_a_backward_values_raw(P, A, B, G, dS=torch.empty(2, device="cuda"))
