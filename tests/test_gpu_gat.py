"""GPU parity of the graph-attention head (Section VI-E) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from tests.gat_gate import gat_backward_magnitudes, kink_free
from tests.gates import TOL_BF16, TOL_F32, TOL_F64
from tests.gpu_helpers import dev, gate, host, log
from workloads import CsrPattern, dense_normal, er_exact_degree, rmat, tiny_case, workload

pytestmark = pytest.mark.gpu

TOL = {torch.float32: TOL_F32, torch.bfloat16: TOL_BF16, torch.float64: TOL_F64}


def _ref(S, H, a1, a2, slope, softmax, rows=None):
    """Oracle output and its magnitude companion.

    With the softmax the weights are positive and sum to 1, and the score rounding
    error moves each weight by a relative amount: sum_j w_ij |H_j| bounds the error.
    Without it the weight is the score itself, whose rounding error is relative to
    |S_ij| (|a1|.|H_i| + |a2|.|H_j|), not to the (possibly cancelled) score: the
    companion is sum_j |S_ij| (|a1|.|H_i| + |a2|.|H_j|) |H_j|."""
    s, t = oracle.gat_scores(H, a1, a2)
    w = oracle.gat_edges(S, s, t, slope, softmax)
    ref = oracle.spmm_a(S, w, H, rows=rows)
    if softmax:
        return ref, oracle.spmm_a(S, np.abs(w), np.abs(H), rows=rows)
    ms, mt = oracle.gat_scores(np.abs(H), np.abs(a1), np.abs(a2))
    rowsof = np.repeat(np.arange(S.m), np.diff(S.rowptr))
    wm = np.abs(np.asarray(S.val, np.float64)) * (ms[rowsof] + mt[S.colidx])
    return ref, oracle.spmm_a(S, wm, np.abs(H), rows=rows)


CASES = [
    ("er_r64", lambda: er_exact_degree(700, 700, 12, seed=401), 64, False),
    ("er_r3", lambda: er_exact_degree(300, 300, 9, seed=402), 3, False),
    ("rmat_r128_split", lambda: rmat(11, 8, seed=403), 128, True),
    ("rmat_r8", lambda: rmat(10, 16, seed=404), 8, True),
    ("er_r1024", lambda: er_exact_degree(96, 96, 7, seed=405), 1024, False),   # widest fp32/bf16 rows
    ("er_r512", lambda: er_exact_degree(80, 80, 6, seed=406), 512, False),     # widest fp64 rows
]


@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_gat_forward_parity(case):
    _, build, r, split = [c for c in CASES if c[0] == case][0]
    S32 = build()
    for dtype in (torch.float32, torch.float64, torch.bfloat16):
        if dtype == torch.bfloat16 and r % 8:
            continue
        if dtype == torch.float64 and r > 512:  # fp64 rows stop at 512
            continue
        npdt = np.float64 if dtype == torch.float64 else np.float32
        S = S32 if dtype != torch.float64 else CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx,
                                                            S32.val.astype(np.float64))
        H = dense_normal(S.n, r, 410, dtype=npdt)
        a1 = dense_normal(1, r, 411, sigma=r ** -0.5, dtype=npdt)[0]
        a2 = dense_normal(1, r, 412, sigma=r ** -0.5, dtype=npdt)[0]
        odt = torch.float64 if dtype == torch.float64 else torch.float32
        P = F.Pattern.from_csr(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
        if split:
            assert P.schedules["csr"] is not None
        Hd = F.to_bf16(dev(H)) if dtype == torch.bfloat16 else dev(H, dtype)
        Hq = oracle.bf16_round(H) if dtype == torch.bfloat16 else H
        a1d, a2d = dev(a1, odt), dev(a2, odt)
        s, t = F.gat_scores(Hd, a1d, a2d)
        es, et = oracle.gat_scores(Hq, a1, a2)
        ms, mt = oracle.gat_scores(np.abs(Hq), np.abs(a1), np.abs(a2))
        gate(f"{case} scores s {dtype}", host(s), es, ms, TOL_F64 if dtype == torch.float64 else TOL_F32)
        gate(f"{case} scores t {dtype}", host(t), et, mt, TOL_F64 if dtype == torch.float64 else TOL_F32)
        for softmax in (True, False):
            log(f"gat {case} dtype={dtype} softmax={softmax}")
            out = host(F.gat_forward(P, Hd, a1d, a2d, negative_slope=0.2, softmax=softmax))
            if dtype == torch.bfloat16:
                # bf16 storage moves the scores themselves by up to u * sum |a||H|, which the
                # softmax turns into relative weight changes of that size: gate the GPU against
                # the oracle on the same rounded features (accumulation error only), and keep
                # only a sanity bound against the unrounded ones.
                refq, magq = _ref(S, Hq, a1, a2, 0.2, softmax)
                gate(f"{case} gat bf16-rounded softmax={softmax}", out, refq, magq, TOL_F32)
                ref, mag = _ref(S, H, a1, a2, 0.2, softmax)
                gate(f"{case} gat bf16 vs unrounded softmax={softmax}", out, ref, mag, 0.1)
            else:
                ref, mag = _ref(S, H, a1, a2, 0.2, softmax)
                gate(f"{case} gat {dtype} softmax={softmax}", out, ref, mag, TOL[dtype])


def test_gat_closed_forms_on_gpu():
    S = er_exact_degree(300, 300, 7, seed=420)
    H = dense_normal(300, 16, 421)
    log("gat closed forms")
    P = F.Pattern.from_csr(S)
    z = torch.zeros(16, device="cuda")
    out = host(F.gat_forward(P, dev(H), z, z, softmax=True))
    ref = np.stack([H[S.colidx[S.rowptr[i]:S.rowptr[i + 1]]].astype(np.float64).mean(axis=0) for i in range(300)])
    assert np.max(np.abs(out - ref)) <= 1e-5 * (1 + np.abs(ref).max())
    # a row with no stored entries gives exactly 0
    rp = np.array([0, 0, 2, 3], np.int32)
    ci = np.array([0, 2, 1], np.int32)
    S0 = CsrPattern(3, 3, rp, ci, np.ones(3, np.float32))
    P0 = F.Pattern.from_csr(S0)
    H0 = dense_normal(3, 8, 422)
    o0 = host(F.gat_forward(P0, dev(H0), torch.ones(8, device="cuda"), torch.ones(8, device="cuda")))
    assert np.all(o0[0] == 0)


@pytest.mark.timeout(600)
def test_gat_rmat20_r128_sampled():
    w = workload("rmat20_ef16_r64")
    S = w["S"]
    r = 128
    H = dense_normal(S.n, r, 430)
    a1 = dense_normal(1, r, 431, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 432, sigma=r ** -0.5)[0]
    log(f"gat rmat20 r=128 nnz={S.nnz}")
    P = F.Pattern.from_csr(S)
    lens = np.diff(S.rowptr.astype(np.int64))
    rows = np.unique(np.concatenate([np.random.default_rng(433).choice(S.m, 2048, replace=False),
                                     np.argsort(lens)[-16:], np.flatnonzero(lens == 0)[:8]]))
    for dtype in (torch.float32, torch.bfloat16):
        Hd = F.to_bf16(dev(H)) if dtype == torch.bfloat16 else dev(H)
        out = F.gat_forward(P, Hd, dev(a1), dev(a2), softmax=True)
        Hq = oracle.bf16_round(H) if dtype == torch.bfloat16 else H
        ref, mag = _ref(S, Hq, a1, a2, 0.2, True, rows=rows)
        gate(f"rmat20 gat {dtype}", host(out[torch.from_numpy(rows).cuda()]), ref, mag, TOL_F32)


@pytest.mark.parametrize("softmax", [True, False])
def test_gat_edge_values_and_unfused_head(softmax):
    S = rmat(11, 8, seed=440)
    r = 64
    H = dense_normal(S.n, r, 441)
    a1 = dense_normal(1, r, 442, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 443, sigma=r ** -0.5)[0]
    log(f"gat edge values softmax={softmax}")
    P = F.Pattern.from_csr(S, long_len=64, chunk=32)
    w = host(F.gat_edge_values(P, dev(H), dev(a1), dev(a2), softmax=softmax))
    s, t = oracle.gat_scores(H, a1, a2)
    ew = oracle.gat_edges(S, s, t, 0.2, softmax)
    if softmax:
        mag = np.abs(ew)
    else:
        ms, mt = oracle.gat_scores(np.abs(H), np.abs(a1), np.abs(a2))
        rowsof = np.repeat(np.arange(S.m), np.diff(S.rowptr))
        mag = np.abs(S.val.astype(np.float64)) * (ms[rowsof] + mt[S.colidx])
    gate(f"edge values softmax={softmax}", w, ew, mag, TOL_F32)
    out = host(F.gat_forward_unfused(P, dev(H), dev(a1), dev(a2), softmax=softmax))
    ref, mg = _ref(S, H, a1, a2, 0.2, softmax)
    gate(f"unfused head softmax={softmax}", out, ref, mg, TOL_F32)


# ------------------------------------------------------------ adjoint of the attention head

def _gate_adjoint(name, got, S, H, a1, a2, dO, softmax, tol):
    """Every output of the attention adjoint against the oracle, element by element,
    relative to its magnitude companion (tests/gat_gate.py: the oracle's steps on
    absolute values plus the weights' sensitivity to score rounding)."""
    ref = oracle.gat_backward(S, H, a1, a2, dO, slope=0.2, softmax=softmax)
    mag = gat_backward_magnitudes(S, H, a1, a2, dO, slope=0.2, softmax=softmax)
    for out, g, want, m in zip(("dH", "da1", "da2", "dS"), got, ref, mag):
        gate(f"{name} {out}", host(g), want, m, tol)


BWD_CASES = [
    ("er_r64", lambda: er_exact_degree(700, 700, 12, seed=601), 64, False),
    ("rmat_r128_split", lambda: rmat(11, 8, seed=602), 128, True),
    ("rmat_r8_split", lambda: rmat(10, 16, seed=603), 8, True),
    ("er_r3", lambda: er_exact_degree(300, 300, 9, seed=604), 3, False),
    ("er_r1024", lambda: er_exact_degree(96, 96, 7, seed=605), 1024, False),
    ("er_r512", lambda: er_exact_degree(80, 80, 6, seed=606), 512, False),
]


@pytest.mark.parametrize("case", [c[0] for c in BWD_CASES])
def test_gat_backward_parity(case):
    _, build, r, split = [c for c in BWD_CASES if c[0] == case][0]
    S32 = build()
    for dtype in (torch.float32, torch.float64, torch.bfloat16):
        if dtype == torch.bfloat16 and r % 8:
            continue
        if dtype == torch.float64 and r > 512:  # fp64 rows stop at 512
            continue
        npdt = np.float64 if dtype == torch.float64 else np.float32
        S = S32 if dtype != torch.float64 else CsrPattern(S32.m, S32.n, S32.rowptr, S32.colidx,
                                                            S32.val.astype(np.float64))
        H = dense_normal(S.n, r, 610, dtype=npdt)
        a1 = dense_normal(1, r, 611, sigma=r ** -0.5, dtype=npdt)[0]
        a2 = dense_normal(1, r, 612, sigma=r ** -0.5, dtype=npdt)[0]
        dO = dense_normal(S.m, r, 613, dtype=npdt)
        odt = torch.float64 if dtype == torch.float64 else torch.float32
        Hd = F.to_bf16(dev(H)) if dtype == torch.bfloat16 else dev(H, dtype)
        Hq = oracle.bf16_round(H) if dtype == torch.bfloat16 else H
        S, _ = kink_free(S, Hq, a1, a2)
        P = F.Pattern.from_csr(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
        tol = TOL_F64 if dtype == torch.float64 else TOL_F32
        for softmax in (True, False):
            log(f"gat backward {case} {dtype} softmax={softmax}")
            a1d, a2d = dev(a1, odt), dev(a2, odt)
            out = F.gat_forward(P, Hd, a1d, a2d, softmax=softmax)
            got = F.gat_backward(P, Hd, a1d, a2d, out, dev(dO, odt), softmax=softmax, want_dS=True)
            # the oracle on the same (rounded, for bf16) features isolates accumulation error
            _gate_adjoint(f"{case} {dtype} softmax={softmax}", got, S, Hq, a1, a2, dO, softmax, tol)


@pytest.mark.parametrize("case", [c[0] for c in BWD_CASES if c[2] % 8 == 0])
def test_gat_backward_bf16_upstream_gradient(case):
    """bf16 features and a bf16 dO (FMM_DC_BF16): against the oracle on the rounded H and
    dO at the float32 gate, so the only extra error is dO's rounding; repeatable bit for
    bit."""
    _, build, r, split = [c for c in BWD_CASES if c[0] == case][0]
    S = build()
    H = dense_normal(S.n, r, 610)
    a1 = dense_normal(1, r, 611, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 612, sigma=r ** -0.5)[0]
    dO = dense_normal(S.m, r, 613)
    Hd, dO16 = F.to_bf16(dev(H)), F.to_bf16(dev(dO))
    Hq, dOq = oracle.bf16_round(H), oracle.bf16_round(dO)
    S, _ = kink_free(S, Hq, a1, a2)
    P = F.Pattern.from_csr(S, long_len=64 if split else 1 << 30, chunk=32 if split else 1 << 30, split=split)
    a1d, a2d = dev(a1), dev(a2)
    for softmax in (True, False):
        log(f"gat backward bf16 dO {case} softmax={softmax}")
        out = F.gat_forward(P, Hd, a1d, a2d, softmax=softmax)
        got = F.gat_backward(P, Hd, a1d, a2d, out, dO16, softmax=softmax, want_dS=True)
        _gate_adjoint(f"{case} bf16 dO softmax={softmax}", got, S, Hq, a1, a2, dOq, softmax, TOL_F32)
        again = F.gat_backward(P, Hd, a1d, a2d, out, dO16, softmax=softmax, want_dS=True)
        assert all(torch.equal(x, y) for x, y in zip(got, again))
    # the autograd option hands the adjoint the rounded upstream gradient
    Ht = Hd.clone().requires_grad_(True)
    (F.gat(P, Ht, a1d, a2d, grad_bf16=True) * dev(dO)).sum().backward()
    out = F.gat_forward(P, Hd, a1d, a2d)
    eH = F.gat_backward(P, Hd, a1d, a2d, out, dO16)[0]
    assert torch.equal(Ht.grad, eH.to(torch.bfloat16))
    with pytest.raises(TypeError):  # float32 features take a float32 dO only
        F.gat_backward(P, dev(H), a1d, a2d, F.gat_forward(P, dev(H), a1d, a2d), dO16)
    with pytest.raises(TypeError):
        F.gat_backward(P, Hd, a1d, a2d, out.double(), dO16)
    # attention vectors of the wrong length or device, and a misshapen lse, are refused
    # before any launch
    with pytest.raises(ValueError):
        F.gat_forward(P, Hd, a1d[:-1], a2d)
    with pytest.raises(ValueError):
        F.gat_forward(P, Hd, a1d, a2d.cpu())
    with pytest.raises(ValueError):
        F.gat_forward(P, Hd, a1d, a2d, lse=torch.empty(S.m - 1, device="cuda"))


@pytest.mark.parametrize("softmax", [True, False])
def test_gat_autograd_and_gradcheck(softmax):
    S = rmat(9, 8, seed=620)
    r = 16
    H = dense_normal(S.n, r, 621)
    a1 = dense_normal(1, r, 622, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 623, sigma=r ** -0.5)[0]
    G = dense_normal(S.m, r, 624)
    S, _ = kink_free(S, H, a1, a2)
    log(f"gat autograd softmax={softmax}")
    P = F.Pattern.from_csr(S, long_len=32, chunk=16)
    Ht, a1t, a2t = dev(H).requires_grad_(True), dev(a1).requires_grad_(True), dev(a2).requires_grad_(True)
    vt = dev(S.val).requires_grad_(True)
    out = F.gat(P, Ht, a1t, a2t, values=vt, softmax=softmax)
    (out * dev(G)).sum().backward()
    _gate_adjoint("autograd", (Ht.grad, a1t.grad, a2t.grad, vt.grad), S, H, a1, a2, G, softmax, TOL_F32)
    small = tiny_case(14, 14, 3, 0.35, seed=625)
    Ss = small["S"]
    Ps = F.Pattern.from_csr(Ss, val_dtype=torch.float64)
    args = (dev(small["A"]).requires_grad_(True), dev(np.array([0.3, -0.2, 0.5])).requires_grad_(True),
            dev(np.array([-0.4, 0.1, 0.2])).requires_grad_(True),
            dev(np.asarray(Ss.val, np.float64)).requires_grad_(True))
    assert torch.autograd.gradcheck(lambda h, x, y, v: F.gat(Ps, h, x, y, values=v, softmax=softmax), args,
                                    eps=1e-6, atol=1e-8)


@pytest.mark.timeout(600)
def test_gat_backward_rmat20_r128_full():
    """The adjoint at the benchmark's size (R-MAT scale 20, 16.1M entries, r = 128, the
    pattern's default split and line order), every output against the oracle."""
    w = workload("rmat20_ef16_r64")
    S = w["S"]
    r = 128
    H = dense_normal(S.n, r, 630)
    a1 = dense_normal(1, r, 631, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 632, sigma=r ** -0.5)[0]
    dO = dense_normal(S.m, r, 633)
    S, k = kink_free(S, H, a1, a2)
    log(f"gat backward rmat20 r=128 nnz={S.nnz} ({k} entries at the kink given value 0)")
    P = F.Pattern.from_csr(S)
    Hd, a1d, a2d = dev(H), dev(a1), dev(a2)
    lse = torch.empty(S.m, device="cuda")
    out = F.gat_forward(P, Hd, a1d, a2d, softmax=True, lse=lse)
    got = F.gat_backward(P, Hd, a1d, a2d, out, dev(dO), softmax=True, want_dS=True, lse=lse)
    _gate_adjoint("rmat20", got, S, H, a1, a2, dO, True, TOL_F32)


def test_gat_autotune_keeps_results():
    S = rmat(11, 8, seed=640)
    r = 32
    H = dense_normal(S.n, r, 641)
    a1 = dense_normal(1, r, 642, sigma=r ** -0.5)[0]
    a2 = dense_normal(1, r, 643, sigma=r ** -0.5)[0]
    dO = dense_normal(S.m, r, 644)
    S, _ = kink_free(S, H, a1, a2)
    log("gat autotune")
    P = F.Pattern.from_csr(S)
    tuning = F.gat_autotune(P, dev(H), dev(a1), dev(a2), dO=dev(dO))
    assert set(tuning) == {"csr", "csc"}
    lse = torch.empty(S.m, device="cuda")
    out = F.gat_forward(P, dev(H), dev(a1), dev(a2), lse=lse)
    ref, mag = _ref(S, H, a1, a2, 0.2, True)
    gate("tuned forward", host(out), ref, mag, TOL_F32)
    got = F.gat_backward(P, dev(H), dev(a1), dev(a2), out, dev(dO), want_dS=True, lse=lse)
    _gate_adjoint("tuned", got, S, H, a1, a2, dO, True, TOL_F32)


def test_gat_backward_edge_cases():
    """No stored entries (every weight absent: dH = 0 and da = 0), a row without entries
    among others, and a wide head (r = 512, the L = 64 x NV = 2 shape)."""
    log("gat backward edge cases")
    S0 = CsrPattern(5, 5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    P0 = F.Pattern.from_csr(S0)
    H0 = dev(dense_normal(5, 8, 650))
    a = dev(dense_normal(1, 8, 651)[0])
    lse = torch.empty(5, device="cuda")
    out = F.gat_forward(P0, H0, a, a, lse=lse)
    dH, da1, da2, dS = F.gat_backward(P0, H0, a, a, out, dev(dense_normal(5, 8, 652)), want_dS=True, lse=lse)
    assert not host(dH).any() and not host(da1).any() and not host(da2).any() and dS.numel() == 0
    rp = np.array([0, 2, 2, 5, 6], np.int32)
    ci = np.array([1, 3, 0, 2, 3, 1], np.int32)
    S1 = CsrPattern(4, 4, rp, ci, np.linspace(0.5, 1.5, 6).astype(np.float32))
    for r in (8, 512):
        H = dense_normal(S1.n, r, 653)
        a1 = dense_normal(1, r, 654, sigma=r ** -0.5)[0]
        a2 = dense_normal(1, r, 655, sigma=r ** -0.5)[0]
        dO = dense_normal(S1.m, r, 656)
        Sk, _ = kink_free(S1, H, a1, a2)
        P1 = F.Pattern.from_csr(Sk)
        lse = torch.empty(4, device="cuda")
        out = F.gat_forward(P1, dev(H), dev(a1), dev(a2), lse=lse)
        got = F.gat_backward(P1, dev(H), dev(a1), dev(a2), out, dev(dO), want_dS=True, lse=lse)
        _gate_adjoint(f"edge r={r}", got, Sk, H, a1, a2, dO, True, TOL_F32)
