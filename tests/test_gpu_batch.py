"""Batched persistent launch over many uneven graphs: equality with the single-graph
calls (bit for bit under the row-block schedule), oracle parity for every schedule,
autotuning, and hipGraph replay against the eager launch."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_07673_amd as F
from tests.gates import TOL_BF16, TOL_F32
from tests.gpu_helpers import gate, host, log, ref_fusedmm_a, ref_fusedmm_a_backward
from workloads import batch_er

pytestmark = pytest.mark.gpu


def _setup(dtype, nbatch=12, r=64, seed=77):
    graphs = batch_er(nbatch, r, seed=seed, nmin=64, nmax=4096, dmin=8, dmax=64)
    pats = [F.Pattern.from_csr(g["S"]) for g in graphs]
    A32 = [torch.from_numpy(g["A"]).cuda() for g in graphs]
    B32 = [torch.from_numpy(g["B"]).cuda() for g in graphs]
    G = [torch.from_numpy(g["G"]).cuda() for g in graphs]
    if dtype == torch.bfloat16:
        A = [F.to_bf16(a) for a in A32]
        B = [F.to_bf16(b) for b in B32]
    else:
        A, B = A32, B32
    return graphs, pats, A, B, G


def _single(pats, A, B, G):
    out = []
    for P, a, b, g in zip(pats, A, B, G):
        c, _ = F.fusedmm_a_raw(P, a, b)
        da, db = F.fusedmm_a_backward_raw(P, a, b, g)
        out.append((c, da, db))
    torch.cuda.synchronize()
    return out


def _check_oracle(graphs, plan, tol, tag):
    for k, g in enumerate(graphs):
        S, A, B, G = g["S"], g["A"], g["B"], g["G"]
        ref, mag = ref_fusedmm_a(S, A, B)
        gate(f"{tag} graph {k} C", host(plan.C[k]), ref, mag, tol)
        dA, dB, mA, mB = ref_fusedmm_a_backward(S, A, B, G)
        gate(f"{tag} graph {k} dA", host(plan.dA[k]), dA, mA, tol)
        gate(f"{tag} graph {k} dB", host(plan.dB[k]), dB, mB, tol)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batch_row_block_equals_single_graph_calls(dtype):
    graphs, pats, A, B, G = _setup(dtype)
    log(f"batch row-block dtype={dtype} graphs={len(graphs)}")
    plan = F.BatchPlan(pats, A, B, G)
    single = _single(pats, A, B, G)
    for place in (F.BatchPlan.PLACE_XCD, F.BatchPlan.PLACE_GLOBAL, F.BatchPlan.PLACE_QUEUES):
        plan.set_schedule(tile_nnz=2048, placement=place, row_wave=False, col_wave=False)
        for rep in range(2):  # the queue counters start from zero again on the second launch
            for t in plan.C + plan.dA + plan.dB:
                t.fill_(float("nan"))
            log(f"batch row-block placement={place} launch {rep}")
            plan.run()
            torch.cuda.synchronize()
            for k, (c, da, db) in enumerate(single):
                assert torch.equal(plan.C[k], c), (k, place, rep)
                assert torch.equal(plan.dA[k], da), (k, place, rep)
                assert torch.equal(plan.dB[k], db), (k, place, rep)
    _check_oracle(graphs, plan, TOL_BF16 if dtype == torch.bfloat16 else TOL_F32, "row-block")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batch_wave_schedules_and_autotune(dtype):
    graphs, pats, A, B, G = _setup(dtype, seed=78)
    tol = TOL_BF16 if dtype == torch.bfloat16 else TOL_F32
    plan = F.BatchPlan(pats, A, B, G)
    for place in (F.BatchPlan.PLACE_XCD, F.BatchPlan.PLACE_QUEUES):
        for rw, cw in ((True, False), (False, True), (True, True)):
            log(f"batch wave rw={rw} cw={cw} placement={place} dtype={dtype}")
            plan.set_schedule(tile_nnz=8192, placement=place, row_wave=rw, col_wave=cw)
            plan.run()
            torch.cuda.synchronize()
            _check_oracle(graphs, plan, tol, f"wave rw={rw} cw={cw} placement={place}")
            first = [t.clone() for t in plan.C + plan.dA + plan.dB]
            plan.run()
            torch.cuda.synchronize()
            assert all(torch.equal(x, y) for x, y in zip(first, plan.C + plan.dA + plan.dB))  # repeatable
    log("batch autotune")
    info = plan.autotune()
    assert info["n_candidates"] >= 18 and info["best_ms"] > 0
    plan.run()
    torch.cuda.synchronize()
    _check_oracle(graphs, plan, tol, "autotuned")


@pytest.mark.parametrize("how", ["autotuned", "queues"])
def test_batch_graph_replay_matches_eager(how):
    graphs, pats, A, B, G = _setup(torch.bfloat16, seed=79)
    plan = F.BatchPlan(pats, A, B, G)
    log(f"batch {how} + capture")
    if how == "autotuned":
        plan.autotune()
    else:  # the queue counters must be back at zero for every replay
        plan.set_schedule(tile_nnz=2048, placement=F.BatchPlan.PLACE_QUEUES)
    plan.run()
    torch.cuda.synchronize()
    eager = [t.clone() for t in plan.C + plan.dA + plan.dB]
    side = torch.cuda.Stream()
    with pytest.raises(F.FmmError):
        plan.launch(side)  # nothing captured yet
    plan.capture(side)
    assert plan.info()["graph_captured"] == 1
    for rep in range(3):
        for t in plan.C + plan.dA + plan.dB:
            t.zero_()  # eager work between replays
        torch.cuda.synchronize()
        plan.launch(side)
        side.synchronize()
        assert all(torch.equal(x, y) for x, y in zip(eager, plan.C + plan.dA + plan.dB)), rep
    plan.set_schedule(tile_nnz=2048)  # a new schedule makes the captured graph stale
    assert plan.info()["graph_captured"] == 0
    with pytest.raises(F.FmmError):
        plan.launch(side)


def test_batch_bf16_upstream_gradient():
    """bf16 A, B and dC (FMM_BATCH_DC_BF16): every graph's adjoint within the float32 gate
    of the oracle on the rounded A, B, dC, and within the bf16 gate of the oracle on the
    float32 originals, under a row-block, a wavefront and the autotuned schedule."""
    graphs, pats, A, B, G = _setup(torch.bfloat16, nbatch=8, seed=81)
    G16 = [F.to_bf16(g) for g in G]
    plan = F.BatchPlan(pats, A, B, G16)

    def check(tag):
        plan.run()
        torch.cuda.synchronize()
        for k, g in enumerate(graphs):
            S = g["S"]
            Aq, Bq, Gq = oracle.bf16_round(g["A"]), oracle.bf16_round(g["B"]), oracle.bf16_round(g["G"])
            dA, dB, mA, mB = ref_fusedmm_a_backward(S, Aq, Bq, Gq)
            gate(f"{tag} graph {k} dA", host(plan.dA[k]), dA, mA, TOL_F32)
            gate(f"{tag} graph {k} dB", host(plan.dB[k]), dB, mB, TOL_F32)
            dA, dB, mA, mB = ref_fusedmm_a_backward(S, g["A"], g["B"], g["G"])
            gate(f"{tag} graph {k} dB vs float32 inputs", host(plan.dB[k]), dB, mB, TOL_BF16)
    for rw, cw, place in ((False, False, F.BatchPlan.PLACE_XCD), (True, True, F.BatchPlan.PLACE_XCD),
                          (False, False, F.BatchPlan.PLACE_QUEUES)):
        log(f"batch bf16 dC rw={rw} cw={cw} placement={place}")
        plan.set_schedule(tile_nnz=2048, placement=place, row_wave=rw, col_wave=cw)
        check(f"bf16 dC rw={rw} cw={cw} placement={place}")
    log("batch bf16 dC autotune")
    plan.autotune()
    check("bf16 dC autotuned")


def test_batch_forward_only_and_oracle_bf16_rounded():
    graphs, pats, A, B, G = _setup(torch.bfloat16, nbatch=5, seed=80)
    with pytest.raises(TypeError):  # one dC dtype for every graph
        F.BatchPlan(pats, A, B, [F.to_bf16(g) for g in G[:-1]] + [G[-1]])
    with pytest.raises(TypeError):  # float32 storage takes a float32 dC only
        F.BatchPlan(pats, [a.float() for a in A], [b.float() for b in B], [F.to_bf16(g) for g in G])
    plan = F.BatchPlan(pats, A, B, forward=True, backward=False)
    log("batch forward only")
    plan.run()
    torch.cuda.synchronize()
    assert plan.dA is None
    for k, g in enumerate(graphs):
        Ar, Br = oracle.bf16_round(g["A"]), oracle.bf16_round(g["B"])
        ref, mag = ref_fusedmm_a(g["S"], Ar, Br)
        gate(f"fwd-only graph {k}", host(plan.C[k]), ref, mag, TOL_F32)


@pytest.mark.timeout(900)
def test_batch256_autotuned_plan_at_full_size():
    """The bench's batch at its own size (256 ER graphs, n log-uniform in [1024, 65536],
    degree uniform in [8, 64], r = 64, bfloat16 storage): after autotuning, the largest and
    the smallest graphs, and the densest one, checked in full against the oracle (on the
    bf16-rounded A and B at the float32 gate, and on the float32 originals at the bf16
    gate)."""
    r = 64
    graphs = batch_er(256, r, seed=5)
    ns = np.array([g["S"].m for g in graphs])
    dens = np.array([g["S"].nnz / max(1, g["S"].m) for g in graphs])
    pick = sorted({int(np.argmax(ns)), int(np.argmin(ns)), int(np.argmax(dens))})
    log(f"batch256: {len(graphs)} graphs, n {ns.min()}..{ns.max()}, checking {pick}")
    pats = [F.Pattern.from_csr(g["S"]) for g in graphs]
    A = [F.to_bf16(torch.from_numpy(g["A"]).cuda()) for g in graphs]
    B = [F.to_bf16(torch.from_numpy(g["B"]).cuda()) for g in graphs]
    G = [torch.from_numpy(g["G"]).cuda() for g in graphs]
    plan = F.BatchPlan(pats, A, B, G)
    log("batch256 autotune")
    info = plan.autotune()
    log(f"batch256 tuned: {info}")
    side = torch.cuda.Stream()
    plan.capture(side)
    for t in plan.C + plan.dA + plan.dB:
        t.fill_(float("nan"))
    torch.cuda.synchronize()
    plan.launch(side)
    side.synchronize()
    for k in pick:
        g = graphs[k]
        S = g["S"]
        log(f"batch256 graph {k}: n={S.m} nnz={S.nnz}")
        Aq, Bq = oracle.bf16_round(g["A"]), oracle.bf16_round(g["B"])
        ref, mag = ref_fusedmm_a(S, Aq, Bq)
        gate(f"batch256 graph {k} C", host(plan.C[k]), ref, mag, TOL_F32)
        dA, dB, mA, mB = ref_fusedmm_a_backward(S, Aq, Bq, g["G"])
        gate(f"batch256 graph {k} dA", host(plan.dA[k]), dA, mA, TOL_F32)
        gate(f"batch256 graph {k} dB", host(plan.dB[k]), dB, mB, TOL_F32)
        ref, mag = ref_fusedmm_a(S, g["A"], g["B"])
        gate(f"batch256 graph {k} C vs float32 inputs", host(plan.C[k]), ref, mag, TOL_BF16)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batch_patterns_without_values(dtype):
    """Graphs whose pattern stores no values (every weight 1) mixed with valued ones: with
    tiles whose operands are staged in LDS (2048 entries) and tiles that are not (8192), the
    row-block schedule equals the single-graph calls bit for bit, and the oracle with unit
    weights holds at the float32 gate."""
    from workloads import CsrPattern
    graphs, _, A, B, G = _setup(dtype, nbatch=6, seed=97)
    pats = []
    for k, g in enumerate(graphs):
        S = g["S"]
        if k % 2 == 0:  # drop the values: the pattern alone
            pats.append(F.Pattern(S.rowptr, S.colidx, None, (S.m, S.n)))
            g["S"] = CsrPattern(S.m, S.n, S.rowptr, S.colidx, np.ones(S.nnz, dtype=np.float32))
        else:
            pats.append(F.Pattern.from_csr(S))
    plan = F.BatchPlan(pats, A, B, G)
    single = _single(pats, A, B, G)
    for tile in (2048, 8192):
        log(f"batch without values dtype={dtype} tile={tile}")
        plan.set_schedule(tile_nnz=tile, placement=F.BatchPlan.PLACE_QUEUES, row_wave=False, col_wave=False)
        for t in plan.C + plan.dA + plan.dB:
            t.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        for k, (c, da, db) in enumerate(single):
            assert torch.equal(plan.C[k], c) and torch.equal(plan.dA[k], da) and torch.equal(plan.dB[k], db), (k, tile)
    for k, g in enumerate(graphs):
        S, Aq, Bq = g["S"], g["A"], g["B"]
        if dtype == torch.bfloat16:
            Aq, Bq = oracle.bf16_round(Aq), oracle.bf16_round(Bq)
        ref, mag = ref_fusedmm_a(S, Aq, Bq)
        gate(f"no-values graph {k} C", host(plan.C[k]), ref, mag, TOL_F32)
        dA, dB, mA, mB = ref_fusedmm_a_backward(S, Aq, Bq, g["G"])
        gate(f"no-values graph {k} dA", host(plan.dA[k]), dA, mA, TOL_F32)
        gate(f"no-values graph {k} dB", host(plan.dB[k]), dB, mB, TOL_F32)


@pytest.mark.parametrize("dtype,r", [(torch.float32, 4), (torch.float32, 256), (torch.bfloat16, 8),
                                     (torch.bfloat16, 512)])
def test_batch_smallest_and_widest_r(dtype, r):
    """The narrowest rows of each storage type (one 16-byte vector: most lanes of a group
    idle) and the widest a batch plan takes (64 lanes of 16 bytes): both schedules, staged
    and unstaged tiles, bit-exact against the single-graph calls under the row-block schedule
    and within the float32 gate of the oracle on the stored inputs."""
    graphs, pats, A, B, G = _setup(dtype, nbatch=5, r=r, seed=98)
    log(f"batch r={r} dtype={dtype}")
    plan = F.BatchPlan(pats, A, B, G)
    single = _single(pats, A, B, G)
    for tile, rw, cw in ((2048, False, False), (8192, False, False), (2048, True, True)):
        plan.set_schedule(tile_nnz=tile, placement=F.BatchPlan.PLACE_QUEUES, row_wave=rw, col_wave=cw)
        for t in plan.C + plan.dA + plan.dB:
            t.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        if not (rw or cw):
            for k, (c, da, db) in enumerate(single):
                assert torch.equal(plan.C[k], c) and torch.equal(plan.dA[k], da) and torch.equal(plan.dB[k], db), \
                    (k, tile)
        _check_oracle_stored(graphs, plan, dtype, f"r={r} tile={tile} rw={rw} cw={cw}")


def _check_oracle_stored(graphs, plan, dtype, tag):
    """Every graph against the oracle on the inputs as stored (bf16-rounded for bf16), at the
    float32 gate."""
    for k, g in enumerate(graphs):
        S, Aq, Bq = g["S"], g["A"], g["B"]
        if dtype == torch.bfloat16:
            Aq, Bq = oracle.bf16_round(Aq), oracle.bf16_round(Bq)
        ref, mag = ref_fusedmm_a(S, Aq, Bq)
        gate(f"{tag} graph {k} C", host(plan.C[k]), ref, mag, TOL_F32)
        dA, dB, mA, mB = ref_fusedmm_a_backward(S, Aq, Bq, g["G"])
        gate(f"{tag} graph {k} dA", host(plan.dA[k]), dA, mA, TOL_F32)
        gate(f"{tag} graph {k} dB", host(plan.dB[k]), dB, mB, TOL_F32)
