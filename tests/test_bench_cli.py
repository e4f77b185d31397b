"""bench.py's host-side contract, checked without a GPU: the multi-GPU request is refused
with a message, the byte models add up, and the counter summaries parse."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_gather_model_bytes():
    m = n = 1 << 20
    nnz, r, e = 32 * m, 128, 4
    fwd = bench.kernel_bytes("fwd", m, n, nnz, r, e)
    # rowptr, colidx+val, A read, B gathered once per entry, C written
    assert fwd == 4 * (m + 1) + 8 * nnz + e * m * r + e * r * nnz + 4 * m * r
    col = bench.kernel_bytes("bwd_col", m, n, nnz, r, e)
    assert col - bench.kernel_bytes("bwd_row", m, n, nnz, r, e) == e * r * nnz  # one more gathered row per entry
    assert bench.kernel_bytes_min("fwd", m, n, nnz, r, e) < fwd


def test_committed_counter_summaries_parse():
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        if f.startswith("traffic_") and f.endswith(".json"):
            t = json.load(open(os.path.join(ROOT, "profiles", f)))
            assert t["scale"]["FETCH_SIZE"] and t["scale"]["WRITE_SIZE"]
            assert t["command"].startswith("rocprofv3")
            if "regions" in t:  # marked regions of an application bench: bytes per step
                assert all(r["bytes_per_step"] > 0 and r["dispatches"] > 0 for r in t["regions"].values())
                continue
            kernel = "batch_" if f.startswith("traffic_batch") else "line_kernel<"
            assert any(kernel in k for k in t["kernels"])


def _write_pmc(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, k, v in rows:
            fh.write(f'{i},"{k}",{counter},{v}\n')


def test_counter_calibration_when_the_runs_number_dispatches_differently(tmp_path):
    """The two counter runs may differ in launch count (the autotuner's choices): the
    calibration copies are found in each run by themselves and scale each counter."""
    kib = bench.COPY_BYTES / 1024.0
    lk = "void fmm::line_kernel<3, float, float, float, float, 32, 1, 4, 2>(fmm::LineArgs)"
    probe = "fmm::(anonymous namespace)::stream_copy_kernel(HIP_vector_type<unsigned int, 4u> const*)"
    fetch = [(1, "__amd_rocclr_copyBuffer", 2.0), (2, lk, 100.0), (3, lk, 100.0), (4, probe, 2 * kib)] + \
        [(10 + i, "__amd_rocclr_copyBuffer", kib / 2) for i in range(3)]
    write = [(1, "__amd_rocclr_copyBuffer", 4.0), (2, lk, 30.0), (3, lk, 30.0), (4, lk, 30.0), (5, lk, 30.0),
             (6, probe, 4 * kib)] + [(20 + i, "__amd_rocclr_copyBuffer", kib) for i in range(3)]
    _write_pmc(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_pmc(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = str(tmp_path / "t.json")
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), out, command="rocprofv3 test")
    t = json.load(open(out))
    assert t["scale"] == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    assert t["copy_dispatches"] == {"FETCH_SIZE": [10, 11, 12], "WRITE_SIZE": [20, 21, 22]}
    k = t["kernels"]["line_kernel<3, float, float, float, float, 32, 1, 4, 2>"]
    assert k["FETCH_SIZE"] == 100.0 and k["WRITE_SIZE"] == 30.0 and k["dispatches"] == 4
    # a write run whose largest runtime copy is not the calibration size gives no scale
    _write_pmc(str(tmp_path / "w2"), "WRITE_SIZE", write[:6])
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w2"), out)
    assert json.load(open(out))["scale"] == {"FETCH_SIZE": None, "WRITE_SIZE": None}


def test_application_byte_models():
    n, nnz, r = 1 << 20, 16 << 20, 128
    # bf16 features move fewer bytes than fp32 ones, by exactly the feature-row terms
    f32, f16 = bench.gat_forward_bytes(n, nnz, r, 4), bench.gat_forward_bytes(n, nnz, r, 2)
    assert f32 - f16 == 2 * r * (n + nnz)
    assert bench.gat_backward_bytes(n, nnz, r, 4) > 2 * f32 - 8 * n * r  # two gathering passes
    # one ALS side with no CG steps: rhs SpMM + Gram pass + CG start
    one = bench.als_sweep_bytes(n, n, nnz, r, cg_steps=0) // 2
    index = 4 * (n + 1) + 8 * nnz + 4 * r * nnz
    assert one == 2 * index + 12 * n * r + 20 * n * r + 4 * n
    per_cg = (bench.als_sweep_bytes(n, n, nnz, r, cg_steps=1) - 2 * one) // 2
    assert per_cg == index + 24 * n * r + 8 * n


def _write_stats(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "trace_kernel_stats.csv"), "w") as fh:
        fh.write("Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs\n")
        for name, calls, avg in rows:
            fh.write(f'"{name}",{calls},{calls * avg},{avg},1.0,{avg},{avg}\n')


def test_counter_table_aggregates_the_step(tmp_path):
    """Bytes per launch = FETCH x scale_f + WRITE x scale_w; the step's aggregate counts every
    hot-path launch, and the bf16 rounding only when the step rounds dC itself."""
    kib = bench.COPY_BYTES / 1024.0
    lk = "void fmm::line_kernel<3, float, float, float, float, 32, 1, 4, 2>(fmm::LineArgs)"
    rnd = "fmm::(anonymous namespace)::f32_to_bf16_x8_kernel(HIP_vector_type<float, 4u> const*)"
    cp = "__amd_rocclr_copyBuffer"
    fetch = [(1, lk, 1000.0), (2, lk, 1000.0), (3, rnd, 100.0)] + [(10 + i, cp, kib / 2) for i in range(3)]
    write = [(1, lk, 500.0), (2, lk, 500.0), (3, rnd, 50.0)] + [(10 + i, cp, kib) for i in range(3)]
    for name in ("fused_f32", "fused_bf16_dc_bf16"):
        _write_pmc(str(tmp_path / name / "f"), "FETCH_SIZE", fetch)
        _write_pmc(str(tmp_path / name / "w"), "WRITE_SIZE", write)
        _write_stats(str(tmp_path / name / "t"), [(lk, 2, 1000.0), (rnd, 1, 100.0)])
    out = str(tmp_path / "c.md")
    bench.counter_table(out, [f"{n}={tmp_path / n / 't'}:{tmp_path / n / 'f'}:{tmp_path / n / 'w'}"
                              for n in ("fused_f32", "fused_bf16_dc_bf16")])
    text = open(out).read()
    per_launch = (1000.0 * 2 + 500.0) * 1024 / 1e6          # MB: FETCH scaled by 2, WRITE by 1
    assert f"| {per_launch:.1f} |" in text
    blocks = text.split("## ")
    f32, dc16 = blocks[1], blocks[2]
    # fused_f32 sums the two line-kernel launches only; the dC step adds the rounding launch
    assert f"{2 * per_launch:.1f} (sum)" in f32
    rounding = (100.0 * 2 + 50.0) * 1024 / 1e6
    assert f"{2 * per_launch + rounding:.1f} (sum)" in dc16


def _small_workload():
    from workloads import dense_normal, rmat

    S = rmat(9, 8, seed=81)
    r = 8
    return {"S": S, "r": r, "A": dense_normal(S.m, r, 82), "B": dense_normal(S.n, r, 83),
            "G": dense_normal(S.m, r, 84)}


def test_error_report_measures_each_variant():
    """The oracle leg's error report: exact outputs give zero error, a planted error in one
    element of dB is found in dB alone, and bf16 variants are compared both ways."""
    import numpy as np

    import oracle

    w = _small_workload()
    S = w["S"]
    ST = oracle.transpose(S)
    colptr = np.concatenate([[0], np.cumsum(np.bincount(S.colidx, minlength=S.n))])
    assert np.array_equal(colptr, ST.rowptr)
    rows, cols = bench.sample_lines(S.rowptr, 64, 1), bench.sample_lines(colptr, 64, 2)
    exact = oracle.fusedmm_a_outputs_sampled(S, ST, w["A"], w["B"], w["G"], rows, cols)
    bad = tuple(x.copy() for x in exact)
    k = int(np.argmax(np.abs(bad[2]).sum(axis=1)))
    bad[2][k, 0] += 1e-3 * max(1.0, abs(bad[2][k, 0]))
    rnd = oracle.bf16_round
    bf = oracle.fusedmm_a_outputs_sampled(S, ST, w["A"], w["B"], w["G"], rows, cols, prep=(rnd, rnd, None))
    rep = bench.error_report(w, {"fused_f32": exact, "unfused_f32": bad, "fused_bf16": bf}, rows, cols)
    assert all(rep["fused_f32"][o]["componentwise"] == 0.0 for o in ("C", "dA", "dB"))
    assert rep["fused_f32"]["within_gate"]
    assert rep["unfused_f32"]["C"]["componentwise"] == 0.0 and rep["unfused_f32"]["dA"]["componentwise"] == 0.0
    assert rep["unfused_f32"]["dB"]["componentwise"] > 1e-5 and not rep["unfused_f32"]["within_gate"]
    b = rep["fused_bf16"]
    assert all(b["vs_bf16_rounded_inputs"][o]["componentwise"] == 0.0 for o in ("C", "dA", "dB"))
    assert 0.0 < b["vs_f32_inputs"]["C"]["componentwise"] <= 2e-2 and b["within_gate"]


def test_cpu_baseline_reports_its_sample():
    w = _small_workload()
    cb = bench.cpu_baseline(w, target_s=0.05, single_s=0.02)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert "median of 3 runs" in cb["sample"] and "-march=native" in cb["build"]
    assert cb["single_thread"]["cores"] == 1 and cb["cpu_model"]


def test_gather_summary_scales_each_row_size(tmp_path):
    """The gather calibration reads known bytes (rows x (row bytes + 4)) against FETCH_SIZE
    per probe kernel, and the plain copy's scale beside them."""
    kib = bench.COPY_BYTES / 1024.0
    rows = []
    for k, rb in enumerate(bench.GATHER_ROW_BYTES):
        known = (bench.PROBE_BYTES // rb) * (rb + 4)
        name = f"void fmm::(anonymous namespace)::gather_rows_kernel<{rb // 16}>(unsigned int const*)"
        rows += [(10 * k + i, name, known / 1024.0 / (1.0 + k)) for i in range(3)]
    rows += [(100 + i, "__amd_rocclr_copyBuffer", kib / 2) for i in range(3)]
    _write_pmc(str(tmp_path / "f"), "FETCH_SIZE", rows)
    out = bench.gather_summary(str(tmp_path / "f"), str(tmp_path / "g.md"), command="rocprofv3 test")
    assert [round(out[rb], 6) for rb in bench.GATHER_ROW_BYTES] == [1.0, 2.0, 3.0, 4.0]
    assert "| 2.000 |" in open(tmp_path / "g.md").read()  # the copy reads half its bytes


def test_batch_compulsory_bytes_count_every_array_once():
    m, n, nnz, r = 1000, 800, 12000, 64
    got = bench.batch_graph_bytes_min(m, n, nnz, r, 2, 4)
    index = 4 * (m + 1) + 8 * nnz + 4 * (n + 1) + 8 * nnz      # CSR and CSC, values included
    dense = 2 * m * r + 2 * n * r + 4 * m * r + 4 * m * r + 4 * m * r + 4 * n * r  # A, B, dC, C, dA, dB
    assert got == index + dense


def test_marked_summary_counts_only_the_marked_regions(tmp_path):
    """Bytes per step of each region = the dispatches strictly between its two markers,
    FETCH x 2 and WRITE x 1 (the copy calibration), divided by the step count."""
    kib = bench.COPY_BYTES / 1024.0
    mk = "fmm::(anonymous namespace)::stream_read_kernel(unsigned int __vector(4) const*, unsigned long)"
    k = "void fmm::gat_kernel<float, 32>(fmm::GatArgs)"
    cp = "__amd_rocclr_copyBuffer"
    fetch = [(1, k, 999.0), (2, mk, 0.1), (3, k, 10.0), (4, k, 30.0), (5, mk, 0.1), (6, k, 7.0), (7, mk, 0.1)] + \
        [(20 + i, cp, kib / 2) for i in range(3)]
    write = [(1, k, 999.0), (2, mk, 0.0), (3, k, 1.0), (4, k, 3.0), (5, mk, 0.0), (6, k, 5.0), (7, mk, 0.0)] + \
        [(20 + i, cp, kib) for i in range(3)]
    _write_pmc(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_pmc(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = str(tmp_path / "traffic_gat_rmat20_r128_h4.json")
    bench.marked_summary(str(tmp_path / "f"), str(tmp_path / "w"), out, ["fwd_f32", "bwd_f32"], 2,
                         "gat_rmat20_r128_h4", command="rocprofv3 test")
    t = json.load(open(out))
    assert t["regions"]["fwd_f32"]["bytes_per_step"] == int(1024 * ((10 + 30) * 2 + (1 + 3)) / 2)
    assert t["regions"]["bwd_f32"]["bytes_per_step"] == int(1024 * (7 * 2 + 5) / 2)
    assert t["regions"]["fwd_f32"]["dispatches"] == 2


def test_tuning_arg_round_trips():
    t = {"csr": {"variant": 3, "long_len": 256, "line_order": False, "gather_hints": 32768},
         "csc": {"variant": 1, "long_len": None, "line_order": True, "gather_hints": None}}
    arg = bench.tuning_arg(t)
    assert arg == "csr=3:256:0:32768,csc=1:0:1:0"
    assert bench.parse_tuning_arg(arg) == t
    old = bench.parse_tuning_arg("csr=3:256:1,csc=3:256:0")  # the form without hints
    assert old["csr"]["gather_hints"] is None and old["csr"]["line_order"] is True


def test_trace_summary_reports_the_timed_region(tmp_path):
    """Launches between the first two marker dispatches of a kernel trace are averaged on
    their own, next to the statistics of the whole run."""
    d = tmp_path / "t"
    os.makedirs(d)
    mk = "fmm::(anonymous namespace)::stream_read_kernel(unsigned int __vector(4) const*, unsigned long)"
    lk = "void fmm::line_kernel<4, float, float, float, float, 64, 1, 4, 1>(fmm::LineArgs, int)"
    rows = [(lk, 0, 30), (mk, 100, 101), (lk, 200, 210), (lk, 300, 312), (mk, 400, 401), (lk, 500, 540)]
    with open(d / "trace_kernel_trace.csv", "w") as fh:
        fh.write("Kind,Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for k, a, b in rows:
            fh.write(f'KERNEL_DISPATCH,"{k}",{a * 1000},{b * 1000}\n')
    _write_stats(str(d), [(lk, 4, 23000.0), (mk, 2, 1000.0)])
    out = str(tmp_path / "s.md")
    bench.trace_summary(str(d), out)
    text = open(out).read()
    assert "| 2 | 11.0 |" in text  # two timed launches of 10 and 12 us


def test_sq_summary_reports_valu_issue_use(tmp_path, monkeypatch):
    """VALU issue use = VALU wave-instructions over busy CU-cycles, per hot-path kernel and
    run; the bench lines read it back while the sources match."""
    lk = "void fmm::line_kernel<4, float, float, float, float, 64, 1, 4, 1>(fmm::LineArgs, int)"
    other = "some_torch_kernel"
    d = tmp_path / "run"
    os.makedirs(d)
    vals = {"SQ_INSTS_VALU": 300.0, "SQ_BUSY_CU_CYCLES": 1000.0, "SQ_ACTIVE_INST_VALU": 310.0,
            "SQ_INSTS_VALU_FMA_F32": 150.0, "SQ_INSTS_VMEM_RD": 40.0, "SQ_INSTS_FLAT": 10.0,
            "SQ_INSTS_SALU": 20.0, "SQ_WAVES": 8.0}
    with open(d / "pmc_counter_collection.csv", "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i in (1, 2):  # two dispatches of the line kernel, the second twice as long
            for c, v in vals.items():
                fh.write(f'{i},"{lk}",{c},{v * i}\n')
        for c, v in vals.items():  # not a hot-path kernel: left out
            fh.write(f'3,"{other}",{c},{v}\n')
    prof = tmp_path / "profiles"
    os.makedirs(prof)
    table = bench.sq_summary(str(prof / "sq_issue.md"), [f"rmat22_ef16_r256={d}"], command="rocprofv3 test")
    k = table["rmat22_ef16_r256"]["kernels"]["line_kernel<4, float, float, float, float, 64, 1, 4, 1>"]
    assert k["dispatches"] == 2 and abs(k["valu_issue_frac"] - 0.3) < 1e-12 and abs(k["fma_share_of_valu"] - 0.5) < 1e-12
    assert len(table["rmat22_ef16_r256"]["kernels"]) == 1
    # the run is keyed to the line-kernel sources (a batch-only change leaves it valid)
    assert table["rmat22_ef16_r256"]["source_hash"] == bench.source_hash(bench.SRC_GLOBS)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    stored = json.load(open(prof / "sq_issue.json"))["runs"]["rmat22_ef16_r256"]["source_hash"]
    monkeypatch.setattr(bench, "source_hash", lambda globs=None: stored)
    assert abs(bench.load_valu_issue("rmat22_ef16_r256", "line_kernel<4, float") - 0.3) < 1e-12
    assert bench.load_valu_issue("batch256_r64", "void fmm::batch_queue_kernel") is None
    monkeypatch.setattr(bench, "source_hash", lambda globs=None: "another")
    assert bench.load_valu_issue("rmat22_ef16_r256", "line_kernel<4, float") is None
