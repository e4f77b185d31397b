"""Benchmark: fused FusedMMA forward + adjoint on one MI355X.

One step = C = FusedMMA(S, A, B) (fused), then the adjoint for the loss sum(C * G):
dA (row pass over the CSR) and dB (column pass over the stored transpose).  Inputs
are seeded synthetic data resident in HBM before timing starts.  The default
workload is R-MAT scale 22 (4,194,304 vertices, edge factor 16, duplicates removed:
65.2M stored entries with power-law row and column lengths), r = 256, float32; the
paper's skewed real-world matrices are not available and this stands in for them.

Prints one JSON line with the step throughput (GFLOP/s, counting 12 r nnz flops per
step as the paper counts SDDMM and SpMM at 2 r nnz each), the roofline entry of the
dominant kernel (timed with HIP events on the launch stream; its fraction of the HBM
peak under the gather, compulsory and counter byte counts), side measurements (unfused
float32 and fused bfloat16 steps, FusedMMB), and the oracle leg: the error of every
output of each variant against the FP64 oracle on sampled lines, and the oracle's own
throughput on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "FusedMM fwd+bwd GFLOP/s and % HBM peak; fused/BF16 vs unfused FP32 at tol"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(kind, m, n, nnz, r, e):
    """Algorithmic HBM bytes of one launch under the gather model (every stored
    entry fetches its dense row; index arrays, held rows and outputs move once)."""
    if kind == "fwd":        # FusedMMA: rowptr, colidx+val, A, gathered B, C
        return 4 * (m + 1) + 8 * nnz + e * m * r + e * r * nnz + 4 * m * r
    if kind == "bwd_row":    # dA = FusedMMA(S, dC, B): rowptr, colidx+val, dC, gathered B, dA
        return 4 * (m + 1) + 8 * nnz + 4 * m * r + e * r * nnz + 4 * m * r
    if kind == "bwd_col":    # dB: colptr, rowidx+valT, B, gathered A and dC, dB
        return 4 * (n + 1) + 8 * nnz + e * n * r + (e + 4) * r * nnz + 4 * n * r
    raise ValueError(kind)


def kernel_bytes_min(kind, m, n, nnz, r, e):
    """Compulsory bytes: every array once (no re-fetch of gathered rows)."""
    if kind == "fwd":
        return 4 * (m + 1) + 8 * nnz + e * m * r + e * n * r + 4 * m * r
    if kind == "bwd_row":
        return 4 * (m + 1) + 8 * nnz + 4 * m * r + e * n * r + 4 * m * r
    if kind == "bwd_col":
        return 4 * (n + 1) + 8 * nnz + e * n * r + (e + 4) * m * r + 4 * n * r
    raise ValueError(kind)


def batch_graph_bytes_min(m, n, nnz, r, e, ed):
    """Compulsory bytes of one graph's fused forward + adjoint in the batched launch: the CSR
    and CSC index arrays and values, A and B (e bytes per element), dC (ed), and the outputs
    C, dA, dB (float32), each once."""
    return 4 * (m + 1) + 8 * nnz + 4 * (n + 1) + 8 * nnz + e * (m + n) * r + ed * m * r + 4 * (2 * m + n) * r


def gat_forward_bytes(n, nnz, r, e):
    """Gather-model bytes of one attention head's forward: the scores pass reads H once and
    writes s, t; the line pass reads rowptr, colidx + value and t_j per entry, gathers H_j
    per entry and writes out and lse per row."""
    return e * n * r + 8 * n + 4 * (n + 1) + nnz * (8 + 4 + e * r) + n * (4 * r + 4 + 4)


def gat_backward_bytes(n, nnz, r, e):
    """Gather-model bytes of one attention head's adjoint: the row pass (held dO_i and
    out_i, per entry colidx + value, t_j and a gathered H_j, dS written) writes D_i and the
    packed row scalars; the column pass (held H_j, per entry rowidx + value, the packed row
    scalars and a gathered dO_i) writes dt_j and dH_j; the da pass reads H, ds and dt."""
    rows = 4 * (n + 1) + n * (8 * r + 8) + nnz * (8 + 4 + e * r + 4) + n * (4 + 12)
    cols = 4 * (n + 1) + n * (e * r + 4 * r + 4) + nnz * (8 + 12 + 4 * r)
    da = n * (e * r + 8)
    return rows + cols + da


def als_sweep_bytes(m, n, nnz, r, cg_steps=10):
    """Gather-model bytes of one ALS sweep (float32 factors): per side, the right-hand
    side SpMM, the Gram pass of the start vector, the CG start (reads b, q, x; writes r, p)
    and cg_steps fused CG passes, each holding p_i, gathering F_j per entry, reading X and
    R and writing X, R, P and <R, R>."""
    def side(lines):
        index = 4 * (lines + 1) + 8 * nnz + 4 * r * nnz
        rhs = index + 4 * lines * r
        gram = index + 8 * lines * r
        start = 20 * lines * r + 4 * lines
        cg = index + 24 * lines * r + 8 * lines
        return rhs + gram + start + cg_steps * cg
    return side(m) + side(n)


def sample_lines(ptr, k, seed):
    """A seeded sample of lines for the error report: k random lines, the 16 longest (split
    lines on R-MAT) and up to 8 empty ones, sorted and unique."""
    lens = np.diff(np.asarray(ptr, dtype=np.int64))
    rng = np.random.default_rng(seed)
    rand = rng.choice(lens.shape[0], size=min(k, lens.shape[0]), replace=False)
    longest = np.argsort(lens, kind="stable")[-16:]
    empty = np.flatnonzero(lens == 0)[:8]
    return np.unique(np.concatenate([rand, longest, empty])).astype(np.int64)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s=5.0, single_s=3.0, reps=3):
    """The FP64 oracle (FusedMMA forward + adjoint) timed on the first K rows of the same
    workload: its -O3 -march=native build (same source and arithmetic as the parity build),
    with all of the host's threads (the reported value) and with one thread, median of
    `reps` runs each.  Only the rows of A, B and G the sample touches are promoted to
    float64 (restrict_rows), outside the timed region."""
    import oracle

    S, r = w["S"], w["r"]
    oracle.select_build("native")

    def prep(K):
        Sk, cols = oracle.restrict_rows(S, np.arange(K))
        return (Sk, np.ascontiguousarray(w["A"][:K], dtype=np.float64),
                np.ascontiguousarray(w["B"][cols], dtype=np.float64),
                np.ascontiguousarray(w["G"][:K], dtype=np.float64))

    def run(args):
        Sk, Ak, Bk, Gk = args
        t0 = time.perf_counter()
        oracle.fusedmm_a(Sk, Ak, Bk)
        oracle.fusedmm_a_backward(Sk, Ak, Bk, Gk)
        return time.perf_counter() - t0

    def sample(K, target):
        # grow the row sample until one run takes at least half the target time, then
        # take the median of `reps` runs
        args = prep(K)
        t = run(args)
        while t < 0.5 * target and K < S.m:
            K = int(min(S.m, max(2 * K, K * target / max(t, 1e-3))))
            args = prep(K)
            t = run(args)
        ts = [t] + [run(args) for _ in range(reps - 1)]
        return K, float(np.median(ts)), ts, int(S.rowptr[K])

    threads = oracle.num_threads()
    K, t, ts, nz = sample(min(S.m, 8192), target_s)
    oracle.set_num_threads(1)
    try:
        K1, t1, ts1, nz1 = sample(min(S.m, 1024), single_s)
    finally:
        oracle.set_num_threads(threads)
    oracle.select_build("default")
    runs = lambda x: ", ".join(f"{v:.2f}" for v in x)  # noqa: E731
    return {"value": round(12.0 * r * nz / t / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "build": "gcc " + oracle.build_flags("native"),
            "sample": f"first {K} of {S.m} rows ({nz} nonzeros), FusedMMA forward + adjoint in float64, "
                      f"median of {len(ts)} runs ({runs(ts)} s)",
            "single_thread": {"value": round(12.0 * r * nz1 / t1 / 1e9, 3), "cores": 1,
                              "sample": f"first {K1} rows ({nz1} nonzeros), median of {len(ts1)} runs "
                                        f"({runs(ts1)} s)"}}


def error_report(w, outputs, rows, cols):
    """Error of every output of each measured step variant against the FP64 oracle, on the
    sampled rows of C and dA and the sampled columns of dB (exact for those outputs: lines
    are independent).  For each output: componentwise max |x - ref| / mag, with mag the
    oracle on absolute values (the gate of the parity tests), and normwise
    ||x - ref||_F / ||ref||_F.  bfloat16 variants are compared with the oracle on the
    float32 inputs (storage error included) and on the bf16-rounded inputs (accumulation
    error alone)."""
    import oracle

    S = w["S"]
    ST = oracle.transpose(S)
    SA, STA = oracle.absolute(S), oracle.absolute(ST)
    A, B, G = w["A"], w["B"], w["G"]
    rnd, ab = oracle.bf16_round, np.abs
    rab = lambda x: np.abs(oracle.bf16_round(x))  # noqa: E731
    refs = {}

    def ref(kind):
        if kind not in refs:
            pa, pg = {"f32": ((None, None, None), (ab, ab, ab)),
                      "bf16": ((rnd, rnd, None), (rab, rab, ab)),
                      "bf16_dc": ((rnd, rnd, rnd), (rab, rab, rab))}[kind]
            refs[kind] = (oracle.fusedmm_a_outputs_sampled(S, ST, A, B, G, rows, cols, prep=pa),
                          oracle.fusedmm_a_outputs_sampled(SA, STA, A, B, G, rows, cols, prep=pg))
        return refs[kind]

    def errs(got, kind):
        (rC, rA, rB), (mC, mA, mB) = ref(kind)
        out = {}
        for name, x, r, m in (("C", got[0], rC, mC), ("dA", got[1], rA, mA), ("dB", got[2], rB, mB)):
            zero = m == 0
            comp = float("inf") if np.any(x[zero] != 0) else \
                float(np.max(np.abs(x - r)[~zero] / m[~zero], initial=0.0))
            den = np.linalg.norm(r)
            out[name] = {"componentwise": float(f"{comp:.3e}"),
                         "normwise": float(f"{(np.linalg.norm(x - r) / den if den > 0 else 0.0):.3e}")}
        return out

    rep = {"sample": f"{rows.size} rows of C and dA, {cols.size} columns of dB (random, the 16 longest, "
                     f"empty ones); seeded",
           "gate": {"f32": 1e-5, "bf16_storage": 2e-2},
           "measure": "componentwise max|x-ref|/mag (mag: the oracle on absolute values); normwise "
                      "||x-ref||_F/||ref||_F"}
    for v, got in outputs.items():
        if v.startswith("fused_bf16"):
            kind = "bf16_dc" if v.endswith("dc_bf16") else "bf16"
            rep[v] = {"vs_f32_inputs": errs(got, "f32"), "vs_bf16_rounded_inputs": errs(got, kind)}
            rep[v]["within_gate"] = all(x["componentwise"] <= 2e-2 for x in rep[v]["vs_f32_inputs"].values())
        else:
            rep[v] = errs(got, "f32")
            rep[v]["within_gate"] = all(x["componentwise"] <= 1e-5 for x in rep[v].values() if isinstance(x, dict))
    return rep


COPY_BYTES = 1 << 30
# the sources that define the line kernels (their counters go stale when these change)
SRC_GLOBS = ("paper_2203_07673_amd/csrc/fmm_lines.hpp", "paper_2203_07673_amd/csrc/fmm_launch.hpp",
             "paper_2203_07673_amd/csrc/lines_*.hip")
# and those of the batched persistent kernel, which runs the same per-line body
BATCH_SRC_GLOBS = SRC_GLOBS + ("paper_2203_07673_amd/csrc/batch*.hip", "paper_2203_07673_amd/csrc/batch_kernels.hpp")


def source_globs(workload_name):
    return BATCH_SRC_GLOBS if workload_name.startswith("batch") else SRC_GLOBS


def source_hash(globs=SRC_GLOBS):
    """SHA-256 over the HIP sources: counter data is valid only for the kernels it measured."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for pat in globs:
        for f in sorted(glob.glob(os.path.join(ROOT, pat))):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _csv_rows(d, suffix):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _short_kernel(name):
    if "line_kernel<" in name:
        return "line_kernel<" + name.split("line_kernel<", 1)[1].split(">", 1)[0] + ">"
    return name[:120]


def calibration_dispatches(per):
    """Dispatch ids of the plain copies --calibrate-copy ran: the runtime's copy-kernel
    dispatches (not the library's streaming probes) whose counter reads within 1% of the
    largest copy reading of the run (the calibration copy of COPY_BYTES is larger than any
    copy the workload makes)."""
    copies = {i: v for i, (k, v) in per.items() if "copy" in k.lower() and "fmm::" not in k}
    if not copies:
        return []
    top = max(copies.values())
    return sorted(i for i, v in copies.items() if top > 0 and abs(v - top) < 0.01 * top)


def pmc_summary(fetch_dir, write_dir, out_json, command="", workload_name=None, tuned=""):
    """Per-kernel FETCH_SIZE / WRITE_SIZE (KiB per dispatch) from two counter runs of the
    same command, with scale factors from the plain device copy of COPY_BYTES bytes that
    --calibrate-copy ran.  The copies are found in each run on its own, as its largest
    copy dispatches (those of the write run must each write COPY_BYTES): the autotuner
    may make a different number of launches in the two runs, so their dispatch numbers
    need not line up."""
    runs = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        runs[counter] = {}
        for row in _csv_rows(d, "counter_collection.csv"):
            if row.get("Counter_Name") == counter:
                runs[counter][int(row["Dispatch_Id"])] = (row["Kernel_Name"], float(row["Counter_Value"]))
    want_kib = COPY_BYTES / 1024.0
    calib = {c: calibration_dispatches(per) for c, per in runs.items()}
    scale = {"FETCH_SIZE": None, "WRITE_SIZE": None}
    w = calib["WRITE_SIZE"]
    # the write run names the copies (each writes COPY_BYTES); the fetch run must hold as many
    if w and all(abs(runs["WRITE_SIZE"][i][1] - want_kib) < 0.01 * want_kib for i in w) \
            and len(calib["FETCH_SIZE"]) == len(w):
        for c in scale:
            mean = sum(runs[c][i][1] for i in calib[c]) / len(calib[c])
            scale[c] = want_kib / mean if mean > 0 else None
    else:
        calib = {c: [] for c in runs}
    kernels = {}
    for c, per in runs.items():
        for i, (k, v) in per.items():
            if i in calib[c]:
                continue
            kernels.setdefault(_short_kernel(k), {}).setdefault(c, []).append(v)
    summary = {}
    for k, v in kernels.items():
        summary[k] = {c: sum(x) / len(x) for c, x in v.items()}
        summary[k]["dispatches"] = max(len(x) for x in v.values())
    if workload_name is None:  # traffic_<workload>.json
        workload_name = os.path.basename(out_json)[len("traffic_"):].rsplit(".", 1)[0]
    out = {"command": command, "source_hash": source_hash(source_globs(workload_name)), "copy_bytes": COPY_BYTES,
           "copy_dispatches": {c: sorted(v) for c, v in calib.items()}, "scale": scale, "tuned_arg": tuned,
           "note": "KiB per dispatch as the counters read them; bytes = (FETCH*scale_f + WRITE*scale_w)*1024",
           "kernels": summary}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


ROUNDING = "bf16 rounding (A, B once; dC every step with a bf16 upstream gradient)"
ROLES = {0: "SDDMM", 1: "SpMM, one operand", 2: "SpMM, two operands (dB = dP^T A + R^T dC)",
         3: "fused one-row (FusedMMA forward / adjoint row pass)", 4: "fused two-row (adjoint column pass)"}


def _role(key):
    if key.startswith("line_kernel<"):
        return ROLES.get(int(key[len("line_kernel<"):].split(",", 1)[0]), "line kernel")
    if "merge_kernel" in key:
        return "split-line merge"
    if "batch_kernel<" in key:
        return "batched persistent (all passes of every graph)"
    if "batch_queue_kernel<" in key:
        return "batched persistent, XCD queues (all passes of every graph)"
    if "f32_to_bf16" in key:
        return ROUNDING
    return None


def _pmc_per_key(d, counter):
    per = {}
    for row in _csv_rows(d, "counter_collection.csv"):
        if row.get("Counter_Name") == counter:
            per[int(row["Dispatch_Id"])] = (_short_kernel(row["Kernel_Name"]), float(row["Counter_Value"]))
    return per


def counter_table(out_md, runs, command=""):
    """Counter-measured HBM traffic and rate of the hot-path kernels of several profiled
    step variants.  Each run is NAME=TRACE_DIR:FETCH_DIR:WRITE_DIR, three rocprofv3 runs
    of the same --profile-step command (kernel trace, FETCH_SIZE, WRITE_SIZE).  Counter
    KiB are scaled by what the same counters read for the plain device copy of COPY_BYTES
    that --calibrate-copy runs in that command."""
    want_kib = COPY_BYTES / 1024.0
    lines = ["# Counter-measured HBM traffic: fused vs unfused steps", "",
             f"Command: `{command}`", "",
             f"Peak: {HBM_PEAK_GBS:.0f} GB/s (MI355X HBM3E). Bytes per launch = FETCH_SIZE x scale_f + "
             "WRITE_SIZE x scale_w (KiB x 1024); the scales make a plain 1 GiB device copy read and write "
             "1 GiB. Rate = bytes per launch / average kernel-trace duration.", ""]
    for spec in runs:
        name, dirs = spec.split("=", 1)
        trace_dir, fetch_dir, write_dir = dirs.split(":")
        fetch, write = _pmc_per_key(fetch_dir, "FETCH_SIZE"), _pmc_per_key(write_dir, "WRITE_SIZE")
        cf, cw = calibration_dispatches(fetch), calibration_dispatches(write)
        if not cw or len(cf) != len(cw) or any(abs(write[i][1] - want_kib) >= 0.01 * want_kib for i in cw):
            raise SystemExit(f"{name}: no calibration copy found")
        sf = want_kib / (sum(fetch[i][1] for i in cf) / len(cf))
        sw = want_kib / (sum(write[i][1] for i in cw) / len(cw))
        byk = {}
        # a --profile-step command makes the same launches in its three runs, so its
        # dispatches pair up by number
        for i, (k, v) in fetch.items():
            if i in cf or i in cw or i not in write:
                continue
            b = (v * sf + write[i][1] * sw) * 1024.0
            byk.setdefault(k, []).append(b)
        stats = {_short_kernel(r["Name"]): r for r in _csv_rows(trace_dir, "kernel_stats.csv")}
        lines += [f"## {name}", "", f"Scales: FETCH x {sf:.4f}, WRITE x {sw:.4f}.", "",
                  "| kernel | role | calls | avg us | counter MB / launch | counter GB/s | % of peak |",
                  "|---|---|---|---|---|---|---|"]
        tot_b = tot_t = 0.0
        for k in sorted(byk, key=lambda k: -float(stats.get(k, {}).get("TotalDurationNs", 0))):
            role = _role(k)
            if role is None or k not in stats:
                continue
            calls = int(stats[k]["Calls"])
            avg_ns = float(stats[k]["AverageNs"])
            b = sum(byk[k]) / len(byk[k])
            gbs = b / avg_ns
            lines.append(f"| `{k}` | {role} | {calls} | {avg_ns / 1e3:.1f} | {b / 1e6:.1f} | {gbs:.0f} | "
                         f"{100 * gbs / HBM_PEAK_GBS:.1f} |")
            # the rounding of A and B happens once, before the steps; with a bf16 upstream
            # gradient the rounding of dC is part of every step (and A, B share the kernel)
            if role != ROUNDING or "dc_bf16" in name:
                tot_b += b * calls
                tot_t += avg_ns * calls
        if tot_t > 0:
            lines.append(f"| **all hot-path launches** | | | {tot_t / 1e3:.1f} (sum) | {tot_b / 1e6:.1f} (sum) | "
                         f"**{tot_b / tot_t:.0f}** | **{100 * tot_b / tot_t / HBM_PEAK_GBS:.1f}** |")
        lines.append("")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def timed_region(trace_dir):
    """Per-kernel launch count and average duration (us) of the dispatches between the first
    two marker launches of a kernel trace (the bench's timed steps, warm-up included), or
    None when the trace holds no such pair."""
    disp = _csv_rows(trace_dir, "kernel_trace.csv")
    if not disp:
        return None
    disp.sort(key=lambda r: int(r["Start_Timestamp"]))
    marks = [k for k, r in enumerate(disp) if MARKER_KERNEL in r["Kernel_Name"]][:2]
    if len(marks) < 2:
        return None
    out = {}
    for r in disp[marks[0] + 1:marks[1]]:
        k = _short_kernel(r["Kernel_Name"])
        out.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: (len(v), sum(v) / len(v)) for k, v in out.items()}


def trace_summary(trace_dir, out_md, command=""):
    rows = _csv_rows(trace_dir, "kernel_stats.csv")
    timed = timed_region(trace_dir)
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", ""]
    if timed:
        lines += ["Columns *timed calls* and *timed avg us*: the launches between the two marker launches that "
                  "bracket the bench's timed fused float32 steps (warm-up included). The other columns cover every "
                  "launch of the run, autotune candidates included.", ""]
    lines += ["| kernel | calls | avg us | min us | max us | total % |" + (" timed calls | timed avg us |" if timed else ""),
              "|---|---|---|---|---|---|" + ("---|---|" if timed else "")]
    for r in sorted(rows, key=lambda r: -float(r.get("TotalDurationNs", 0))):
        k = _short_kernel(r["Name"])
        extra = ""
        if timed:
            extra = f" {timed[k][0]} | {timed[k][1]:.1f} |" if k in timed else " | |"
        lines.append(f"| `{k}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |" + extra)
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def load_traffic(workload_name, kernel_key):
    """Counter-measured HBM bytes per launch of a kernel, if the committed counter summary
    for this workload was taken on the current kernel sources (else None)."""
    f = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash(source_globs(workload_name)):
        return None
    k = t["kernels"].get(kernel_key)
    sf, sw = t["scale"].get("FETCH_SIZE"), t["scale"].get("WRITE_SIZE")
    if not k or sf is None or sw is None:
        return None
    return (k["FETCH_SIZE"] * sf + k["WRITE_SIZE"] * sw) * 1024.0


# Instruction-issue counters, one rocprofv3 --pmc pass (8 SQ counters, the most one pass holds).
SQ_COUNTERS = ("SQ_INSTS_VALU", "SQ_BUSY_CU_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU_FMA_F32",
               "SQ_INSTS_VMEM_RD", "SQ_INSTS_FLAT", "SQ_INSTS_SALU", "SQ_WAVES")
SQ_FILE = "sq_issue.json"


def sq_summary(out_md, runs, command=""):
    """VALU issue use per hot-path kernel from one --pmc pass of SQ_COUNTERS per run
    (NAME=DIR).  A CU has 4 SIMDs of 16 lanes and a wave64 VALU instruction takes 4 cycles on
    one, so a CU issues at most one VALU wave-instruction per cycle: VALU issue use =
    SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES (both summed over the CUs).  Writes OUT_MD and, beside
    it, profiles' SQ_FILE with the same figures for the bench lines."""
    table = {}
    for spec in runs:
        name, d = spec.split("=", 1)
        per = {}
        for row in _csv_rows(d, "counter_collection.csv"):
            if row.get("Counter_Name") in SQ_COUNTERS:
                key = _short_kernel(row["Kernel_Name"])
                if _role(key) is None:
                    continue
                did = int(row["Dispatch_Id"])
                per.setdefault(key, {}).setdefault(did, {})
                per[key][did][row["Counter_Name"]] = per[key][did].get(row["Counter_Name"], 0.0) + \
                    float(row["Counter_Value"])
        kern = {}
        for key, ds in per.items():
            mean = {c: sum(v.get(c, 0.0) for v in ds.values()) / len(ds) for c in SQ_COUNTERS}
            busy = mean["SQ_BUSY_CU_CYCLES"]
            kern[key] = {"dispatches": len(ds), **{c: mean[c] for c in SQ_COUNTERS},
                         "valu_issue_frac": mean["SQ_INSTS_VALU"] / busy if busy > 0 else None,
                         "fma_share_of_valu": mean["SQ_INSTS_VALU_FMA_F32"] / mean["SQ_INSTS_VALU"]
                         if mean["SQ_INSTS_VALU"] > 0 else None}
        table[name] = {"source_hash": source_hash(source_globs(name)), "kernels": kern}
    lines = ["# VALU issue use of the hot-path kernels (SQ counters)", "", f"Command: `{command}`", "",
             "A CU has 4 SIMDs of 16 lanes; a wave64 VALU instruction occupies one SIMD for 4 cycles, so a CU "
             "issues at most one VALU wave-instruction per cycle. VALU issue use = SQ_INSTS_VALU / "
             "SQ_BUSY_CU_CYCLES (both summed over the CUs, per dispatch). FMA share = SQ_INSTS_VALU_FMA_F32 / "
             "SQ_INSTS_VALU: the part of the issued VALU work that is the method's own multiply-adds.", ""]
    for name, run in table.items():
        kern = run["kernels"]
        lines += [f"## {name}", "", "| kernel | role | dispatches | VALU wave-instr | VMEM rd | FLAT | SALU | "
                  "busy CU-cycles | VALU issue use | FMA share |", "|---|---|---|---|---|---|---|---|---|---|"]
        for key, k in sorted(kern.items(), key=lambda kv: -kv[1]["SQ_BUSY_CU_CYCLES"]):
            lines.append(f"| `{key}` | {_role(key)} | {k['dispatches']} | {k['SQ_INSTS_VALU']:.4g} | "
                         f"{k['SQ_INSTS_VMEM_RD']:.4g} | {k['SQ_INSTS_FLAT']:.4g} | {k['SQ_INSTS_SALU']:.4g} | "
                         f"{k['SQ_BUSY_CU_CYCLES']:.4g} | {k['valu_issue_frac']:.3f} | {k['fma_share_of_valu']:.3f} |")
        lines.append("")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    with open(os.path.join(os.path.dirname(os.path.abspath(out_md)), SQ_FILE), "w") as fh:
        json.dump({"command": command, "runs": table}, fh, indent=1)
    print("\n".join(lines))
    return table


def load_valu_issue(run, kernel_prefix):
    """VALU issue use of a kernel in a run of the committed SQ summary, while the sources of
    that run's kernels hash as they did when it was taken (else None)."""
    f = os.path.join(ROOT, "profiles", SQ_FILE)
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    entry = t.get("runs", {}).get(run)
    if not entry or entry.get("source_hash") != source_hash(source_globs(run)):
        return None
    k = next((v for kk, v in entry["kernels"].items() if kk.startswith(kernel_prefix)), None)
    v = None if k is None else k.get("valu_issue_frac")
    return None if v is None else round(v, 4)


MARKER_KERNEL = "stream_read_kernel"
# sources of the application passes (their counter data go stale when these change)
APP_SRC_GLOBS = {"gat_rmat20_r128_h4": SRC_GLOBS + ("paper_2203_07673_amd/csrc/gat*.hip",),
                 "als_er1m_d32_r128": SRC_GLOBS + ("paper_2203_07673_amd/csrc/als.hip",)}


def marker(dev):
    """A one-vector streaming read: a dispatch that marks region boundaries in a counter run
    (its kernel appears nowhere else in the application benches)."""
    import torch

    import paper_2203_07673_amd as F

    buf = torch.zeros(4, dtype=torch.float32, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    F.stream_read(buf, sink)
    torch.cuda.synchronize()


def marked_summary(fetch_dir, write_dir, out_json, regions, steps, workload_name, command=""):
    """Counter bytes per step of each marked region of a profiled run: the dispatches between
    consecutive marker dispatches (region i lies between markers i and i + 1), FETCH and
    WRITE scaled by the plain copies of --calibrate-copy, summed, divided by `steps`."""
    per = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        rows = _csv_rows(d, "counter_collection.csv")
        per[counter] = {int(r["Dispatch_Id"]): (r["Kernel_Name"], float(r["Counter_Value"]))
                        for r in rows if r.get("Counter_Name") == counter}
    want_kib = COPY_BYTES / 1024.0
    out = {"command": command, "source_hash": source_hash(APP_SRC_GLOBS[workload_name]), "steps": steps,
           "regions": {}, "scale": {}}
    for counter, d in per.items():
        calib = calibration_dispatches(d)
        if not calib:
            raise SystemExit(f"{counter}: no calibration copy found")
        out["scale"][counter] = want_kib / (sum(d[i][1] for i in calib) / len(calib))
        marks = sorted(i for i, (k, _) in d.items() if MARKER_KERNEL in k)
        if len(marks) != len(regions) + 1:
            raise SystemExit(f"{counter}: {len(marks)} markers for {len(regions)} regions")
        for name, a, b in zip(regions, marks, marks[1:]):
            kib = sum(v for i, (k, v) in d.items() if a < i < b)
            reg = out["regions"].setdefault(name, {"dispatches": sum(1 for i in d if a < i < b)})
            reg[counter + "_KiB_per_step"] = kib / steps
    for reg in out["regions"].values():
        reg["bytes_per_step"] = int(1024.0 * (reg["FETCH_SIZE_KiB_per_step"] * out["scale"]["FETCH_SIZE"] +
                                              reg["WRITE_SIZE_KiB_per_step"] * out["scale"]["WRITE_SIZE"]))
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def region_traffic(workload_name, region):
    """Counter bytes per step of a region from profiles/traffic_<workload>.json, if it was
    taken on the current sources (else None)."""
    f = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash(APP_SRC_GLOBS[workload_name]):
        return None
    reg = t.get("regions", {}).get(region)
    return None if reg is None else reg["bytes_per_step"]


def run_batch(args):
    """Batched workload: 256 ER graphs (n log-uniform in [1024, 65536], degree uniform in
    [8, 64]), r = 64, bfloat16 storage, fused forward + adjoint of every graph in one
    persistent launch replayed from a hipGraph after autotuning."""
    import torch

    import paper_2203_07673_amd as F
    from workloads import batch_er

    t0 = time.perf_counter()
    r = 64
    graphs = batch_er(256, r, seed=5)
    nnz = sum(g["S"].nnz for g in graphs)
    rows = sum(g["S"].m for g in graphs)
    log(f"generated 256 graphs: rows={rows} nnz={nnz} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pats = [F.Pattern.from_csr(g["S"], device=dev) for g in graphs]
    A32 = [torch.from_numpy(g["A"]).to(dev) for g in graphs]
    B32 = [torch.from_numpy(g["B"]).to(dev) for g in graphs]
    G = [torch.from_numpy(g["G"]).to(dev) for g in graphs]
    A = [F.to_bf16(a) for a in A32]
    B = [F.to_bf16(b) for b in B32]
    plan = F.BatchPlan(pats, A, B, G)
    if args.tuned:  # TILE_NNZ:XCD_AWARE:ROW_WAVE:COL_WAVE, as a bench run's autotune chose it
        tile, xcd, roww, colw = (int(x) for x in args.tuned.split(":"))
        plan.set_schedule(tile, xcd, bool(roww), bool(colw))
        info = plan.info()
        log(f"schedule from --tuned: {info}")
    else:
        info = plan.autotune()
        log(f"autotuned: {info}")
    tuned_arg = f"{info['tile_nnz']}:{info['xcd_aware']}:{info['row_schedule']}:{info['col_schedule']}"
    side = torch.cuda.Stream()
    plan.capture(side)
    with torch.cuda.stream(side):
        for _ in range(args.warmup):
            plan.launch(side)
        side.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(side)
        for _ in range(args.steps):
            plan.launch(side)
        e1.record(side)
        side.synchronize()
        t_step = (time.perf_counter() - t0) / args.steps
        k_ms = e0.elapsed_time(e1) / args.steps
    flops = 12.0 * r * nnz
    gflops = flops / t_step / 1e9
    log(f"batched fwd+bwd {t_step * 1e3:.3f} ms ({k_ms:.3f} ms by events) -> {gflops:.1f} GFLOP/s")

    e = 2
    bytes_launch = 0   # gather model, summed over the three passes of every graph
    bytes_min = 0      # compulsory: every array of every graph once per launch
    for g in graphs:
        S = g["S"]
        for kind in ("fwd", "bwd_row", "bwd_col"):
            bytes_launch += kernel_bytes(kind, S.m, S.n, S.nnz, r, e)
        bytes_min += batch_graph_bytes_min(S.m, S.n, S.nnz, r, e, 4)
    achieved = bytes_min / (k_ms * 1e-3) / 1e9
    # counter-measured bytes per launch of the chosen schedule's kernel, when the committed
    # counter summary covers the current sources
    waves = 64 // info["lanes"]  # line groups sharing a wavefront in the wavefront-per-line schedule
    kname = "batch_queue_kernel" if info["xcd_aware"] == 2 else "batch_kernel"
    kernel_key = (f"void fmm::{kname}<unsigned short, float, {info['lanes']}, 8, "
                  f"{waves if info['row_schedule'] else 1}, {waves if info['col_schedule'] else 1}>")
    traffic = None
    f = os.path.join(ROOT, "profiles", "traffic_batch256_r64.json")
    if os.path.exists(f):
        with open(f) as fh:
            t = json.load(fh)
        k = next((v for kk, v in t["kernels"].items() if kk.startswith(kernel_key)), None)
        if (t.get("source_hash") == source_hash(BATCH_SRC_GLOBS) and k and t["scale"]["FETCH_SIZE"]
                and t.get("tuned_arg") == tuned_arg):
            traffic = (k["FETCH_SIZE"] * t["scale"]["FETCH_SIZE"] + k["WRITE_SIZE"] * t["scale"]["WRITE_SIZE"]) * 1024.0

    variants = {"autotune": info}
    if not args.no_variants:
        def loop(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps

        C = [torch.empty(P.m, r, dtype=torch.float32, device=dev) for P in pats]

        def unbatched(Al, Bl, fused):
            for P, a, b, g, c in zip(pats, Al, Bl, G, C):
                _, R = F.fusedmm_a_raw(P, a, b, out=c, fused=fused)
                F.fusedmm_a_backward_raw(P, a, b, g, fused=fused, R_ws=R)
        t_ub = loop(lambda: unbatched(A, B, True))
        t_uf = loop(lambda: unbatched(A32, B32, False))
        variants["per_graph_calls_fused_bf16_ms"] = round(t_ub * 1e3, 3)
        variants["per_graph_calls_unfused_f32_ms"] = round(t_uf * 1e3, 3)
        variants["speedup_batched_bf16_vs_per_graph_unfused_f32"] = round(t_uf / t_step, 3)
        plan.run(side)
        side.synchronize()
        t_eager = loop(lambda: plan.run(side))
        variants["eager_persistent_launch_ms"] = round(t_eager * 1e3, 3)
        # the same batch with bfloat16 upstream gradients (already bfloat16 in HBM, as from a
        # bfloat16 layer above): its own autotune and hipGraph
        G16 = [F.to_bf16(g) for g in G]
        plan16 = F.BatchPlan(pats, A, B, G16)
        plan16.autotune()
        plan16.capture(side)
        with torch.cuda.stream(side):
            for _ in range(2):
                plan16.launch(side)
            side.synchronize()
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record(side)
            for _ in range(args.steps):
                plan16.launch(side)
            f1.record(side)
            side.synchronize()
        variants["batched_bf16_dc_bf16_ms"] = round(f0.elapsed_time(f1) / args.steps, 4)
        variants["batched_bf16_dc_bf16_schedule"] = plan16.info()
        del plan16, G16

    out = {
        "metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "batch256_r64", "graphs": 256, "rows": rows, "nnz": nnz, "r": r, "storage": "bf16",
                   "step": "hipGraph replay of one persistent launch: fused forward + adjoint of every graph",
                   "flops_per_step": flops, "tuning_arg": tuned_arg},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else int(traffic),
                     "traffic_gbs": None if traffic is None else round(traffic / (k_ms * 1e-3) / 1e9, 1),
                     "frac_counters": None if traffic is None else
                     round(traffic / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic_over_compulsory": None if traffic is None else round(traffic / bytes_min, 3),
                     "kernel": f"{kname} (persistent, all passes): {kernel_key}", "kernel_ms": round(k_ms, 4),
                     "bytes_per_launch": int(bytes_min),
                     "bytes_model": "compulsory: every array of every graph once per launch (rows gathered "
                                    "again hit in L2, so the gather model is no bound here)",
                     "bytes_gather_model": int(bytes_launch),
                     "frac_gather_model": round(bytes_launch / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     # share of the CUs' VALU issue slots the kernel used (committed SQ counters)
                     "valu_issue_frac": load_valu_issue("batch256_r64", kernel_key)},
        "variants": variants,
    }
    if not args.no_variants:
        # random-gather ceilings at the batch's row size (64 bf16 = 128 B): the queue kernel's
        # L2 misses are gathers of such rows, mostly of the graphs the XCDs are working on
        gc = gather_ceiling(dev, 2 * r)
        out["roofline"]["gather_ceiling"] = gc
        if traffic is not None:
            out["roofline"]["frac_counters_of_gather_ceiling"] = round(
                traffic / (k_ms * 1e-3) / 1e9 / gc["mall_resident_gbs"], 4)
        log(f"gather ceilings ({gc['row_bytes']} B rows): HBM random {gc['hbm_random_gbs']:.0f} GB/s, "
            f"MALL-resident {gc['mall_resident_gbs']:.0f} GB/s, L2-resident {gc['l2_resident_gbs']:.0f} GB/s")
    if args.calibrate_copy:
        calibrate_copy(dev)
    print(json.dumps(out), flush=True)


def run_gat(args):
    """Graph-attention head (Section VI-E): 4 heads of r = 128 on the R-MAT scale 20
    graph, softmax-normalised; fused one-pass forward vs the unfused sequence (edge values
    written to memory, then an SpMM), and the adjoint of every head."""
    import torch

    import paper_2203_07673_amd as F
    from workloads import dense_normal, workload

    w = workload("rmat20_ef16_r64")
    S = w["S"]
    r, heads = 128, 4
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = F.Pattern.from_csr(S, device=dev)
    Hs = [torch.from_numpy(dense_normal(S.n, r, 500 + h)).to(dev) for h in range(heads)]
    a = [(torch.from_numpy(dense_normal(1, r, 600 + h, sigma=r ** -0.5)[0]).to(dev),
          torch.from_numpy(dense_normal(1, r, 700 + h, sigma=r ** -0.5)[0]).to(dev)) for h in range(heads)]
    outs = [torch.empty(S.m, r, device=dev) for _ in range(heads)]
    dOs = [torch.from_numpy(dense_normal(S.m, r, 800 + h)).to(dev) for h in range(heads)]
    tuning = F.gat_autotune(P, Hs[0], a[0][0], a[0][1], dO=dOs[0], softmax=True)
    log(f"attention autotuned: {tuning}")

    def step(Hl):
        for h in range(heads):
            F.gat_forward(P, Hl[h], a[h][0], a[h][1], softmax=True, out=outs[h])

    if args.profile_step:  # marked regions for a counter run: fp32 forward steps, then adjoint steps
        lses_p = [torch.empty(S.m, device=dev) for _ in range(heads)]
        for h in range(heads):
            F.gat_forward(P, Hs[h], a[h][0], a[h][1], softmax=True, out=outs[h], lse=lses_p[h])
        marker(dev)
        for _ in range(args.steps):
            step(Hs)
        marker(dev)
        for _ in range(args.steps):
            for h in range(heads):
                F.gat_backward(P, Hs[h], a[h][0], a[h][1], outs[h], dOs[h], softmax=True, lse=lses_p[h])
        marker(dev)
        calibrate_copy(dev)
        print(json.dumps({"profile_step": "regions fwd_f32, bwd_f32", "steps": args.steps, "tuning": tuning}))
        return

    def timeit(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t32 = timeit(lambda: step(Hs), args.steps, args.warmup)
    H16 = [F.to_bf16(x) for x in Hs]
    t16 = timeit(lambda: step(H16), args.steps, args.warmup)

    def step_unfused(Hl):
        for h in range(heads):
            F.gat_forward_unfused(P, Hl[h], a[h][0], a[h][1], softmax=True, out=outs[h])

    tu = timeit(lambda: step_unfused(Hs), args.steps, args.warmup)

    # adjoint of every head (dH, da1, da2) from the forward outputs and an upstream gradient

    lses = [torch.empty(S.m, device=dev) for _ in range(heads)]

    def fwd_lse(Hl):
        for h in range(heads):
            F.gat_forward(P, Hl[h], a[h][0], a[h][1], softmax=True, out=outs[h], lse=lses[h])

    def step_bwd(Hl):
        for h in range(heads):
            F.gat_backward(P, Hl[h], a[h][0], a[h][1], outs[h], dOs[h], softmax=True, lse=lses[h])
    fwd_lse(Hs)
    tb32 = timeit(lambda: step_bwd(Hs), args.steps, args.warmup)
    fwd_lse(H16)
    tb16 = timeit(lambda: step_bwd(H16), args.steps, args.warmup)

    def step_bwd_do16(Hl):  # bf16 features and a bf16 upstream gradient, rounded in the step
        for h in range(heads):
            F.gat_backward(P, Hl[h], a[h][0], a[h][1], outs[h], F.to_bf16(dOs[h]), softmax=True, lse=lses[h])
    tb16g = timeit(lambda: step_bwd_do16(H16), args.steps, args.warmup)
    nnz, n = S.nnz, S.n
    bytes32 = heads * gat_forward_bytes(n, nnz, r, 4)
    bbytes32 = heads * gat_backward_bytes(n, nnz, r, 4)

    def roofline(nbytes, t, what, region):
        achieved = nbytes / t / 1e9
        traffic = region_traffic("gat_rmat20_r128_h4", region)
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": what,
                "frac_counters": None if traffic is None else round(traffic / t / 1e9 / HBM_PEAK_GBS, 4),
                "bytes_per_step": int(nbytes), "bytes_model": "gather (each stored entry fetches its rows)"}
    out = {"metric": "graph-attention forward (4 heads, softmax) ms", "workload": "gat_rmat20_r128_h4",
           "nnz": nnz, "n": n, "r": r, "heads": heads,
           "fused_f32_ms": round(t32 * 1e3, 4), "fused_bf16_ms": round(t16 * 1e3, 4),
           "unfused_f32_ms": round(tu * 1e3, 4), "speedup_fused_f32_vs_unfused_f32": round(tu / t32, 3),
           "backward_f32_ms": round(tb32 * 1e3, 4), "backward_bf16_ms": round(tb16 * 1e3, 4),
           "backward_bf16_dO_bf16_ms": round(tb16g * 1e3, 4),
           "train_step_f32_ms": round((t32 + tb32) * 1e3, 4),
           "roofline": roofline(bytes32, t32, "fused forward of every head, fp32 (scores, line pass, merges)",
                                "fwd_f32"),
           "roofline_backward": roofline(bbytes32, tb32, "adjoint of every head, fp32 (row, column, da passes)",
                                         "bwd_f32"),
           "tuning": tuning}
    print(json.dumps(out), flush=True)


def run_als(args):
    """ALS application (Section VI-E): one sweep = 10 batched CG steps for A, then 10 for
    B (the paper's 20 CG iterations), each step's query vectors from one FusedMM-shaped
    pass; observations are a noisy rank-128 product on an ER pattern (2^20 x 2^20, 32 per
    row)."""
    import torch

    import paper_2203_07673_amd as F
    from workloads import CsrPattern, dense_normal, er_exact_degree

    m = n = 1 << 20
    d, r = 32, 128
    S = er_exact_degree(m, n, d, seed=21)
    At = dense_normal(m, r, 22, sigma=r ** -0.5)
    Bt = dense_normal(n, r, 23, sigma=r ** -0.5)
    rows = np.repeat(np.arange(m), d)
    obs = np.empty(S.nnz, np.float32)
    for b0 in range(0, S.nnz, 1 << 22):
        b1 = min(S.nnz, b0 + (1 << 22))
        obs[b0:b1] = np.einsum("ij,ij->i", At[rows[b0:b1]], Bt[S.colidx[b0:b1]])
    obs += np.float32(0.01) * np.random.default_rng(24).standard_normal(S.nnz, dtype=np.float32)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = F.Pattern.from_csr(CsrPattern(m, n, S.rowptr, S.colidx, obs), device=dev)
    A = torch.from_numpy(dense_normal(m, r, 25, sigma=0.1)).to(dev)
    B = torch.from_numpy(dense_normal(n, r, 26, sigma=0.1)).to(dev)
    loss0 = float(F.als_residual(P, A, B))
    F.als_sweep(P, A, B, 1e-3, 10)  # warm-up sweep
    torch.cuda.synchronize()
    if args.profile_step:  # one marked region of sweeps for a counter run
        marker(dev)
        for _ in range(args.steps):
            F.als_sweep(P, A, B, 1e-3, 10)
        marker(dev)
        calibrate_copy(dev)
        print(json.dumps({"profile_step": "region sweep", "steps": args.steps}))
        return
    sweeps = max(1, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(sweeps):
        F.als_sweep(P, A, B, 1e-3, 10)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / sweeps
    loss = float(F.als_residual(P, A, B))
    # per sweep: 2 x 11 Gram passes (4 r nnz flops each) + 2 right-hand-side SpMMs (2 r nnz)
    flops = 2 * (11 * 4 * r * S.nnz + 2 * r * S.nnz)
    nbytes = als_sweep_bytes(m, n, S.nnz, r)
    achieved = nbytes / t / 1e9
    traffic = region_traffic("als_er1m_d32_r128", "sweep")
    out = {"metric": "ALS sweep (20 batched CG iterations) ms", "workload": "als_er1m_d32_r128",
           "nnz": S.nnz, "r": r, "ms_per_sweep": round(t * 1e3, 3), "gflops": round(flops / t / 1e9, 1),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "frac_counters": None if traffic is None else round(traffic / t / 1e9 / HBM_PEAK_GBS, 4),
                        "kernel": "whole sweep (right-hand sides, Gram passes, fused CG passes)",
                        "bytes_per_sweep": int(nbytes), "bytes_model": "gather (each stored entry fetches F_j)"},
           "loss_start": loss0, "loss_after": loss, "sweeps_timed": sweeps}
    print(json.dumps(out), flush=True)


def restore_tuning(P, tuning):
    """Put back an autotuned configuration (P.tuning)."""
    P.apply_tuning(tuning)


def tuning_arg(tuning):
    """--tuned form of P.tuning: csr=VARIANT:LONG_LEN:ORDER:HINTS,csc=... (LONG_LEN 0 = no split,
    HINTS = hot minor lines of the gather hints, 0 = none)."""
    return ",".join(f"{k}={t['variant']}:{t['long_len'] or 0}:{int(t['line_order'])}:{t.get('gather_hints') or 0}"
                    for k, t in tuning.items())


def parse_tuning_arg(arg):
    """Inverse of tuning_arg (a missing HINTS field means none)."""
    tuning = {}
    for part in arg.split(","):
        k, v = part.split("=")
        f = [int(x) for x in v.split(":")]
        tuning[k] = {"variant": f[0], "long_len": f[1] or None, "line_order": bool(f[2]),
                     "gather_hints": (f[3] if len(f) > 3 else 0) or None}
    return tuning


def calibrate_copy(dev):
    """Three plain device copies of COPY_BYTES: the reference dispatches for scaling counters."""
    import torch

    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


PROBE_BYTES = 4 << 30  # long enough for the streaming probes to reach their full rate


def median_event_ms(fn, reps):
    """Median over `reps` calls of fn (after two untimed ones) of its HIP-event time on the
    current stream."""
    import torch

    for _ in range(2):
        fn()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


# working sets of the gather ceilings: the whole probe buffer (rows come from HBM), 192 MiB
# (held by the 256 MB MALL but by no L2) and 2 MiB (held by every XCD's 4 MB L2)
GATHER_SETS = (("hbm_random", PROBE_BYTES), ("mall_resident", 192 << 20), ("l2_resident", 2 << 20))


def gather_ceiling(dev, row_bytes, reps=5):
    """Measured ceilings of random row gathers with the library's gather probe (one 16-byte
    load per lane, as the line kernels gather rows): PROBE_BYTES worth of rows of row_bytes
    bytes per launch, drawn uniformly (seeded) from each working set of GATHER_SETS.  Rate =
    rows x (row bytes + 4 index bytes) / median event time."""
    import torch

    import paper_2203_07673_amd as F
    from paper_2203_07673_amd import _capi as CA

    src = torch.empty(PROBE_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(13)
    n = PROBE_BYTES // row_bytes
    out = {"row_bytes": row_bytes, "rows_per_launch": n, "kernel": "fmm_stream_gather (gather_rows_kernel)"}
    for name, ws in GATHER_SETS:
        rows = torch.randint(0, ws // row_bytes, (n,), generator=gen, device=dev, dtype=torch.int32)
        F.stream_gather(src, row_bytes, rows, sink)  # checks every index once; the timed calls go straight in
        stream = torch.cuda.current_stream().cuda_stream
        t = median_event_ms(lambda: CA.call("fmm_stream_gather", src.data_ptr(), row_bytes, rows.data_ptr(), n,
                                            0x9E3779B9, sink.data_ptr(), stream), reps)
        out[f"{name}_gbs"] = round(n * (row_bytes + 4) / (t * 1e-3) / 1e9, 1)
        del rows
    return out


def copy_ceiling(dev, reps=10):
    """Measured HBM ceilings on contiguous traffic: the library's read-only pass over
    PROBE_BYTES and its plain copy of PROBE_BYTES / 2 (read + write, PROBE_BYTES moved),
    both on the current stream; torch's device-to-device copy of the same for comparison."""
    import torch

    import paper_2203_07673_amd as F

    src = torch.empty(PROBE_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    half = src[:PROBE_BYTES // 8]
    dst = torch.empty_like(half)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    median_ms = lambda fn: median_event_ms(fn, reps)  # noqa: E731

    t_copy = median_ms(lambda: F.stream_copy(half, dst))
    t_read = median_ms(lambda: F.stream_read(src, sink))
    t_torch = median_ms(lambda: dst.copy_(half))
    gbs = lambda nbytes, t: round(nbytes / (t * 1e-3) / 1e9, 1)  # noqa: E731
    return {"gbs": gbs(PROBE_BYTES, t_copy), "read_gbs": gbs(PROBE_BYTES, t_read),
            "torch_copy_gbs": gbs(PROBE_BYTES, t_torch), "bytes_moved": PROBE_BYTES,
            "kernels": "fmm_stream_copy (read + write), fmm_stream_read (read only), torch copy_"}


GATHER_ROW_BYTES = (128, 256, 512, 1024)


def calibrate_gather(dev, reps=3):
    """Gather probes of known size for counter calibration: each row of a PROBE_BYTES buffer
    read once, in a seeded random order, at each of GATHER_ROW_BYTES per row (the row sizes
    of the workloads' gathered rows: 64 bf16 or 32 fp32 elements up to 256 fp32), `reps`
    times each; then the plain copies of --calibrate-copy."""
    import torch

    import paper_2203_07673_amd as F

    src = torch.empty(PROBE_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    for rb in GATHER_ROW_BYTES:
        rows = torch.randperm(PROBE_BYTES // rb, generator=gen, device=dev, dtype=torch.int32)
        for _ in range(reps):
            F.stream_gather(src, rb, rows, sink)
        torch.cuda.synchronize()
        del rows
    calibrate_copy(dev)


def gather_summary(fetch_dir, out_md, command=""):
    """FETCH_SIZE of the gather probes against the bytes they move (every row once plus its
    4-byte index), next to the plain copy's scale: the factor each access shape needs."""
    per = {}
    for row in _csv_rows(fetch_dir, "counter_collection.csv"):
        if row.get("Counter_Name") == "FETCH_SIZE":
            per[int(row["Dispatch_Id"])] = (row["Kernel_Name"], float(row["Counter_Value"]))
    lines = ["# FETCH_SIZE scale on gather-shaped traffic", "", f"Command: `{command}`", "",
             f"Each probe reads every row of a {PROBE_BYTES >> 30} GiB buffer once, in a seeded random order "
             "(default cache policy, one 16-byte load per lane, as the line kernels gather rows). Known bytes = "
             "rows x (row bytes + 4 index bytes). Scale = known bytes / (FETCH_SIZE KiB x 1024).", "",
             "| probe | dispatches | FETCH_SIZE (KiB, mean) | known bytes | scale |", "|---|---|---|---|---|"]
    out = {}
    for rb in GATHER_ROW_BYTES:
        tag = f"gather_rows_kernel<{rb // 16}>"
        vals = [v for k, v in per.values() if tag in k.replace(" ", "")]
        if not vals:
            continue
        n = PROBE_BYTES // rb
        known = n * (rb + 4)
        kib = sum(vals) / len(vals)
        out[rb] = known / (kib * 1024.0)
        lines.append(f"| gather, {rb} B rows | {len(vals)} | {kib:.0f} | {known} | {out[rb]:.3f} |")
    calib = calibration_dispatches(per)
    if calib:
        kib = sum(per[i][1] for i in calib) / len(calib)
        lines.append(f"| plain device copy of {COPY_BYTES >> 30} GiB (reads) | {len(calib)} | {kib:.0f} | "
                     f"{COPY_BYTES} | {COPY_BYTES / (kib * 1024.0):.3f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return out


def cold_cache_steps(step, reps, kinds, dev):
    """The step timed with L2 and MALL flushed before each repetition (a 1 GiB scratch
    buffer is overwritten between steps, outside the timed events)."""
    import torch

    scratch = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    per_step, per_kernel = [], {k: [] for k in kinds}
    for i in range(reps):
        scratch.fill_(float(i))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        step(ev)
        torch.cuda.synchronize()
        per_step.append(ev[0].elapsed_time(ev[3]))
        for j, k in enumerate(kinds):
            per_kernel[k].append(ev[j].elapsed_time(ev[j + 1]))
    return {"median_ms": round(float(np.median(per_step)), 4), "reps": reps, "flush_bytes": COPY_BYTES,
            "kernel_ms": {k: round(float(np.median(v)), 4) for k, v in per_kernel.items()}}


def profile_step(args, F, P, A, B, make_step, time_steps, flops, nnz):
    """One step variant alone, for kernel traces and counter runs of that variant."""
    import torch

    dev = A.device
    if args.tuned:
        restore_tuning(P, parse_tuning_arg(args.tuned))
    if args.profile_step == "fused_f32":
        step = make_step(A, B, fused=True)
    elif args.profile_step == "unfused_f32":
        R_ws = torch.empty(nnz, dtype=torch.float32, device=dev)
        dP_ws = torch.empty(nnz, dtype=torch.float32, device=dev)
        step = make_step(A, B, fused=False, R_ws=R_ws, dP_ws=dP_ws)
    else:
        step = make_step(F.to_bf16(A), F.to_bf16(B), fused=True, dc_bf16=args.profile_step == "fused_bf16_dc_bf16")
    t, kt = time_steps(step, args.steps, args.warmup)
    if args.calibrate_copy:
        calibrate_copy(dev)
    print(json.dumps({"profile_step": args.profile_step, "workload": args.workload, "tuning": P.tuning,
                      "ms_per_step": round(t * 1e3, 4),
                      "gflops": round(flops / t / 1e9, 1), "kernel_ms": {k: round(v, 4) for k, v in kt.items()}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rmat22_ef16_r256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for counter scaling)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "OUT_MD"),
                    help="summarise a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--counter-table", nargs="+", metavar="OUT_MD NAME=TRACE:FETCH:WRITE",
                    help="markdown table of counter-measured traffic per hot-path kernel and step variant")
    ap.add_argument("--marked-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON", "REGIONS"),
                    help="counter bytes per step of the marked regions (comma-separated names) of a --profile-step "
                         "regions run of the attention or ALS workload, and exit")
    ap.add_argument("--profile-step", choices=("fused_f32", "unfused_f32", "fused_bf16", "fused_bf16_dc_bf16",
                                               "regions"),
                    help="run only this step variant, for profiling (no autotune: the batch depth and split "
                         "threshold come from --tuned, else the defaults)")
    ap.add_argument("--tuned", default="",
                    help="csr=VARIANT:LONG_LEN:ORDER:HINTS,csc=... as a bench run's autotune chose "
                         "them (config.tuning_arg; LONG_LEN 0 = no split schedule, ORDER 0/1, HINTS 0 = no gather "
                         "hints); for batch256_r64 TILE_NNZ:XCD_AWARE:ROW_WAVE:COL_WAVE")
    ap.add_argument("--calibrate-gather", action="store_true",
                    help="run only the gather probes of known size and the plain copies (for a --pmc run)")
    ap.add_argument("--gather-summary", nargs=2, metavar=("FETCH_DIR", "OUT_MD"),
                    help="summarise a FETCH_SIZE run of --calibrate-gather and exit")
    ap.add_argument("--sq-summary", nargs="+", metavar="OUT_MD NAME=DIR",
                    help="VALU issue use per hot-path kernel from --pmc runs of SQ_COUNTERS, and exit")
    ap.add_argument("--command", default="", help="command line recorded in summaries")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, command=args.command, tuned=args.tuned)
        return
    if args.trace_summary:
        trace_summary(*args.trace_summary, command=args.command)
        return
    if args.counter_table:
        counter_table(args.counter_table[0], args.counter_table[1:], command=args.command)
        return
    if args.sq_summary:
        sq_summary(args.sq_summary[0], args.sq_summary[1:], command=args.command)
        return
    if args.gather_summary:
        gather_summary(*args.gather_summary, command=args.command)
        return
    if args.marked_summary:
        fd, wd, oj, regs = args.marked_summary
        wname = os.path.basename(oj)[len("traffic_"):].rsplit(".", 1)[0]
        marked_summary(fd, wd, oj, regs.split(","), args.steps, wname, command=args.command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_gather:
        import torch

        torch.cuda.set_device(0)
        calibrate_gather(torch.device("cuda:0"))
        return
    if args.workload == "batch256_r64":
        run_batch(args)
        return
    if args.workload == "gat_rmat20_r128_h4":
        run_gat(args)
        return
    if args.workload == "als_er1m_d32_r128":
        run_als(args)
        return

    import torch

    import paper_2203_07673_amd as F
    from workloads import workload

    t_gen = time.perf_counter()
    w = workload(args.workload)
    S, r = w["S"], w["r"]
    m, n, nnz = S.m, S.n, S.nnz
    log(f"generated {args.workload}: m={m} n={n} nnz={nnz} r={r} in {time.perf_counter() - t_gen:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # every launch and timing event of the bench goes to one dedicated stream
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    t_prep = time.perf_counter()
    P = F.Pattern.from_csr(S, device=dev)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t_prep
    log(f"pattern prep (validate + transpose + schedule) {prep_s:.2f}s; "
        f"schedules csr={P.schedules['csr'] is not None} csc={P.schedules['csc'] is not None}")
    A = torch.from_numpy(w["A"]).to(dev)
    B = torch.from_numpy(w["B"]).to(dev)
    G = torch.from_numpy(w["G"]).to(dev)
    C = torch.empty(m, r, dtype=torch.float32, device=dev)
    dA = torch.empty(m, r, dtype=torch.float32, device=dev)
    dB = torch.empty(n, r, dtype=torch.float32, device=dev)

    kinds = ("fwd", "bwd_row", "bwd_col")

    def make_step(Ai, Bi, fused=True, R_ws=None, dP_ws=None, dc_bf16=False):
        # dc_bf16: the upstream gradient is rounded to bfloat16 in the step (timed with the
        # row pass) and both adjoint passes read it as stored
        def step(ev=None):
            if ev is not None:
                ev[0].record()
            F.fusedmm_a_raw(P, Ai, Bi, out=C, fused=fused, R_ws=R_ws)
            if ev is not None:
                ev[1].record()
            Gs = F.to_bf16(G) if dc_bf16 else G
            F.fusedmm_a_backward_raw(P, Ai, Bi, Gs, dA=dA, need=(True, False), fused=fused, R_ws=R_ws, dP_ws=dP_ws)
            if ev is not None:
                ev[2].record()
            F.fusedmm_a_backward_raw(P, Ai, Bi, Gs, dB=dB, need=(False, True), fused=fused, R_ws=R_ws, dP_ws=dP_ws)
            if ev is not None:
                ev[3].record()
        return step

    def time_steps(step, steps, warmup, per_kernel=True, step_ms=None):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)] if per_kernel else None
        t0 = time.perf_counter()
        for s in range(steps):
            step(evs[s] if per_kernel else None)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        ktimes = None
        if per_kernel:
            ktimes = {k: float(np.mean([evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(steps)]))
                      for i, k in enumerate(kinds)}
            if step_ms is not None:
                step_ms.extend(evs[s][0].elapsed_time(evs[s][3]) for s in range(steps))
        return t, ktimes

    flops = 12.0 * r * nnz
    if args.profile_step:
        if args.profile_step == "regions":
            raise SystemExit("--profile-step regions is for the attention and ALS workloads")
        profile_step(args, F, P, A, B, make_step, time_steps, flops, nnz)
        return
    P.autotune(A, B, G, form="a")
    tuning = P.tuning
    log(f"autotuned (f32): {tuning}")
    step_f32 = make_step(A, B, fused=True)
    log(f"timing fused f32: warmup {args.warmup}, steps {args.steps}")
    step_ms = []
    marker(dev)  # brackets the timed steps' dispatches in a kernel trace (outside the timed region)
    t_step, kt = time_steps(step_f32, args.steps, args.warmup, step_ms=step_ms)
    marker(dev)
    gflops = flops / t_step / 1e9
    # sampled outputs of the last timed step of each variant, for the error report
    colptr_h = np.concatenate([[0], np.cumsum(np.bincount(S.colidx, minlength=n))])
    rows_s, cols_s = sample_lines(S.rowptr, 1024, 7), sample_lines(colptr_h, 1024, 8)
    rows_d, cols_d = torch.from_numpy(rows_s).to(dev), torch.from_numpy(cols_s).to(dev)
    outputs = {}

    def keep(name):
        torch.cuda.synchronize()
        outputs[name] = tuple(x.index_select(0, i).double().cpu().numpy()
                              for x, i in ((C, rows_d), (dA, rows_d), (dB, cols_d)))
    keep("fused_f32")
    log(f"fused f32 step {t_step * 1e3:.3f} ms -> {gflops:.1f} GFLOP/s; kernels (ms) {kt}")

    e = 4
    dom = max(kinds, key=lambda k: kt[k])
    dom_bytes = kernel_bytes(dom, m, n, nnz, r, e)
    achieved = dom_bytes / (kt[dom] * 1e-3) / 1e9
    step_bytes = sum(kernel_bytes(k, m, n, nnz, r, e) for k in kinds)
    # exact instantiation of the dominant kernel, to look up its counter data
    from paper_2203_07673_amd import _capi as CA
    orient = CA.FMM_CSC if dom == "bwd_col" else CA.FMM_CSR
    L, NV, VW, U = P.launch_shape(orient, dom == "bwd_col", r, CA.FMM_F32)
    op = 4 if dom == "bwd_col" else 3
    kernel_key = f"line_kernel<{op}, float, float, float, float, {L}, {NV}, {VW}, {U}>"
    traffic = load_traffic(args.workload, kernel_key)

    def pass_key(kind):
        o = CA.FMM_CSC if kind == "bwd_col" else CA.FMM_CSR
        Lk, NVk, VWk, Uk = P.launch_shape(o, kind == "bwd_col", r, CA.FMM_F32)
        return f"line_kernel<{4 if kind == 'bwd_col' else 3}, float, float, float, float, {Lk}, {NVk}, {VWk}, {Uk}>"
    # counter-measured bytes of the whole step (the three passes' instantiations), when
    # the committed counter summary covers them
    pass_traffic = [load_traffic(args.workload, pass_key(k)) for k in kinds]
    step_traffic = None if any(x is None for x in pass_traffic) else sum(pass_traffic)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "kernel": {"fwd": "FusedMMA forward", "bwd_row": "adjoint row pass dA",
                           "bwd_col": "adjoint column pass dB"}[dom] + f" ({kernel_key})",
                "kernel_ms": round(kt[dom], 4), "bytes_per_launch": int(dom_bytes),
                "bytes_model": "gather (each stored entry fetches its dense row(s))",
                "frac_gather_model": round(achieved / HBM_PEAK_GBS, 4),
                "frac_note": "frac counts every gathered row as moved (the gather model); rows served from L2 or "
                             "the MALL let it pass 1, as on R-MAT, where hub rows are gathered many times. "
                             "frac_counters uses the counted L2-to-fabric bytes, frac_compulsory_bytes every "
                             "array once.",
                "frac_compulsory_bytes": round(kernel_bytes_min(dom, m, n, nnz, r, e) / (kt[dom] * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4),
                "bytes_compulsory": int(kernel_bytes_min(dom, m, n, nnz, r, e)),
                "frac_counters": None if traffic is None else
                round(traffic / (kt[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "step_traffic": None if step_traffic is None else int(step_traffic),
                "step_traffic_frac": None if step_traffic is None else
                round(step_traffic / (sum(kt.values()) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                # share of the CUs' VALU issue slots the kernel used (committed SQ counters)
                "valu_issue_frac": load_valu_issue(args.workload, kernel_key)}

    variants = {}
    if not args.no_variants:
        vsteps = max(3, args.steps // 4)
        R_ws = torch.empty(nnz, dtype=torch.float32, device=dev)
        dP_ws = torch.empty(nnz, dtype=torch.float32, device=dev)
        t_unf, kt_unf = time_steps(make_step(A, B, fused=False, R_ws=R_ws, dP_ws=dP_ws), vsteps, 2)
        keep("unfused_f32")
        variants["unfused_f32"] = {"ms_per_step": round(t_unf * 1e3, 4), "gflops": round(flops / t_unf / 1e9, 1),
                                   "kernel_ms": {k: round(v, 4) for k, v in kt_unf.items()}}
        log(f"unfused f32 step {t_unf * 1e3:.3f} ms")
        del R_ws, dP_ws
        A16, B16 = F.to_bf16(A), F.to_bf16(B)
        P.autotune(A16, B16, G, form="a")
        t_bf, kt_bf = time_steps(make_step(A16, B16, fused=True), vsteps, 2)
        keep("fused_bf16")
        variants["fused_bf16"] = {"ms_per_step": round(t_bf * 1e3, 4), "gflops": round(flops / t_bf / 1e9, 1),
                                  "kernel_ms": {k: round(v, 4) for k, v in kt_bf.items()},
                                  "tuning_arg": tuning_arg(P.tuning)}
        log(f"fused bf16 step {t_bf * 1e3:.3f} ms")

        # bfloat16 upstream gradient as well (rounded inside the timed step)
        t_bg, kt_bg = time_steps(make_step(A16, B16, fused=True, dc_bf16=True), vsteps, 2)
        keep("fused_bf16_dc_bf16")
        variants["fused_bf16_dc_bf16"] = {"ms_per_step": round(t_bg * 1e3, 4), "gflops": round(flops / t_bg / 1e9, 1),
                                          "kernel_ms": {k: round(v, 4) for k, v in kt_bg.items()},
                                          "note": "dC rounded to bfloat16 in the step (in the bwd_row time)"}
        log(f"fused bf16 step with a bf16 upstream gradient {t_bg * 1e3:.3f} ms")
        restore_tuning(P, tuning)
        variants["speedup_fused_bf16_vs_unfused_f32"] = round(t_unf / t_bf, 3)
        variants["speedup_fused_bf16_dc_bf16_vs_unfused_f32"] = round(t_unf / t_bg, 3)
        variants["speedup_fused_f32_vs_unfused_f32"] = round(t_unf / t_step, 3)
        del A16, B16
        # learned edge values: the adjoint also returns dL/dS; fused, dS is written by the
        # row pass that computes dA, unfused it costs two SDDMM passes on top
        Q = P.with_values(P.val.clone())
        dS = torch.empty(nnz, dtype=torch.float32, device=dev)

        def make_values_step(fused, R_ws=None, dP_ws=None):
            def step(ev=None):
                if ev is not None:
                    ev[0].record()
                F.fusedmm_a_raw(Q, A, B, out=C, fused=fused, R_ws=R_ws)
                if ev is not None:
                    ev[1].record()
                F.fusedmm_a_backward_values_raw(Q, A, B, G, dS=dS, dA=dA, want_dA=fused, fused=fused)
                if not fused:
                    F.fusedmm_a_backward_raw(Q, A, B, G, dA=dA, need=(True, False), fused=False, R_ws=R_ws,
                                             dP_ws=dP_ws)
                if ev is not None:
                    ev[2].record()
                F.fusedmm_a_backward_raw(Q, A, B, G, dB=dB, need=(False, True), fused=fused, R_ws=R_ws, dP_ws=dP_ws)
                if ev is not None:
                    ev[3].record()
            return step
        t_lv, kt_lv = time_steps(make_values_step(True), vsteps, 2)
        R_ws = torch.empty(nnz, dtype=torch.float32, device=dev)
        dP_ws = torch.empty(nnz, dtype=torch.float32, device=dev)
        t_lvu, kt_lvu = time_steps(make_values_step(False, R_ws, dP_ws), vsteps, 2)
        del R_ws, dP_ws, Q, dS
        names = {"fwd": "fwd", "bwd_row": "dS_and_dA", "bwd_col": "dB"}
        variants["learned_values_fused_f32"] = {"ms_per_step": round(t_lv * 1e3, 4),
                                                "kernel_ms": {names[k]: round(v, 4) for k, v in kt_lv.items()}}
        variants["learned_values_unfused_f32"] = {"ms_per_step": round(t_lvu * 1e3, 4),
                                                  "kernel_ms": {names[k]: round(v, 4) for k, v in kt_lvu.items()}}
        log(f"learned values step: fused {t_lv * 1e3:.3f} ms, unfused {t_lvu * 1e3:.3f} ms")
        # FusedMMB forward, fused and unfused
        Cb = torch.empty(n, r, dtype=torch.float32, device=dev)
        Rb = torch.empty(nnz, dtype=torch.float32, device=dev)
        for fused in (True, False):
            for _ in range(2):
                F.fusedmm_b_raw(P, A, B, out=Cb, fused=fused, R_ws=Rb)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(vsteps):
                F.fusedmm_b_raw(P, A, B, out=Cb, fused=fused, R_ws=Rb)
            e1.record()
            torch.cuda.synchronize()
            variants[f"fusedmm_b_fwd_{'fused' if fused else 'unfused'}_ms"] = round(e0.elapsed_time(e1) / vsteps, 4)
        # FusedMMB training step: forward (on the transposed copy), then the adjoint's dB
        # pass on the transposed copy and its two-row dA pass on the CSR
        Gb = torch.from_numpy(np.ascontiguousarray(w["B"][:, ::-1])).to(dev)  # an n x r upstream gradient
        dAb = torch.empty(m, r, dtype=torch.float32, device=dev)
        dBb = torch.empty(n, r, dtype=torch.float32, device=dev)

        def b_step():
            F.fusedmm_b_raw(P, A, B, out=Cb)
            F.fusedmm_b_backward_raw(P, A, B, Gb, dA=dAb, dB=dBb)
        for _ in range(2):
            b_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(vsteps):
            b_step()
        e1.record()
        torch.cuda.synchronize()
        tb = e0.elapsed_time(e1) / vsteps
        variants["fusedmm_b_step_fused_f32"] = {"ms_per_step": round(tb, 4), "gflops": round(flops / tb / 1e6, 1)}
        del Cb, Rb, Gb, dAb, dBb
        # spread of the timed steps, then the same step with L2 and MALL flushed before each
        variants["fused_f32_step_ms_percentiles"] = {
            q: round(float(np.percentile(step_ms, p)), 4) for q, p in (("p10", 10), ("median", 50), ("p90", 90))}
        cold = cold_cache_steps(step_f32, vsteps, kinds, dev)
        variants["fused_f32_cold_cache"] = cold
        log(f"cold-cache fused f32 step: median {cold['median_ms']:.3f} ms")
        ceiling = copy_ceiling(dev)
        roofline["copy_ceiling"] = ceiling
        roofline["frac_of_copy_ceiling"] = round(achieved / ceiling["gbs"], 4)
        roofline["frac_of_read_ceiling"] = round(achieved / ceiling["read_gbs"], 4)
        log(f"ceilings: copy {ceiling['gbs']:.0f} GB/s, read {ceiling['read_gbs']:.0f} GB/s, torch copy "
            f"{ceiling['torch_copy_gbs']:.0f} GB/s; dominant kernel at {achieved / ceiling['gbs']:.3f} / "
            f"{achieved / ceiling['read_gbs']:.3f} of them")
        # random-gather ceilings at the dominant kernel's gathered row size: what the L2-miss
        # path sustains for rows from HBM and for rows held by the MALL
        gc = gather_ceiling(dev, 1 << (min(1024, r * e).bit_length() - 1))  # the probe takes 16·2^k bytes
        roofline["gather_ceiling"] = gc
        if traffic is not None:
            rate = traffic / (kt[dom] * 1e-3) / 1e9
            roofline["frac_counters_of_gather_ceiling"] = round(rate / gc["mall_resident_gbs"], 4)
        log(f"gather ceilings ({gc['row_bytes']} B rows): HBM random {gc['hbm_random_gbs']:.0f} GB/s, "
            f"MALL-resident {gc['mall_resident_gbs']:.0f} GB/s, L2-resident {gc['l2_resident_gbs']:.0f} GB/s")
        variants["pattern_prep_s"] = round(prep_s, 3)
        variants["step_bytes_gather_model"] = int(step_bytes)
        variants["step_hbm_frac_gather_model"] = round(step_bytes / t_step / 1e9 / HBM_PEAK_GBS, 4)

    if args.calibrate_copy:
        calibrate_copy(dev)

    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "nnz": nnz, "r": r, "storage": "f32",
                   "tuning": tuning, "tuning_arg": tuning_arg(tuning),
                   "step": "fused FusedMMA forward + adjoint (dA row pass, dB column pass)",
                   "flops_per_step": flops},
        "roofline": roofline,
        "variants": variants,
    }
    if not args.no_cpu_baseline:
        # the oracle leg: the CPU baseline, and the oracle as the checker of every variant
        log("error report against the FP64 oracle (sampled lines)")
        out["errors"] = error_report(w, outputs, rows_s, cols_s)
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
