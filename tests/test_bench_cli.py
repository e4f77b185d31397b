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
            assert any(k.startswith("line_kernel<") for k in t["kernels"])
