"""bench.py's contract pieces that need no GPU: the one-GPU refusal, the
algorithmic byte count behind the roofline, and the committed counter
record it reads."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes():
    # per element 4 coefficient words + x read + x write, per column y + w
    # read + w write: m = 4, n = 262144 in FP32 is 28.3 MB per iteration,
    # the robust program m = 2, q = 200, n = 3600 is 43.2 MB
    assert bench.sweep_bytes(4, 262144, 1, 4) == 28311552
    assert bench.sweep_bytes(2, 3600, 200, 4) == 43200000
    assert bench.sweep_bytes(4, 262144, 1, 8) == 2 * 28311552


def test_traffic_record_is_readable():
    # the committed record parses and names the kernel, the workload and
    # the source digest it was taken on
    path = os.path.join(ROOT, "profiles", "k_chain_m4_n262144_mixed.md")
    rec = [ln for ln in open(path) if ln.startswith("traffic-record:")]
    assert len(rec) == 1
    kv = dict(t.split("=", 1) for t in rec[0].split()[1:])
    assert kv["kernel"] == "k_chain" and kv["m"] == "4" and kv["n"] == "262144"
    assert float(kv["bytes_per_launch"]) > 0.5 * bench.sweep_bytes(4, 262144, 1, 4)
    assert len(kv["sources"]) == 16
    got, src = bench.traffic_record("k_chain", "mixed", 4, 262144)
    if kv["sources"] == bench.kernel_sources_digest():
        assert got == float(kv["bytes_per_launch"]) and src.endswith("k_chain_m4_n262144_mixed.md")
    else:
        assert got is None
