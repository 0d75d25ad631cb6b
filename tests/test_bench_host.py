"""Host-side logic of bench.py (no GPU): the one-GPU rule, the stored counter traffic
that is valid only for the sources it was measured on, and the CPU-baseline record."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stored_traffic_matches_the_current_sources():
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    work = "c3_heterogeneous_ricker_8192x8192_f32"
    ent = data[work]["fused_step"]
    # bytes of a launch: at least the algorithmic 16 B per node of the one-pass step
    assert ent["bytes_per_launch"] >= 16 * 8192 * 8192
    if ent["source_hash"] == bench.kernel_source_hash():
        assert bench.load_traffic(work, "fused_step", 0.0) == float(ent["bytes_per_launch"])
    assert bench.load_traffic("no_such_workload", "fused_step", 0.0) is None
    assert bench.load_traffic(work, "no_such_kernel", 0.0) is None


def test_cpu_baseline_record():
    from paper_2006_10142_amd import workloads as wl
    p = wl.config_c3(dtype="f32", nsteps=2, n=96)
    rec = bench.cpu_baseline(p, 2)
    for key in ("value", "unit", "cores", "kind", "sample", "one_thread", "cpu_model"):
        assert key in rec
    assert rec["kind"] == "oracle" and rec["unit"] == "Mpts/s" and rec["cores"] >= 1
    assert np.isfinite(rec["value"]) and rec["value"] > 0
    assert rec["one_thread"]["value"] > 0
