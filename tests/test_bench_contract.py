"""The benchmark's contract, checked without a GPU: one GPU only, and the
committed counter summary it reads belongs to the kernels in the tree."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "single" in r.stderr, r.stderr
    assert r.stdout.strip() == ""


def test_committed_counters_match_the_kernel_sources():
    """profiles/fluid_sweep_traffic_256.json was taken on the kernels in the
    tree (else bench.py reports traffic and VALU issue as null): its hash is
    the hash of physics.h and sweeps.h, and it holds both figures."""
    with open(os.path.join(ROOT, "profiles", "fluid_sweep_traffic_256.json")) as f:
        rec = json.load(f)
    assert rec["kernel_hash"] == bench.kernel_source_hash()
    assert rec["cells"] == 256 ** 3 and rec["esize"] == 4
    traffic, valu = bench.load_counters("fluid_sweep_traffic_256.json", 4, 256 ** 3)
    assert traffic == rec["bytes_per_launch"] and traffic > rec["algorithmic_bytes_per_launch"] * 0.9
    assert valu == rec["valu_wave_insts_per_launch"] and valu > 0


def test_valu_issue_peak():
    # 256 CUs x 4 SIMDs x 64 lanes / 4 cycles x 2.4 GHz
    assert abs(bench.VALU_PEAK_LANE_INSTS - 3.93216e13) < 1e6
