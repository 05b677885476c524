"""Host side of the benchmark script: the one-GPU contract, the named side
workloads and the traffic table (no GPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2110_15425_amd import cm  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_every_side_workload_is_a_valid_sweep():
    assert len(set(bench.SIDE_WORKLOADS)) == len(bench.SIDE_WORKLOADS)
    for name in bench.SIDE_WORKLOADS:
        w, how = bench._side(name)
        assert how in ("launch", "density", "timecourse", "unfused"), name
        assert cm.validate(w) == cm.OK, name


def test_traffic_table_shape():
    t = bench.TRAFFIC
    assert len(t["sources_sha256"]) == 64 and t["batch"] == bench.BATCH
    # keyed "runs_per_lane,block,tail_sweeps" of the profiled launch shape
    for k, v in t["bytes_per_launch"].items():
        rpl, block, tail = (int(x) for x in k.split(","))
        assert rpl >= 1 and block in (256, 512, 1024) and 0 <= tail <= bench.BATCH and v > 0, k
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f


def test_roofline_peak_and_step_count():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert bench.PEAK_LANE_OPS == pytest.approx(39.3216e12)
    assert 60 <= bench.LANE_OPS_PER_STEP["fp32_step"] <= 70
