"""Host-side checks of bench.py: the one-GPU contract and the committed
counter figures it reports as HBM traffic."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_figures_match_the_current_sources():
    # the counter table covers every launch size the autotuner can pick for
    # the 64-vector 1024^2 workload (both FFT-length rules: plan flags 0 and
    # PC_PLAN_SMALLEST_FFT; both launch forms: the small items two per CU in
    # a second launch, or not), and only while the kernel and planner
    # sources are the ones the counters were taken on
    import re
    text = open(bench.TRAFFIC_FILE).read()
    for flags in (0, 4):
        for launch in ("split", "single"):
            sizes = {int(v) for v in re.findall(
                rf"traffic plan_flags={flags} launch={launch} vectors_per_launch=(\d+) ", text)}
            for v in (4, 8, 10, 12, 16, 20, 22, 24, 28, 32):
                t = bench.measured_traffic(v, flags, launch)
                assert t is not None, (flags, launch, v)
                assert 1e8 < t < 1e10
            # 64 vectors beyond the 2 GiB staging cap: two launches summing to 64
            assert any(v > 32 and 64 - v in sizes for v in sizes), (flags, launch, sorted(sizes))
            assert bench.measured_traffic(7, flags, launch) is None
            per_vec = [bench.measured_traffic(v, flags, launch) / v for v in (8, 16, 32)]
            assert max(per_vec) / min(per_vec) < 1.25   # bytes grow with the vectors of a launch
        # the two forms write the same staging boxes
        a, b = bench.measured_traffic(32, flags, "split"), bench.measured_traffic(32, flags, "single")
        assert abs(a - b) < 0.1 * b
    assert bench.measured_traffic(8, 2) is None
