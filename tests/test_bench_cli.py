"""bench.py's contract on the CPU: one GPU only, and the roofline objects it
reports (no device needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_hbm_roofline_arithmetic():
    sys.path.insert(0, ROOT)
    import bench
    v = {"total_ms": 2.0, "launches": 4, "bytes": 4.0e9}
    rl = bench.hbm_roofline("spmv", v, "no_such_workload")
    # 1 GB per launch in 0.5 ms = 2000 GB/s
    assert rl["achieved"] == pytest.approx(2000.0)
    assert rl["frac"] == pytest.approx(2000.0 / bench.PEAK_HBM_GBS)
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["traffic"] is None
    assert rl["avg_launch_ms"] == pytest.approx(0.5) and rl["bytes_per_launch"] == pytest.approx(1.0e9)
