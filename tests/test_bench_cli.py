"""Host-side behaviour of bench.py (no GPU): the multi-GPU refusal and the
measured-traffic lookup."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_figure_only_for_its_precision_and_source():
    import bench
    t = bench.measured_traffic("fp64")
    assert t is None or t > 0          # None once the kernel source has changed since the counters
    assert bench.measured_traffic("mixed") is None
