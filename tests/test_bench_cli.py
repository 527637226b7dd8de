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
    """The smoother's committed counter summary names one precision: the
    other precision gets None, and so does the summary's own precision once
    the kernel's source no longer hashes to the recorded value."""
    import bench
    kv = dict(ln.split(":", 1) for ln in open(os.path.join(ROOT, "profiles", "mg0_smooth_traffic.txt")) if ":" in ln)
    prec = kv["precision"].split()[0]
    other = "fp64" if prec == "mixed" else "mixed"
    t = bench.measured_traffic(prec)
    assert t is None or t > 0          # None once the kernel source has changed since the counters
    assert bench.measured_traffic(other) is None


def test_gram_traffic_figure_matches_its_source(tmp_path, monkeypatch):
    """The Gram kernel's committed counter summary is used only for the
    source it was taken on: a copy of the tree with an edited pod.hip gets
    None."""
    import shutil
    import bench
    t = bench.committed_traffic("gram_traffic.txt", ("paper_1704_04139_amd/csrc/pod.hip",), "fp64")
    assert t is None or t > 5.0e8      # at least the snapshot bytes read once
    root = tmp_path / "tree"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_1704_04139_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "gram_traffic.txt"), root / "profiles")
    src = open(os.path.join(ROOT, "paper_1704_04139_amd", "csrc", "pod.hip")).read()
    (root / "paper_1704_04139_amd" / "csrc" / "pod.hip").write_text(src + "\n// edited\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.committed_traffic("gram_traffic.txt", ("paper_1704_04139_amd/csrc/pod.hip",), "fp64") is None
