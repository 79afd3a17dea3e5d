"""Host-side behaviour of bench.py that needs no GPU: it measures one GPU
only and refuses a multi-GPU request before touching the device, and the
HBM-traffic figure is reported only for the kernel source it was counted on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_figure_follows_the_kernel_source(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_source_sha()
    assert len(sha) == 64
    t = bench.measured_traffic()
    assert t is None or t > 0
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    assert bench.measured_traffic() is None
