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


def _fake_record():
    rate = lambda r: {"offered_req_per_s": r, "req_per_s": r * 0.99, "p50_ms": 10.123456,
                      "p99_ms": 20.654321, "requests": 2000, "mean_ms": 11.0}
    return {
        "metric": "m", "value": 8.8e7, "unit": "pts/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "warmup_effective": 10, "ms_per_step": 2.98, "ms_per_step_mean": 2.99,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "w" * 300, "n_interior": 262144, "n_ic": 32768, "n_bc": 32768},
        "roofline": {"bound": "mfma", "achieved": 64.4, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": 0.41, "traffic": 1.13e9, "kernel": "k" * 60,
                     "kernel_ms_avg": 2.96, "kernel_ms_median": 2.95, "flops_per_launch": 1.9e11},
        "cpu_baseline": {"value": 1.3e4, "unit": "pts/s", "cores": 16, "kind": "oracle",
                         "value_1_thread": 3e3, "nproc": 128, "sample": "s" * 200},
        "per_mu": [{"mu": [1.0, 2.0, 3.0], "ms_per_step": 2.9}] * 8,
        "fastlrnr": {"lrnr_ms": 0.119, "fastlrnr_ms": 0.071, "speedup": 1.68, "build_s": 0.3},
        "equal_accuracy": [{"time_ratio_lrnr_over_fast": 1.68}, {"time_ratio_lrnr_over_fast": 4.7}],
        "differentiation": {"ms_per_adam_step": 0.70, "ms_per_adam_step_recompute": 0.94,
                            "fused_loss_grad_ms": 0.64},
        "serving": {"rates": [rate(r) for r in (50, 100, 200, 500, 1000, 2000)]},
        "meta": {"ms_per_meta_step": 1.38},
        "fidelity": {"rows": [{"r_hat": 8, "x": list(range(50))}] * 28},
    }


def test_headline_is_the_compact_last_line(tmp_path):
    sys.path.insert(0, ROOT)
    import json

    import bench
    out = _fake_record()
    path = str(tmp_path / "full.json")
    bench.write_full(out, path)
    line = json.dumps(bench.headline(out, path))
    assert len(line) <= 2048, len(line)
    h = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in h, k
    assert h["roofline"]["frac"] == 0.41 and h["cpu_baseline"]["cores"] == 16
    assert len(h["legs"]["serving_rate_achieved_p50_p99_ms"]) == 6
    assert json.load(open(path))["fidelity"]["rows"][0]["r_hat"] == 8


def test_cpu_baseline_reports_one_thread_and_all_threads():
    sys.path.insert(0, ROOT)
    import bench
    import workloads as wl
    cb = bench.cpu_baseline(wl.small_lrnr(0), wl, seconds=0.05)
    assert cb["kind"] == "oracle" and cb["unit"] == "pts/s"
    assert cb["value"] > 0 and cb["value_1_thread"] > 0
    assert 1 <= cb["cores"] <= bench.cpu_threads()
