"""Benchmark of the LRNR / FastLRNR physics-informed hot path on one MI355X.

One step = one fine-tuning step of the full LRNR at working size: forward jets,
CDR residual loss (interior, initial line, periodic boundary), reverse sweep to
s and b (lrnr_grad_s) and the Adam update of s.  Workload: N = 262144 interior
points plus 32768 initial-line and 32768 boundary points, 5 hidden layers of
width 256, rank 20, sin activation, synthetic net and points (seeded).

Prints one JSON line.  Side measurements (FastLRNR vs LRNR on the small net,
FastLRNR speed-up) are attached under "fastlrnr".

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fast]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "colloc pts/s for PINN loss+grad_s (FastLRNR vs LRNR); p50/p99 new-mu latency"
FP32_MFMA_PEAK_TFLOPS = 157.3


def algorithmic_flops(net_M, net_r, n_r, n_value):
    """Dense-contraction flops of one loss+gradient pass: per interior point
    16 W sum_l (r_l + r_{l+1}) (4 jets, forward and adjoint, multiply-add = 2),
    per value-only boundary evaluation a quarter of that.  Recomputation and
    tile padding are not counted."""
    per_pt = 0
    for l in range(1, len(net_r)):
        W = net_M[l]
        per_pt += 16 * W * (net_r[l - 1] + net_r[l])
    return per_pt * n_r + (per_pt // 4) * n_value, per_pt


def run_lrnr(args, torch, api, wl):
    w = wl.big_lrnr(1)
    net = api.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    m = torch.zeros_like(s)
    v = torch.zeros_like(s)
    pts = api.DevicePoints.from_points(w.pts)
    mu = torch.tensor(w.mu[0], device="cuda")
    cfg = api.LossCfg()
    n_r, n_0, n_b = pts.counts
    ws = api.Workspace()
    gs = torch.empty(net.r_total, device="cuda")

    def step(k, ev=None):
        if ev is not None:
            api.time_next_fused(*ev)
        g, _, loss = api.grad_s(net, s, mu, pts, cfg, with_b=True, ws=ws)
        api.adam_step(s, m, v, g, k)
        return loss

    for k in range(1, args.warmup + 1):
        step(k)
    torch.cuda.synchronize()
    kev = [(api.HipEvent(), api.HipEvent()) for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(args.steps):
        loss = step(args.warmup + 1 + i, kev[i])
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    kern_ms = [a.elapsed_ms(b) for a, b in kev]
    flops, per_pt = algorithmic_flops(w.net.M, w.net.r, n_r, n_0 + 2 * n_b)
    kavg = float(np.mean(kern_ms))
    achieved = flops / (kavg * 1e-3) / 1e12
    return {
        "ms_per_step": total_ms / args.steps,
        "pts_per_s": n_r / (total_ms / args.steps * 1e-3),
        "kernel_ms_avg": kavg,
        "kernel_ms_min": float(np.min(kern_ms)),
        "flops_per_launch": flops,
        "flops_per_interior_point": per_pt,
        "achieved_tflops": achieved,
        "final_loss": float(loss[0]),
        "counts": (n_r, n_0, n_b),
        "w": w,
    }


def time_calls(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def run_fast(args, torch, api, wl):
    """LRNR vs FastLRNR loss+grad_s on the small net (64 wide, rank 8),
    N = 65536 interior points, r_hat = 32 built from 2048 snapshot points."""
    w = wl.fast_case(2)
    net = api.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    pts = api.DevicePoints.from_points(w.pts)
    mu = torch.tensor(w.mu[0], device="cuda")
    cfg = api.LossCfg()
    t = time.time()
    fast = api.FastLRNR(net, s.reshape(1, -1), torch.tensor(w.extra["xt_snap"], device="cuda"),
                        w.extra["r_hat"])
    build_s = time.time() - t
    ws1, ws2 = api.Workspace(), api.Workspace()
    steps = max(20, args.steps)
    ms_l = time_calls(torch, lambda: api.grad_s(net, s, mu, pts, cfg, with_b=False, ws=ws1),
                      steps, 5)
    ms_f = time_calls(torch, lambda: fast.grad_s(s, mu, pts, cfg, ws=ws2), steps, 5)
    n_r = pts.counts[0]
    fast.close()
    return {
        "workload": "small net 64 wide x 4 hidden, rank 8; N=65536 (+8192 IC, +8192 BC); "
                    "r_hat=32 from 2048 snapshot points",
        "lrnr_ms": ms_l, "fastlrnr_ms": ms_f,
        "lrnr_pts_per_s": n_r / (ms_l * 1e-3), "fastlrnr_pts_per_s": n_r / (ms_f * 1e-3),
        "speedup": ms_l / ms_f, "build_s": build_s,
    }


def cpu_baseline(w, wl):
    """The FP64 oracle on a bounded sample of the same workload."""
    from oracle import lrnr_oracle as orc
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    n = 16384
    sub = wl.Points(w.pts.xt_r[:n], w.pts.x_0[:n // 8], w.pts.t_b[:n // 8])
    t = time.time()
    reps = 0
    while True:
        orc.lrnr_loss_chunked(w.net, w.net.s, w.mu[0].astype(np.float64), sub, {}, chunk=8192)
        reps += 1
        el = time.time() - t
        if el > 10.0:
            break
    return {
        "value": reps * n / el, "unit": "pts/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{reps} x loss+grad_s,b on the first {n} interior (+{n // 8} IC, +{n // 8} BC) "
                  f"points of the same workload, FP64 numpy, {el:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fast", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the loss+gradient shards over points with one small all-reduce; see the "
              "design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as wl
    from paper_2410_04001_amd import api

    torch.cuda.init()
    r = run_lrnr(args, torch, api, wl)
    n_r, n_0, n_b = r["counts"]
    fast = None if args.no_fast else run_fast(args, torch, api, wl)
    out = {
        "metric": METRIC,
        "value": r["pts_per_s"],
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "LRNR fine-tuning step (loss + grad_s,b + Adam): 5 hidden layers width "
                        "256, rank 20, sin; N=262144 interior + 32768 IC + 32768 BC points; "
                        "CDR residual mu=(%.3f, %.3f, %.3f)" % tuple(r["w"].mu[0]),
            "n_interior": n_r, "n_ic": n_0, "n_bc": n_b,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": r["achieved_tflops"],
            "peak": FP32_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": r["achieved_tflops"] / FP32_MFMA_PEAK_TFLOPS,
            "traffic": None,
            "kernel": "lrnr_fused_kernel<20, MODE_GRAD>",
            "kernel_ms_avg": r["kernel_ms_avg"],
            "flops_per_launch": r["flops_per_launch"],
        },
    }
    if fast is not None:
        out["fastlrnr"] = fast
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(r["w"], wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
