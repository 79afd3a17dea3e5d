"""Benchmark of the LRNR / FastLRNR physics-informed hot path on one MI355X.

One step = one fine-tuning step of the full LRNR at working size: forward jets,
CDR residual loss (interior, initial line, periodic boundary), reverse sweep to
s and b (lrnr_grad_s) and the Adam update of s.  Workload: N = 262144 interior
points plus 32768 initial-line and 32768 boundary points, 5 hidden layers of
width 256, rank 20, sin activation, synthetic net and points (seeded).

The last line on stdout is one compact JSON record (the headline: metric,
value, median ms per step, roofline, CPU baseline and one-line summaries of
the side legs).  The full record of every leg is written to --out (default
bench_full.json in the working directory); each leg prints a progress line
to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fast]
                  [--no-equal-acc] [--no-diff] [--no-serve] [--serve-rates 50,100,...]
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
# A fresh launch sequence runs at a lower clock for about 9 steps (visible in the
# kernel trace of the working-size step), so at least this many untimed steps
# precede the timed ones whatever --warmup asks for.
CLOCK_RAMP_WARMUP = 10


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

    warm = max(args.warmup, CLOCK_RAMP_WARMUP)
    for k in range(1, warm + 1):
        step(k)
    torch.cuda.synchronize()
    kev = [(api.HipEvent(), api.HipEvent()) for _ in range(args.steps)]
    # one event at every step boundary: per-step times for the median
    bev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    bev[0].record()
    for i in range(args.steps):
        loss = step(warm + 1 + i, kev[i])
        bev[i + 1].record()
    torch.cuda.synchronize()
    step_ms = [bev[i].elapsed_time(bev[i + 1]) for i in range(args.steps)]
    total_ms = bev[0].elapsed_time(bev[-1])
    kern_ms = [a.elapsed_ms(b) for a, b in kev]
    flops, per_pt = algorithmic_flops(w.net.M, w.net.r, n_r, n_0 + 2 * n_b)
    kavg = float(np.mean(kern_ms))
    achieved = flops / (kavg * 1e-3) / 1e12
    # the same step at each of the workload's 8 parameter draws (own s, m, v)
    per_mu = []
    for j in range(0 if args.no_per_mu else len(w.mu)):
        mu_j = torch.tensor(w.mu[j], device="cuda")
        s_j = torch.tensor(w.net.s_flat(), device="cuda")
        m_j, v_j = torch.zeros_like(s_j), torch.zeros_like(s_j)
        it = [0]

        def step_j():
            it[0] += 1
            g, _, _ = api.grad_s(net, s_j, mu_j, pts, cfg, with_b=True, ws=ws)
            api.adam_step(s_j, m_j, v_j, g, it[0])

        ms_j = time_calls(torch, step_j, 10, 3)
        per_mu.append({"mu": [float(x) for x in w.mu[j]], "ms_per_step": ms_j,
                       "pts_per_s": n_r / (ms_j * 1e-3)})
    med = float(np.median(step_ms))
    return {
        "per_mu": per_mu,
        "warmup_effective": warm,
        "ms_per_step": med,
        "ms_per_step_mean": total_ms / args.steps,
        "pts_per_s": n_r / (med * 1e-3),
        "kernel_ms_avg": kavg,
        "kernel_ms_median": float(np.median(kern_ms)),
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


def run_factored_bias(args, torch, api, wl):
    """Factored biases b^l = B^l s_b^l (q = 8 columns per layer, seeded
    Gaussian basis): loss + grad_s + grad_sb against the plain loss + grad_s,b,
    on the small net (N = 65536) for the LRNR and the FastLRNR (r_hat = 32),
    and on the working-size net (N = 262144)."""
    out = {}
    for name, w in (("small", wl.fast_case(2)), ("working", wl.big_lrnr(1))):
        rng = np.random.Generator(np.random.PCG64(5))
        B = [(rng.standard_normal((m, min(8, m))) / math.sqrt(m)).astype(np.float32)
             for m in w.net.M[1:]]
        bb = api.BiasBasis(w.net.M, [b.shape[1] for b in B],
                           np.concatenate([b.reshape(-1) for b in B]))
        s_b = torch.tensor(rng.uniform(-1, 1, bb.q_total).astype(np.float32), device="cuda")
        net = api.DeviceNet.from_net(w.net)
        s = torch.tensor(w.net.s_flat(), device="cuda")
        pts = api.DevicePoints.from_points(w.pts)
        mu = torch.tensor(w.mu[0], device="cuda")
        cfg = api.LossCfg()
        ws = api.Workspace()
        steps = max(20, args.steps)
        row = {
            "plain_ms": time_calls(torch, lambda: api.grad_s(net, s, mu, pts, cfg, ws=ws), steps, 5),
            "factored_ms": time_calls(
                torch, lambda: api.grad_s_factored(net, bb, s, s_b, mu, pts, cfg, ws=ws), steps, 5),
            "n_interior": pts.counts[0], "q": bb.q,
        }
        if name == "small":
            fast = api.FastLRNR(net, s.reshape(1, -1),
                                torch.tensor(w.extra["xt_snap"], device="cuda"), w.extra["r_hat"])
            red = fast.bias_basis(bb)
            row["fastlrnr_plain_ms"] = time_calls(
                torch, lambda: api.grad_s(fast.net, s, mu, pts, cfg, ws=ws), steps, 5)
            row["fastlrnr_factored_ms"] = time_calls(
                torch, lambda: api.grad_s_factored(fast.net, red, s, s_b, mu, pts, cfg, ws=ws),
                steps, 5)
            fast.close()
        out[name] = row
    return out


def run_fidelity(args, torch, api, wl):
    """FastLRNR fidelity against the reduced width r_hat (the sweep of
    Fig. 2 (bottom), on a synthetic net): on the small net (64 wide, rank 8)
    with the 65536 training points of the FastLRNR comparison, the FastLRNR
    loss and grad_s against the LRNR's at the same s, and u and the reduced
    states z_hat^l (against V^{(l+1)T} z^l) at 16384 held-out points, for DEIM and Q-DEIM index selection, each from snapshots at s
    alone and at s plus 7 perturbed copies (each entry scaled by
    1 + 0.1 N(0, 1)); with the build time and the FastLRNR loss+grad time."""
    import numpy as np
    w = wl.fast_case(2)
    net = api.DeviceNet.from_net(w.net)
    s_host = w.net.s_flat()
    s = torch.tensor(s_host, device="cuda")
    pts = api.DevicePoints.from_points(w.pts)
    mu = torch.tensor(w.mu[0], device="cuda")
    cfg = api.LossCfg()
    xs = torch.tensor(w.extra["xt_snap"], device="cuda")
    rng = np.random.Generator(np.random.PCG64(9))
    xt_held = torch.tensor(wl.uniform_points(rng, 16384), device="cuda")
    pert = [s_host] + [(s_host * (1.0 + 0.1 * rng.standard_normal(s_host.shape))).astype(np.float32)
                       for _ in range(7)]
    snaps = {"s": s.reshape(1, -1), "s + 7 perturbed": torch.tensor(np.stack(pert), device="cuda")}
    gs_l, _, loss_l = api.grad_s(net, s, mu, pts, cfg, with_b=False)
    u_l = api.forward_value(net, s, xt_held)
    y_l = [y.double() for y in api.reduced_states(net, s, xt_held)]
    ms_l = time_calls(torch, lambda: api.grad_s(net, s, mu, pts, cfg, with_b=False), 20, 3)
    torch.cuda.synchronize()
    gl = gs_l.double()
    rows = []
    for r_hat in (4, 8, 12, 16, 24, 32, 48, 64):
        for sel in ("deim", "qdeim"):
            for name, snap in snaps.items():
                torch.cuda.synchronize()
                t = time.time()
                fast = api.FastLRNR(net, snap, xs, r_hat, selection=sel)
                torch.cuda.synchronize()
                build_ms = (time.time() - t) * 1e3
                gs_f, loss_f = fast.grad_s(s, mu, pts, cfg)
                u_f = api.forward_value(fast.net, s, xt_held)
                ms_f = time_calls(torch, lambda: fast.grad_s(s, mu, pts, cfg), 20, 3)
                gf = gs_f.double()
                rows.append({
                    "r_hat": r_hat, "selection": sel, "snapshots": name,
                    "grad_rel_err": float((gf - gl).norm() / gl.norm()),
                    "grad_cosine": float((gf @ gl) / (gf.norm() * gl.norm())),
                    "loss_rel_err": float(abs(loss_f[0].double() - loss_l[0].double()) / loss_l[0].double()),
                    "u_heldout_rel_err": float((u_f.double() - u_l.double()).norm() / u_l.double().norm()),
                    "state_rel_err": [float((yf.double() - yl).norm() / yl.norm()) for yf, yl in
                                      zip(api.reduced_states(fast.net, s, xt_held), y_l)],
                    "build_ms": build_ms, "fastlrnr_grad_ms": ms_f, "lrnr_grad_ms": ms_l,
                })
                fast.close()
    return {"workload": "small net 64 wide x 4 hidden, rank 8; N=65536 (+8192 IC, +8192 BC); "
                        "2048 snapshot points; 16384 held-out points",
            "rows": rows}


def run_equal_accuracy(args, torch, api, wl, big):
    """FastLRNR against LRNR at equal residual accuracy.  From s_init, Adam
    (lr 1e-3) with the LRNR gradient and, separately, with the FastLRNR
    gradient on the same training points; after every step the true (full
    LRNR) loss on a held-out point set is evaluated outside the timed region.
    The target is L* = L_0 - (L_0 - L_LRNR@100) / 2; reported: the summed
    step times each method needs to reach it."""
    w = wl.equal_accuracy_case(big=big)
    net = api.DeviceNet.from_net(w.net)
    s_init = torch.tensor(w.net.s_flat(), device="cuda")
    pts = api.DevicePoints.from_points(w.pts)
    held = api.DevicePoints.from_points(w.extra["heldout"])
    mu = torch.tensor(w.mu[0], device="cuda")
    cfg = api.LossCfg()
    fast = api.FastLRNR(net, s_init.reshape(1, -1),
                        torch.tensor(w.extra["xt_snap"], device="cuda"), w.extra["r_hat"])
    ws_t, ws_e = api.Workspace(), api.Workspace()

    def held_loss(s):
        return float(api.residual_loss(net, s, mu, held, cfg, ws=ws_e)[0])

    def train(grad_fn, n_steps):
        # steps run back to back; the trajectory of s is kept and the held-out
        # loss is evaluated afterwards
        s = s_init.clone()
        m, v = torch.zeros_like(s), torch.zeros_like(s)
        traj = torch.empty((n_steps + 1, s.numel()), device="cuda")
        traj[0].copy_(s)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(n_steps)]
        for k in range(1, n_steps + 1):
            evs[k - 1][0].record()
            g = grad_fn(s)
            api.adam_step(s, m, v, g, k)
            evs[k - 1][1].record()
            traj[k].copy_(s)
        torch.cuda.synchronize()
        times = np.array([a.elapsed_time(b) for a, b in evs])
        hist = np.array([held_loss(traj[k].contiguous()) for k in range(n_steps + 1)])
        return hist, times

    lrnr_grad = lambda s: api.grad_s(net, s, mu, pts, cfg, with_b=False, ws=ws_t)[0]
    fast_grad = lambda s: fast.grad_s(s, mu, pts, cfg, ws=ws_t)[0]
    train(lrnr_grad, 3)  # warm-up
    train(fast_grad, 3)
    hl, tl = train(lrnr_grad, 100)
    hf, tf = train(fast_grad, 300)
    L0, L100 = hl[0], hl[100]
    target = L0 - 0.5 * (L0 - L100)

    def reach(h, t):
        idx = np.nonzero(h[1:] <= target)[0]
        if len(idx) == 0:
            return None, None
        k = int(idx[0]) + 1
        return k, float(np.sum(t[:k]))

    kl, ms_l = reach(hl, tl)
    kf, ms_f = reach(hf, tf)
    n_r = pts.counts[0]
    fast.close()
    M = w.net.M
    return {
        "net": f"{len(M) - 2} hidden x {M[1]} wide, rank {max(w.net.r)}",
        "r_hat": w.extra["r_hat"], "n_train": n_r, "n_heldout": held.counts[0],
        "L0": L0, "L_lrnr_100": L100, "L_target": target,
        "L_fast_100": float(hf[100]), "L_fast_300": float(hf[300]),
        "lrnr_steps_to_target": kl, "lrnr_ms_to_target": ms_l,
        "fastlrnr_steps_to_target": kf, "fastlrnr_ms_to_target": ms_f,
        "time_ratio_lrnr_over_fast": (ms_l / ms_f) if (ms_l and ms_f) else None,
        "lrnr_step_ms_median": float(np.median(tl)),
        "fastlrnr_step_ms_median": float(np.median(tf)),
        "lrnr_pts_per_s": n_r / (float(np.median(tl)) * 1e-3),
        "fastlrnr_pts_per_s": n_r / (float(np.median(tf)) * 1e-3),
    }


def run_reference(args, torch, api, wl, big):
    """Error against wall time (the Section 4 comparison of Fig. 3): 20 test
    parameters (10 from each domain of Section 4), the FP64 reference solution
    of eq. 4.1 on the device (lrnr_cdr_reference: 256 grid points, 1000 Strang
    steps, 101 output times on t in [0, 1]); for every case whose solution
    stays bounded, Adam (lr 1e-3) on s from s_init with the LRNR gradient and,
    separately, with the FastLRNR gradient (built once from snapshots at s_init
    and, on the small net, 7 perturbed copies), 400 steps each; every 20 steps the L1 relative
    error of the LRNR at the current s on the reference grid (lrnr_l1_error),
    against the summed step time (HIP events; evaluation outside it)."""
    n_x, n_t, n_out, n_steps, every = 256, 1000, 101, 400, 20
    w = wl.equal_accuracy_case(big=big)
    net = api.DeviceNet.from_net(w.net)
    s_init = torch.tensor(w.net.s_flat(), device="cuda")
    pts = api.DevicePoints.from_points(w.pts)
    cfg = api.LossCfg()
    mus = wl.cdr_test_cases()
    mu_d = torch.tensor(mus, device="cuda")
    api.cdr_reference(mu_d, n_x, n_t, n_out)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        u_ref, st = api.cdr_reference(mu_d, n_x, n_t, n_out)
    ev1.record()
    torch.cuda.synchronize()
    solve_ms = ev0.elapsed_time(ev1) / 5
    st = st.cpu().numpy()
    # throughput: 1024 instances (512 per domain) in one launch
    mu_big = torch.tensor(wl.cdr_test_cases(6, 512, 512), device="cuda")
    api.cdr_reference(mu_big, n_x, n_t, n_out)
    ev0.record()
    for _ in range(3):
        api.cdr_reference(mu_big, n_x, n_t, n_out)
    ev1.record()
    torch.cuda.synchronize()
    solve_ms_1024 = ev0.elapsed_time(ev1) / 3
    rng = np.random.Generator(np.random.PCG64(11))
    s0 = w.net.s_flat()
    n_pert = 0 if big else 7   # the wide net's POD would take ~40 s on 8 snapshot sets
    snaps = [s0] + [(s0 * (1.0 + 0.1 * rng.standard_normal(s0.shape))).astype(np.float32)
                    for _ in range(n_pert)]
    fast = api.FastLRNR(net, torch.tensor(np.stack(snaps), device="cuda"),
                        torch.tensor(w.extra["xt_snap"], device="cuda"), w.extra["r_hat"])
    xt = torch.tensor(wl.grid_points(n_x, n_out), device="cuda")
    ws_t = api.Workspace()
    sums = torch.empty(2, dtype=torch.float64, device="cuda")

    def l1(s, ref):
        u = api.forward_value(net, s, xt)
        api.l1_error_sums(u, ref, out=sums)
        a, b = sums.cpu().numpy()
        return float(a / b)

    def train(grad_fn, ref):
        s = s_init.clone()
        m, v = torch.zeros_like(s), torch.zeros_like(s)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(n_steps)]
        errs, ms, acc = [l1(s, ref)], [0.0], []
        for k in range(1, n_steps + 1):
            evs[k - 1][0].record()
            g = grad_fn(s)
            api.adam_step(s, m, v, g, k)
            evs[k - 1][1].record()
            if k % every == 0:
                errs.append(l1(s, ref))
        torch.cuda.synchronize()
        t = np.cumsum([a.elapsed_time(b) for a, b in evs])
        ms += [float(t[k - 1]) for k in range(every, n_steps + 1, every)]
        return errs, ms

    cases = []
    for i, mu in enumerate(mus):
        if st[i]:
            cases.append({"mu": mu.tolist(), "blow_up_step": int(st[i])})
            continue
        ref = u_ref[i].reshape(-1)
        mu32 = torch.tensor(mu.astype(np.float32), device="cuda")
        lg = lambda s: api.grad_s(net, s, mu32, pts, cfg, with_b=False, ws=ws_t)[0]
        fg = lambda s: fast.grad_s(s, mu32, pts, cfg, ws=ws_t)[0]
        if not any("lrnr_l1" in c for c in cases):   # warm both loops once
            train(lg, ref)
            train(fg, ref)
        el, tl = train(lg, ref)
        ef, tf = train(fg, ref)
        # time LRNR needs to reach FastLRNR's best error
        best_f = min(ef)
        k_l = next((k for k, e in enumerate(el) if e <= best_f), None)
        cases.append({
            "mu": mu.tolist(), "l1_init": el[0],
            "lrnr_l1": el, "lrnr_ms": tl, "fastlrnr_l1": ef, "fastlrnr_ms": tf,
            "lrnr_l1_final": el[-1], "fastlrnr_l1_best": best_f,
            "fastlrnr_ms_to_best": tf[int(np.argmin(ef))],
            "lrnr_ms_to_fast_best": tl[k_l] if k_l is not None else None,
        })
    fast.close()
    M = w.net.M
    run = [c for c in cases if "lrnr_l1" in c]
    return {
        "net": f"{len(M) - 2} hidden x {M[1]} wide, rank {max(w.net.r)}",
        "r_hat": w.extra["r_hat"], "n_train": pts.counts[0], "snapshot_sets": 1 + n_pert,
        "reference": {"n_x": n_x, "n_t": n_t, "n_out": n_out, "instances": len(mus),
                      "ms_per_solve_batch": solve_ms,
                      "ms_per_solve_batch_1024": solve_ms_1024,
                      "instances_per_s_1024": 1024 / (solve_ms_1024 * 1e-3),
                      "blown_up": int(np.count_nonzero(st))},
        "cases": cases,
        "fast_better_or_equal_at_end": sum(1 for c in run if c["fastlrnr_l1"][-1] <= c["lrnr_l1"][-1]),
        "n_run": len(run),
    }


def run_meta(args, torch, api, wl):
    """Meta-learning of the coefficient map with fixed bases (Section 3.1,
    eq. 3.1-3.4 without the basis updates), and of the map and the biases b
    together (U, V fixed): the small net, 64 parameter
    samples sharing 16384 interior (+2048 IC, +2048 BC) points, hypernetwork
    widths (3, 33, 33, 33), R_sparse with gamma = 1.5 and weight 1e-3, Adam
    (lr 1e-3) on Theta for 200 steps.  Reported: ms per meta step (hypernetwork
    forward, batched loss gradient, hypernetwork backward, Adam), its parts,
    and the objective at the first and last step."""
    w = wl.batched_case()
    net = api.DeviceNet.from_net(w.net)
    pts = api.DevicePoints.from_points(w.pts)
    mu = torch.tensor(w.mu, device="cuda")
    R = w.net.r_total
    H = [3, R, R, R]
    theta = torch.tensor(wl.hyper_init(H), device="cuda")
    f = api.Hyper(H, theta)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    cfg = api.LossCfg()
    ws = api.Workspace()
    gamma, lam = 1.5, 1e-3
    hist = []

    def step(k, record=False):
        g, loss, r = api.meta_grad(f, net, mu, pts, cfg, gamma, lam, ws=ws)
        api.adam_step(theta, m, v, g, k)
        if record:
            hist.append((loss, r))

    step(1, True)
    torch.cuda.synchronize()
    n_steps = 200
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for k in range(2, n_steps + 1):
        step(k, record=(k == n_steps))
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / (n_steps - 1)
    s = api.hyper_forward(f, mu)
    gs, _ = api.grad_s_batched(net, s, mu, pts, cfg, ws=ws)
    ms_f = time_calls(torch, lambda: api.hyper_forward(f, mu), 20, 3)
    ms_g = time_calls(torch, lambda: api.grad_s_batched(net, s, mu, pts, cfg, ws=ws), 20, 3)
    ms_b = time_calls(torch, lambda: api.hyper_backward(f, net, mu, gs, gamma, lam), 20, 3)

    def obj(i):
        loss, r = hist[i]
        return float(loss[:, 0].double().mean()) + lam * float(r[0])

    # the same from the same start, training the biases b too (task table of
    # GRAD tasks with per-sample grad_b, mean over the samples)
    net_b = api.DeviceNet.from_net(w.net)
    theta_b = torch.tensor(wl.hyper_init(H), device="cuda")
    f_b = api.Hyper(H, theta_b)
    meta_b = api.MetaStep(f_b, net_b, mu, pts)
    mt, vt = torch.zeros_like(theta_b), torch.zeros_like(theta_b)
    mb, vb = torch.zeros_like(net_b.b), torch.zeros_like(net_b.b)
    hist_b = []
    evb = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    evb[0].record()
    for k in range(1, n_steps + 1):
        g, gb, loss, r = meta_b(cfg, gamma, lam, ws=ws)
        if k in (1, n_steps):
            hist_b.append((loss.clone(), r.clone()))
        api.adam_step(theta_b, mt, vt, g, k)
        api.adam_step(net_b.b, mb, vb, gb, k)
    evb[1].record()
    torch.cuda.synchronize()
    ms_b_step = evb[0].elapsed_time(evb[1]) / n_steps
    obj_b = [float(l[:, 0].double().mean()) + lam * float(rr[0]) for l, rr in hist_b]

    # all of eq. 3.4: Theta, b, U and V (the mean basis gradient over the
    # samples in one fused launch, and R_orth with weight 1e-3) on all 64
    # samples, 200 steps
    net_u = api.DeviceNet.from_net(w.net)
    theta_u = torch.tensor(wl.hyper_init(H), device="cuda")
    f_u = api.Hyper(H, theta_u)
    meta_u = api.MetaStep(f_u, net_u, mu, pts)
    lam_o = 1e-3
    params = [theta_u, net_u.b, net_u.U, net_u.V]
    mom = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    hist_u = []
    evu = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    evu[0].record()
    n_u = n_steps
    for k in range(1, n_u + 1):
        g, gb, loss, r = meta_u(cfg, gamma, lam, ws=ws)
        gU, gV = api.basis_grad_batched(net_u, meta_u.s, mu, pts, cfg, ws=ws)
        ro, gUo, gVo = api.orth_reg(net_u)
        gU = gU + lam_o * gUo
        gV = gV + lam_o * gVo
        if k in (1, n_u):
            hist_u.append((loss.clone(), r.clone(), ro.clone()))
        for p_, (m_, v_), g_ in zip(params, mom, (g, gb, gU, gV)):
            api.adam_step(p_, m_, v_, g_, k)
    evu[1].record()
    torch.cuda.synchronize()
    ms_u_step = evu[0].elapsed_time(evu[1]) / n_u
    obj_u = [float(l[:, 0].double().mean()) + lam * float(rr[0]) + lam_o * float(oo[0])
             for l, rr, oo in hist_u]
    # the basis gradient alone: the 64-sample mean in one launch, and one
    # sample (16384 interior + 2048 IC + 2 x 2048 BC evaluation points)
    s_u = meta_u.s.clone()
    ms_bg64 = time_calls(torch, lambda: api.basis_grad_batched(net_u, s_u, mu, pts, cfg, ws=ws),
                         20, 3)
    s_1, mu_1 = s_u[0].contiguous(), mu[0].contiguous()
    ms_bg1 = time_calls(torch, lambda: api.basis_grad(net_u, s_1, mu_1, pts, cfg, ws=ws), 20, 3)

    n_r = pts.counts[0]
    return {
        "workload": "small net 64 wide x 4 hidden, rank 8; 64 mu samples sharing 16384 interior "
                    "(+2048 IC, +2048 BC) points; hypernetwork (3, 33, 33, 33), sin, ReLU output; "
                    "gamma 1.5, lambda_sparse 1e-3; Adam lr 1e-3, 200 steps",
        "ms_per_meta_step": ms, "pts_per_s": 64 * n_r / (ms * 1e-3),
        "hyper_forward_ms": ms_f, "batched_grad_ms": ms_g, "hyper_backward_ms": ms_b,
        "objective_first": obj(0), "objective_last": obj(1),
        "with_biases": {"ms_per_meta_step": ms_b_step, "objective_first": obj_b[0],
                        "objective_last": obj_b[1]},
        "with_bases_64_samples": {"ms_per_meta_step": ms_u_step, "steps": n_u,
                                  "objective_first": obj_u[0], "objective_last": obj_u[1],
                                  "lambda_orth": lam_o,
                                  "basis_grad_ms_64_samples": ms_bg64,
                                  "basis_grad_ms_per_sample_batched": ms_bg64 / 64,
                                  "basis_grad_ms_one_sample": ms_bg1},
        "theta_params": int(theta.numel()),
    }


def run_pipeline(args, torch, api, wl):
    """The workflow of Section 3 on the small net: (1) meta phase, 300 Adam
    steps (lr 1e-3) on the hypernetwork and the biases over 64 parameter
    samples (32 from each domain of Section 4) sharing the 65536 training
    points, then 300 steps on all of eq. 3.4 (U and V too, R_orth weight 1e-3)
    over the same samples, then the truncation of Section 4 (coefficients that f_hyper
    sets to zero at every training sample are dropped); (2) a FastLRNR
    (r_hat = 32) built from snapshots at
    f_hyper of 8 of those samples; (3) for every bounded test case of the
    reference leg, s_init = f_hyper(mu) and 200 Adam steps with the LRNR and
    with the FastLRNR gradient, the L1 relative error against the reference
    solution every 20 steps against the summed step time."""
    n_x, n_t, n_out, n_steps, every = 256, 1000, 101, 200, 20
    w = wl.equal_accuracy_case(big=False)
    net = api.DeviceNet.from_net(w.net)
    pts = api.DevicePoints.from_points(w.pts)
    cfg = api.LossCfg()
    ws = api.Workspace()
    R = w.net.r_total
    H = [3, R, R, R]
    f = api.Hyper(H, torch.tensor(wl.hyper_init(H), device="cuda"))
    mu_tr = torch.tensor(wl.cdr_test_cases(8, 32, 32).astype(np.float32), device="cuda")
    meta = api.MetaStep(f, net, mu_tr, pts)
    mt, vt = torch.zeros_like(f.theta), torch.zeros_like(f.theta)
    mb, vb = torch.zeros_like(net.b), torch.zeros_like(net.b)
    t0 = time.time()
    objs = []
    for k in range(1, 301):
        g, gb, loss, r = meta(cfg, 1.5, 1e-3, ws=ws)
        if k in (1, 300):
            objs.append(float(loss[:, 0].double().mean()) + 1e-3 * float(r[0]))
        api.adam_step(f.theta, mt, vt, g, k)
        api.adam_step(net.b, mb, vb, gb, k)
    # then all of eq. 3.4 (U and V too, with R_orth) on all 64 samples
    n_bases = 300
    meta_u = api.MetaStep(f, net, mu_tr, pts)
    params = [f.theta, net.b, net.U, net.V]
    mom = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    for k in range(1, n_bases + 1):
        g, gb, loss, r = meta_u(cfg, 1.5, 1e-3, ws=ws)
        gU, gV = api.basis_grad_batched(net, meta_u.s, mu_tr, pts, cfg, ws=ws)
        ro, gUo, gVo = api.orth_reg(net)
        if k in (1, n_bases):
            objs.append(float(loss[:, 0].double().mean()) + 1e-3 * float(r[0])
                        + 1e-3 * float(ro[0]))
        grads = (g, gb, gU + 1e-3 * gUo, gV + 1e-3 * gVo)
        for p_, (m_, v_), g_ in zip(params, mom, grads):
            api.adam_step(p_, m_, v_, g_, k)
    torch.cuda.synchronize()
    meta_s = time.time() - t0
    # truncation (Section 4): coefficients f_hyper sets to zero at every
    # training sample leave the net with their columns of U and V
    r_full = list(net.r)
    net, f, keep = api.truncate(net, f, mu_tr)
    s_snap = api.hyper_forward(f, mu_tr[::8].contiguous())
    fast = api.FastLRNR(net, s_snap, torch.tensor(w.extra["xt_snap"], device="cuda"),
                        w.extra["r_hat"])
    mus = wl.cdr_test_cases()
    u_ref, st = api.cdr_reference(torch.tensor(mus, device="cuda"), n_x, n_t, n_out)
    st = st.cpu().numpy()
    xt = torch.tensor(wl.grid_points(n_x, n_out), device="cuda")
    sums = torch.empty(2, dtype=torch.float64, device="cuda")

    def l1(s, ref):
        api.l1_error_sums(api.forward_value(net, s, xt), ref, out=sums)
        a, b = sums.cpu().numpy()
        return float(a / b)

    def train(grad_fn, s0, ref):
        s = s0.clone()
        m, v = torch.zeros_like(s), torch.zeros_like(s)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(n_steps)]
        errs = [l1(s, ref)]
        for k in range(1, n_steps + 1):
            evs[k - 1][0].record()
            api.adam_step(s, m, v, grad_fn(s), k)
            evs[k - 1][1].record()
            if k % every == 0:
                errs.append(l1(s, ref))
        torch.cuda.synchronize()
        t = np.cumsum([a.elapsed_time(b) for a, b in evs])
        return errs, [0.0] + [float(t[k - 1]) for k in range(every, n_steps + 1, every)]

    cases, warm = [], True
    for i, mu in enumerate(mus):
        if st[i]:
            continue
        mu32 = torch.tensor(mu.astype(np.float32), device="cuda")
        s0 = api.hyper_forward(f, mu32.reshape(1, 3))[0].contiguous()
        ref = u_ref[i].reshape(-1)
        lg = lambda s: api.grad_s(net, s, mu32, pts, cfg, with_b=False, ws=ws)[0]
        fg = lambda s: fast.grad_s(s, mu32, pts, cfg, ws=ws)[0]
        if warm:
            train(lg, s0, ref)
            train(fg, s0, ref)
            warm = False
        el, tl = train(lg, s0, ref)
        ef, tf = train(fg, s0, ref)
        cases.append({"mu": mu.tolist(), "l1_meta_init": el[0], "lrnr_l1": el, "lrnr_ms": tl,
                      "fastlrnr_l1": ef, "fastlrnr_ms": tf})
    fast.close()
    init = [c["l1_meta_init"] for c in cases]
    return {
        "workload": "small net 64 wide x 4 hidden, rank 8; meta phase 300 steps over 64 samples "
                    "of the Section 4 domains (Theta and b), then 300 steps over the same "
                    "samples (Theta, b, U, V), truncation; FastLRNR r_hat=32 "
                    "from 8 meta samples; 200 fine-tuning steps per bounded test case",
        "meta_objective_first": objs[0], "meta_objective_theta_b_last": objs[1],
        "meta_objective_bases_first": objs[2], "meta_objective_bases_last": objs[3],
        "meta_phase_s": meta_s,
        "ranks_before_truncation": r_full, "ranks_after_truncation": list(net.r),
        "l1_meta_init_median": float(np.median(init)),
        "l1_lrnr_final_median": float(np.median([c["lrnr_l1"][-1] for c in cases])),
        "l1_fastlrnr_final_median": float(np.median([c["fastlrnr_l1"][-1] for c in cases])),
        "lrnr_ms_200_median": float(np.median([c["lrnr_ms"][-1] for c in cases])),
        "fastlrnr_ms_200_median": float(np.median([c["fastlrnr_ms"][-1] for c in cases])),
        "cases": cases,
    }


def cpu_reference_solver(wl):
    """The oracle's reference solver on the same 20 test parameters (numpy FFT
    Strang splitting, FP64), one pass."""
    from oracle import cdr_reference as cdr
    t = time.time()
    cdr.cdr_solve_batch(wl.cdr_test_cases(), 256, 1000, 101)
    return (time.time() - t) * 1e3


def run_differentiation(args, torch, api, wl):
    """Differentiation form: 64 instances x 16384 points (own mu and points),
    FastLRNR r_hat = 32 on the small net, CDRLoss and torch.optim.Adam, 200
    steps.  CDRLoss by default runs the fused loss + gradient pass in the
    forward when a backward follows; the recompute form (loss-only forward,
    fused pass in the backward) is timed too."""
    from paper_2410_04001_amd import autograd as ag
    B, n = 64, 16384
    w = wl.instances_case(3, B, n)
    net = api.DeviceNet.from_net(w.net)
    s_init = torch.tensor(w.net.s_flat(), device="cuda")
    fast = api.FastLRNR(net, s_init.reshape(1, -1),
                        torch.tensor(w.extra["xt_snap"], device="cuda"), 32)
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda").contiguous()
    P = w.extra["pts"]
    batch = ag.CDRBatch(fast.net, dev(w.mu), dev(np.stack([p.xt_r for p in P])),
                        dev(np.stack([p.x_0 for p in P])), dev(np.stack([p.t_b for p in P])),
                        api.LossCfg())
    s = torch.nn.Parameter(s_init.repeat(B, 1).contiguous())
    opt = torch.optim.Adam([s], lr=1e-3)

    def step(recompute=None):
        opt.zero_grad(set_to_none=False)
        loss = ag.cdr_loss(s, batch, recompute)
        loss.sum().backward()
        opt.step()
        return loss

    def run(recompute):
        for _ in range(5):
            step(recompute)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(195):
            loss = step(recompute)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 195, loss

    with torch.no_grad():
        l0 = ag.cdr_loss(s, batch).detach().clone()
    ms, loss = run(None)
    s.data.copy_(s_init.repeat(B, 1))
    opt = torch.optim.Adam([s], lr=1e-3)
    ms_rec, _ = run(True)
    ms_grad = time_calls(torch, lambda: batch.loss_and_grad(s.detach()), 20, 3)
    fast.close()
    return {
        "workload": "64 instances x 16384 interior (+2048 IC, +2048 BC) points each, own mu and "
                    "points; FastLRNR r_hat=32 on the 64-wide rank-8 net; 200 Adam steps lr 1e-3",
        "ms_per_adam_step": ms,
        "pts_per_s": B * n / (ms * 1e-3),
        "ms_per_adam_step_recompute": ms_rec,
        "fused_loss_grad_ms": ms_grad,
        "fused_loss_grad_pts_per_s": B * n / (ms_grad * 1e-3),
        "loss_sum_first": float(l0.sum()), "loss_sum_last": float(loss.detach().sum()),
    }


def run_serving(args, torch, api, wl):
    """Serving form: Poisson streams of new-mu requests (N log-uniform in
    [1024, 65536], r_hat drawn from {16, 32, 48}, mu from the CDR law), each
    tuned by K = 100 Adam steps of FastLRNR sparse backprop and evaluated on
    a 256 x 100 grid, through the native continuous-batching engine."""
    from paper_2410_04001_amd import serving
    base = wl.fast_case(2, n=16)
    net = api.DeviceNet.from_net(base.net)
    s0 = torch.tensor(base.net.s_flat(), device="cuda")
    xs = torch.tensor(base.extra["xt_snap"], device="cuda")
    widths = [16, 32, 48]
    fasts = [api.FastLRNR(net, s0.reshape(1, -1), xs, rh) for rh in widths]
    srv = serving.Server([(f.net, s0) for f in fasts], K=100,
                         steps_per_launch=args.serve_steps_per_launch, max_slots=256,
                         max_inflight=2, arena_bytes=2 << 30, max_tiles=1 << 17)
    n_req = args.serve_requests
    st = wl.serving_stream(4, n_req, 1.0)
    reqs = []
    for i in range(n_req):
        pts = wl.request_points(st["pt_seed"][i], int(st["n"][i]))
        reqs.append(srv.request(i, widths.index(int(st["r_hat"][i])), st["mu"][i], pts))
    # a short unmeasured stream first (code objects, pinned pools)
    serving.replay(srv, reqs[:32], st["arrival"][:32] / 2000.0)
    rows = []
    for rate in args.serve_rates:
        done, wall = serving.replay(srv, reqs, st["arrival"] / rate)
        row = serving.latency_summary(done, wall)
        row["offered_req_per_s"] = rate
        row["tuning_pt_steps_per_s"] = row.pop("colloc_pts_per_s") * 100
        rows.append(row)
        print(f"# serving rate {rate}: p50 {row['p50_ms']:.2f} ms p99 {row['p99_ms']:.2f} ms "
              f"achieved {row['req_per_s']:.1f} req/s", file=sys.stderr, flush=True)
    stats = srv.stats()
    srv.close()
    # the same stream with another number of steps per graph launch (more:
    # fewer launches, coarser admission, since a request joins between
    # launches)
    rows_multi = []
    spl = 4 if args.serve_steps_per_launch == 1 else 1
    if args.serve_rates_multi:
        srv = serving.Server([(f.net, s0) for f in fasts], K=100, steps_per_launch=spl,
                             max_slots=256, max_inflight=2, arena_bytes=2 << 30,
                             max_tiles=1 << 17)
        reqs = [srv.request(r.id, r.model, r.mu, wl.request_points(st["pt_seed"][r.id],
                                                                   int(st["n"][r.id])))
                for r in reqs]
        serving.replay(srv, reqs[:32], st["arrival"][:32] / 2000.0)
        for rate in args.serve_rates_multi:
            done, wall = serving.replay(srv, reqs, st["arrival"] / rate)
            row = serving.latency_summary(done, wall)
            row["offered_req_per_s"] = rate
            row["tuning_pt_steps_per_s"] = row.pop("colloc_pts_per_s") * 100
            rows_multi.append(row)
            print(f"# serving ({spl} steps per launch) rate {rate}: p50 {row['p50_ms']:.2f} ms "
                  f"p99 {row['p99_ms']:.2f} ms achieved {row['req_per_s']:.1f} req/s",
                  file=sys.stderr, flush=True)
        srv.close()
    for f in fasts:
        f.close()
    mean_n = float(np.mean(st["n"]))
    return {
        "workload": f"{n_req} requests per rate; N log-uniform [1024, 65536] (mean {mean_n:.0f}), "
                    "N/8 IC and BC points; r_hat in {16, 32, 48} on the 64-wide rank-8 net; "
                    "K=100 Adam steps then a 256x100 grid evaluation",
        "steps_per_launch": args.serve_steps_per_launch,
        "rates": rows,
        "steps_per_launch_other": spl,
        "rates_other": rows_multi,
        "engine": {k: stats[k] for k in ("launches", "steps", "evals", "table_uploads",
                                          "peak_active", "arena_peak")},
    }


KERNEL_SOURCES = ("lrnr_internal.h", "lrnr_fused_impl.h", "lrnr_fused_ws.h", "lrnr_fused_rp20.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lrnr_grad_ws_N262144_w256_r20_traffic.md")


def kernel_source_sha():
    """SHA-256 over the code of the working-size gradient kernel's sources:
    lines with their // comments removed, blank lines dropped, so that an
    edit of comments alone keeps the stored counter figures valid."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2410_04001_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources changed after the counters were taken."""
    try:
        fields = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith(("#", "|", "`")):
                k, v = line.split(":", 1)
                if v.split():
                    fields[k.strip().strip("-* ")] = v.split()[0].strip("`")
        if fields.get("source_sha256") != kernel_source_sha():
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(torch):
    """A plain device copy of known size (1 GiB read, 1 GiB written) for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    a = torch.ones(2 ** 28, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 2 ** 30, "copy_bytes_written": 2 ** 30}), flush=True)


def cpu_threads():
    """Threads the host may use: the CPU share of this process (its affinity
    set), capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(w, wl, seconds=10.0):
    """The FP64 oracle on a bounded sample of the same workload, timed with
    its BLAS limited to one thread and to every thread of the CPU share."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import lrnr_oracle as orc
    n = 16384
    sub = wl.Points(w.pts.xt_r[:n], w.pts.x_0[:n // 8], w.pts.t_b[:n // 8])

    def timed(threads):
        with threadpool_limits(limits=threads):
            used = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
            t = time.time()
            reps = 0
            while True:
                orc.lrnr_loss_chunked(w.net, w.net.s, w.mu[0].astype(np.float64), sub, {},
                                      chunk=8192)
                reps += 1
                el = time.time() - t
                if el > seconds:
                    break
        return reps * n / el, reps, el, used

    n_all = cpu_threads()
    v1, reps1, el1, _ = timed(1)
    va, repsa, ela, used = timed(n_all)
    return {
        "value": va, "unit": "pts/s", "cores": int(used), "kind": "oracle",
        "value_1_thread": v1,
        "nproc": os.cpu_count(),
        "sample": f"loss+grad_s,b on the first {n} interior (+{n // 8} IC, +{n // 8} BC) points "
                  f"of the same workload, FP64 numpy: {repsa} passes in {ela:.1f} s on {used} "
                  f"threads, {reps1} in {el1:.1f} s on 1 thread",
    }


def _r(x, d=4):
    """Round a float to d significant digits for the headline."""
    if x is None or not isinstance(x, (int, float)) or isinstance(x, bool):
        return x
    if x == 0 or not math.isfinite(x):
        return x
    return float(f"{x:.{d}g}")


def headline(out, full_path):
    """The compact last line: the contract's fields, the roofline and CPU
    baseline, and one line per side leg; the full record is at full_path."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "warmup_effective",
            "ms_per_step", "ms_per_step_mean", "higher_is_better", "scaling", "vs_baseline",
            "dtype", "data", "config")
    h = {k: out[k] for k in keys if k in out}
    for k in ("value", "ms_per_step", "ms_per_step_mean"):
        h[k] = _r(h.get(k), 6)
    h["config"] = {k: v for k, v in out["config"].items()}
    rf = dict(out["roofline"])
    for k in ("achieved", "frac", "kernel_ms_avg", "kernel_ms_median", "flops_per_launch",
              "traffic"):
        rf[k] = _r(rf.get(k), 5)
    h["roofline"] = rf
    if "cpu_baseline" in out:
        cb = dict(out["cpu_baseline"])
        for k in ("value", "value_1_thread"):
            cb[k] = _r(cb.get(k), 5)
        h["cpu_baseline"] = cb
    legs = {}
    f = out.get("fastlrnr")
    if f:
        legs["fastlrnr_small_net"] = {k: _r(f[k]) for k in ("lrnr_ms", "fastlrnr_ms", "speedup")}
    ea = out.get("equal_accuracy")
    if ea:
        legs["equal_accuracy_time_ratio"] = [_r(e.get("time_ratio_lrnr_over_fast")) for e in ea]
    d = out.get("differentiation")
    if d:
        legs["differentiation"] = {k: _r(d[k]) for k in ("ms_per_adam_step",
                                                         "ms_per_adam_step_recompute",
                                                         "fused_loss_grad_ms") if k in d}
    sv = out.get("serving")
    if sv:
        legs["serving_rate_achieved_p50_p99_ms"] = [
            [_r(r["offered_req_per_s"]), _r(r["req_per_s"]), _r(r["p50_ms"]), _r(r["p99_ms"])]
            for r in sv["rates"]]
        if sv.get("rates_other"):
            legs[f"serving_{sv['steps_per_launch_other']}_steps_per_launch"] = [
                [_r(r["offered_req_per_s"]), _r(r["req_per_s"]), _r(r["p50_ms"]), _r(r["p99_ms"])]
                for r in sv["rates_other"]]
    mt = out.get("meta")
    if mt:
        legs["meta_ms_per_step"] = _r(mt["ms_per_meta_step"])
        wb = mt.get("with_bases_64_samples")
        if wb:
            legs["meta_with_bases_ms_per_step"] = _r(wb["ms_per_meta_step"])
            legs["basis_grad_ms_per_sample"] = _r(wb["basis_grad_ms_per_sample_batched"])
    h["legs"] = legs
    h["full_record"] = full_path
    return h


def write_full(out, path):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    with open(path, "w") as fh:
        json.dump(out, fh)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fast", action="store_true")
    ap.add_argument("--no-equal-acc", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fidelity", action="store_true")
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--no-bias", action="store_true")
    ap.add_argument("--no-meta", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--no-per-mu", action="store_true",
                    help="skip the step timing at each of the 8 parameter draws")
    ap.add_argument("--serve-rates", type=lambda x: [float(v) for v in x.split(",")],
                    default=[50, 100, 200, 500, 1000, 2000])
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-steps-per-launch", type=int, default=2,
                    help="Adam steps per graph launch of the serving engine (the stream is "
                         "replayed again at --serve-rates-multi with one step per launch, or "
                         "four when this is one)")
    ap.add_argument("--serve-rates-multi", type=lambda x: [float(v) for v in x.split(",") if v],
                    default=[500, 1000],
                    help="rates replayed again with one step per launch (four when the main run "
                         "uses one)")
    ap.add_argument("--out", default="bench_full.json",
                    help="file for the full record of every leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the loss+gradient would shard over points with one small all-reduce; see the "
              "design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as wl
    from paper_2410_04001_amd import api

    torch.cuda.init()
    if args.copy_calibration:
        copy_calibration(torch)
        return
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
        "warmup_effective": r["warmup_effective"],
        "ms_per_step": r["ms_per_step"],
        "ms_per_step_mean": r["ms_per_step_mean"],
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
            "traffic": measured_traffic(),
            "kernel": "lrnr_grad_ws_kernel<20, 2> (+ relaunch of flagged tiles)",
            "kernel_ms_avg": r["kernel_ms_avg"],
            "kernel_ms_median": r["kernel_ms_median"],
            "flops_per_launch": r["flops_per_launch"],
        },
    }
    progress("lrnr", f"{r['ms_per_step']:.4f} ms/step (median), kernel {r['kernel_ms_avg']:.4f} ms, "
             f"frac {out['roofline']['frac']:.3f}")
    out["per_mu"] = r["per_mu"]
    if fast is not None:
        out["fastlrnr"] = fast
        progress("fastlrnr", f"LRNR {fast['lrnr_ms']:.4f} ms, FastLRNR {fast['fastlrnr_ms']:.4f} ms")
    legs = [
        ("factored_bias", args.no_bias, lambda: run_factored_bias(args, torch, api, wl)),
        ("fidelity", args.no_fidelity, lambda: run_fidelity(args, torch, api, wl)),
        ("equal_accuracy", args.no_equal_acc,
         lambda: [run_equal_accuracy(args, torch, api, wl, big) for big in (False, True)]),
        ("reference", args.no_reference,
         lambda: [run_reference(args, torch, api, wl, big) for big in (False, True)]),
        ("meta", args.no_meta, lambda: run_meta(args, torch, api, wl)),
        ("pipeline", args.no_pipeline, lambda: run_pipeline(args, torch, api, wl)),
        ("differentiation", args.no_diff, lambda: run_differentiation(args, torch, api, wl)),
        ("serving", args.no_serve, lambda: run_serving(args, torch, api, wl)),
    ]
    for name, skip, fn in legs:
        if skip:
            continue
        t = time.time()
        out[name] = fn()
        progress(name, f"done in {time.time() - t:.1f} s")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(r["w"], wl)
        progress("cpu_baseline", f"{out['cpu_baseline']['value']:.4g} pts/s on "
                 f"{out['cpu_baseline']['cores']} threads, "
                 f"{out['cpu_baseline']['value_1_thread']:.4g} on 1")
        if "reference" in out:
            out["reference"][0]["reference"]["cpu_oracle_ms"] = cpu_reference_solver(wl)
    write_full(out, args.out)
    print(json.dumps(headline(out, args.out)), flush=True)


def progress(leg, msg):
    print(f"# {leg}: {msg}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
