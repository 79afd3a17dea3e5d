"""Differentiation form: the torch.autograd.Function wrappers (CDRLoss,
LRNRJets) against the FP64 oracle gradients and against central finite
differences (h = 1e-3) of the functions' own forward values; and the
many-instance training run (64 instances of 16384 points, FastLRNR r_hat = 32
on the 64-wide net, 200 Adam steps, lr 1e-3).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import assert_close, log, s_blocks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "the gpu tests need the MI355X"
    from paper_2410_04001_amd import _clib
    _clib.lib()


def mods():
    from paper_2410_04001_amd import api, autograd
    return api, autograd


def dev(x):
    return torch.tensor(np.asarray(x, np.float32), device="cuda").contiguous()


def batch_case(B=4, n=2048, seed=3):
    w = wl.instances_case(seed, B, n)
    api, ag = mods()
    net = api.DeviceNet.from_net(w.net)
    pts = w.extra["pts"]
    xt = dev(np.stack([p.xt_r for p in pts]))
    x0 = dev(np.stack([p.x_0 for p in pts]))
    tb = dev(np.stack([p.t_b for p in pts]))
    batch = ag.CDRBatch(net, dev(w.mu), xt, x0, tb, api.LossCfg())
    s0 = np.tile(w.net.s_flat(), (B, 1)).astype(np.float32)
    # distinct coefficients per instance
    s0 *= (1.0 + 0.05 * np.arange(B, dtype=np.float32))[:, None]
    return w, net, batch, s0


def test_cdr_loss_backward_matches_oracle():
    api, ag = mods()
    w, net, batch, s0 = batch_case()
    B = s0.shape[0]
    log(f"[case] CDRLoss B={B} n=2048 per instance, small net")
    s = dev(s0).requires_grad_(True)
    gout = torch.linspace(0.5, 2.0, B, device="cuda")
    loss = ag.cdr_loss(s, batch)
    (loss * gout).sum().backward()
    torch.cuda.synchronize()
    g = s.grad.cpu().numpy()
    lv = loss.detach().cpu().numpy()
    for i in range(B):
        l4, rgs, _ = orc.lrnr_loss(w.net, w.net.split_s(s0[i]), w.mu[i].astype(np.float64),
                                   w.extra["pts"][i], {}, with_grad=True)
        assert_close(lv[i:i + 1], l4[:1], TOL, f"instance {i} loss")
        assert_close(g[i], float(gout[i]) * rgs, TOL, f"instance {i} d(gout*loss)/ds",
                     blocks=s_blocks(w.net))


def test_cdr_loss_recompute_equals_fused_and_fd():
    api, ag = mods()
    w, net, batch, s0 = batch_case(B=3, n=1024, seed=5)
    grads = []
    for rec in (True, False):
        s = dev(s0).requires_grad_(True)
        ag.cdr_loss(s, batch, recompute=rec).sum().backward()
        torch.cuda.synchronize()
        grads.append(s.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1]), "recompute-in-backward != fused forward gradient"
    # central differences of the function's own (FP32) forward, h = 1e-3,
    # along random directions per instance
    g = grads[0]
    rng = np.random.default_rng(7)
    h = 1e-3
    for trial in range(3):
        d = rng.standard_normal(s0.shape).astype(np.float32)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        with torch.no_grad():
            lp = ag.cdr_loss(dev(s0 + h * d), batch).double().cpu().numpy()
            lm = ag.cdr_loss(dev(s0 - h * d), batch).double().cpu().numpy()
        # the perturbation actually applied after FP32 rounding of s0 +- h d
        dp = (np.float32(s0 + h * d).astype(np.float64) - np.float32(s0 - h * d)) / 2
        fd = (lp - lm) / 2
        an = np.sum(g.astype(np.float64) * dp, axis=1)
        e = np.abs(fd - an) / np.maximum(np.abs(an), 1e-3 * np.abs(lp))
        log(f"  direction {trial}: FD {fd} analytic {an} rel diff {e}")
        assert np.all(e < 2e-2), e


def test_lrnr_jets_backward_matches_oracle_vjp_and_fd():
    api, ag = mods()
    w = wl.small_lrnr(0, 16)
    net = api.DeviceNet.from_net(w.net)
    B, n = 3, 1500
    rng = np.random.Generator(np.random.PCG64(9))
    xt_h = np.stack([wl.uniform_points(rng, n) for _ in range(B)])
    jb = ag.JetsBatch(net, dev(xt_h))
    s0 = np.tile(w.net.s_flat(), (B, 1)) * (1 + 0.1 * np.arange(B))[:, None]
    s0 = s0.astype(np.float32)
    C = rng.standard_normal((B, 4, n)).astype(np.float32)
    log(f"[case] LRNRJets B={B} n={n}, random cotangent")
    s = dev(s0).requires_grad_(True)
    jets = ag.lrnr_jets(s, jb)
    (jets * dev(C)).sum().backward()
    torch.cuda.synchronize()
    g = s.grad.cpu().numpy()
    for i in range(B):
        rgs, _ = orc.lrnr_jets_vjp(w.net, w.net.split_s(s0[i]), xt_h[i].astype(np.float64),
                                   C[i].astype(np.float64))
        assert_close(g[i], rgs, TOL, f"instance {i} jets VJP", blocks=s_blocks(w.net))
        rj = orc.lrnr_forward_jets(w.net, w.net.split_s(s0[i]), xt_h[i].astype(np.float64))
        assert_close(jets[i, 0].detach().cpu().numpy(), rj[0], TOL, f"instance {i} u")
    # FD along one direction
    d = np.random.default_rng(3).standard_normal(s0.shape).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = 1e-3
    with torch.no_grad():
        fp = (ag.lrnr_jets(dev(s0 + h * d), jb).double() * dev(C).double()).sum((1, 2))
        fm = (ag.lrnr_jets(dev(s0 - h * d), jb).double() * dev(C).double()).sum((1, 2))
    dp = (np.float32(s0 + h * d).astype(np.float64) - np.float32(s0 - h * d)) / 2
    fd = ((fp - fm) / 2).cpu().numpy()
    an = np.sum(g.astype(np.float64) * dp, axis=1)
    e = np.abs(fd - an) / np.abs(an)
    log(f"  FD {fd} analytic {an} rel diff {e}")
    assert np.all(e < 2e-2), e


def test_many_instance_adam_run_fastlrnr():
    """64 instances x 16384 points (own mu and points each), FastLRNR r_hat =
    32 built on the device from the 64-wide net, 200 Adam steps (lr 1e-3)
    through CDRLoss + torch.optim.Adam.  Checks: the summed loss decreases;
    at the final coefficients, sampled instances' loss and gradient match the
    oracle's FastLRNR chain on the device's reduced operators."""
    api, ag = mods()
    B, n = 64, 16384
    w = wl.instances_case(3, B, n)
    net = api.DeviceNet.from_net(w.net)
    s_init = dev(w.net.s_flat())
    fast = api.FastLRNR(net, s_init.reshape(1, -1), dev(w.extra["xt_snap"]), 32)
    ops = fast.operators()
    pts = w.extra["pts"]
    xt = dev(np.stack([p.xt_r for p in pts]))
    x0 = dev(np.stack([p.x_0 for p in pts]))
    tb = dev(np.stack([p.t_b for p in pts]))
    batch = ag.CDRBatch(fast.net, dev(w.mu), xt, x0, tb, api.LossCfg())
    s = torch.nn.Parameter(s_init.repeat(B, 1).contiguous())
    opt = torch.optim.Adam([s], lr=1e-3)
    log(f"[case] {B} instances x {n} points, FastLRNR r_hat=32, 200 Adam steps")
    first = None
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for step in range(200):
        opt.zero_grad(set_to_none=False)
        loss = ag.cdr_loss(s, batch)
        loss.sum().backward()
        opt.step()
        if first is None:
            first = loss.detach().clone()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    with torch.no_grad():
        final = ag.cdr_loss(s, batch)
    torch.cuda.synchronize()
    f0, f1 = first.cpu().numpy(), final.cpu().numpy()
    log(f"  200 steps in {ms:.1f} ms ({ms / 200:.3f} ms/step incl. torch Adam); "
        f"sum loss {f0.sum():.4f} -> {f1.sum():.4f}; "
        f"instances improved {(f1 < f0).sum()}/{B}")
    assert f1.sum() < f0.sum()
    assert (f1 < f0).sum() >= B * 3 // 4
    # oracle at the final coefficients for a few instances
    s_fin = s.detach().cpu().numpy()
    loss4, grad = batch.loss_and_grad(s.detach())
    torch.cuda.synchronize()
    loss4, grad = loss4.cpu().numpy(), grad.cpu().numpy()
    for i in (0, 17, 63):
        l4, rgs = orc.fast_loss(w.net, ops, w.net.split_s(s_fin[i]),
                                w.mu[i].astype(np.float64), pts[i], {}, with_grad=True)
        assert_close(loss4[i], l4, TOL, f"instance {i} final loss")
        assert_close(grad[i], rgs, TOL, f"instance {i} final grad_s")
    fast.close()
