"""lrnr_grad_s_noalloc (the workspace-free variant of lrnr_grad_s for callers
that cannot allocate) through the C ABI: two calls in a row, the second on a
smaller input, each bitwise equal to lrnr_grad_s on the same inputs with a
caller workspace (same kernels, same order of operations), and within the
parity bar of the FP64 oracle; sizes beyond the fixed scratch are refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import assert_close, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "the gpu tests need the MI355X"
    from paper_2410_04001_amd import _clib
    _clib.lib()


def _run_noalloc(a, cl, net, s, mu, pts, cfg):
    gs = torch.full((net.r_total,), float("nan"), device="cuda")
    gb = torch.full((net.b_total,), float("nan"), device="cuda")
    loss = torch.full((4,), float("nan"), device="cuda")
    rc = cl.lib().lrnr_grad_s_noalloc(net.c(), a._p(s), a._p(mu), pts.c(), cfg.c(), a._p(gs),
                                      a._p(gb), a._p(loss), a._stream())
    cl.check(rc, "lrnr_grad_s_noalloc")
    return gs, gb, loss


def test_noalloc_matches_grad_s_on_two_calls_the_second_smaller():
    from paper_2410_04001_amd import _clib as cl
    from paper_2410_04001_amd import api as a
    cases = [("wide 256x5 rank 20, N=8192", wl.big_lrnr(1, 8192)),
             ("small 64x4 rank 8, N=1000", wl.small_lrnr(0, 1000))]
    for tag, w in cases:
        log(f"[case] noalloc {tag}")
        net = a.DeviceNet.from_net(w.net)
        s = torch.tensor(w.net.s_flat(), device="cuda")
        pts = a.DevicePoints.from_points(w.pts)
        mu = torch.tensor(w.mu[0], device="cuda")
        cfg = a.LossCfg()
        gs_n, gb_n, loss_n = _run_noalloc(a, cl, net, s, mu, pts, cfg)
        gs, gb, loss = a.grad_s(net, s, mu, pts, cfg)
        torch.cuda.synchronize()
        for x, y, name in ((gs_n, gs, "grad_s"), (gb_n, gb, "grad_b"), (loss_n, loss, "loss")):
            assert torch.equal(x, y), (tag, name, (x - y).abs().max().item())
        l4, rgs, rgb = orc.lrnr_loss(w.net, w.net.s, w.mu[0].astype(np.float64), w.pts, {},
                                     with_grad=True)
        assert_close(loss_n.cpu().numpy(), l4, 1e-4, f"noalloc {tag} loss")
        assert_close(gs_n.cpu().numpy(), rgs, 1e-4, f"noalloc {tag} grad_s")
        assert_close(gb_n.cpu().numpy(), rgb, 1e-4, f"noalloc {tag} grad_b")


def test_noalloc_refuses_sizes_beyond_the_scratch():
    from paper_2410_04001_amd import _clib as cl
    from paper_2410_04001_amd import api as a
    w = wl.small_lrnr(0, 16)
    net = a.DeviceNet.from_net(w.net)
    n = 1 << 20     # about 700 MB of workspace; the points are never read
    big = cl.LrnrPoints(16, n, 16, n // 8, 16, n // 8)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    out = torch.zeros(max(w.net.r_total, 4), device="cuda")
    rc = cl.lib().lrnr_grad_s_noalloc(net.c(), a._p(s), a._p(s), C.byref(big), a.LossCfg().c(),
                                      a._p(out), None, None, a._stream())
    assert rc == cl.EUNSUPPORTED, rc
