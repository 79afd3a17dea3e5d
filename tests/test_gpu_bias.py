"""GPU parity of factored biases b^l = B^l s_b^l (lrnr_bias_compose,
lrnr_bias_grad, fastlrnr_bias_basis) against the FP64 oracle, through the
C ABI.  Bar: loss, grad_s and grad_sb within 1e-4 relative (2-norm and
max-norm, as the other parity tests); the composed biases and the chain-rule
product within 1e-6 (FP64 sums rounded once to FP32); the reduced basis
bitwise (a row gather)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import LOSS_BLOCKS, assert_close, fp32, log, s_blocks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "the gpu tests need the MI355X"
    from paper_2410_04001_amd import _clib
    _clib.lib()


def api():
    from paper_2410_04001_amd import api as a
    return a


def basis(net, q, seed=5, zero_layer=None):
    """B^l [M_l][q_l] with q_l = min(q, M_l) (0 for zero_layer), s_b^l ~ U(-1, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B, sb = [], []
    for l, m in enumerate(net.M[1:], start=1):
        ql = 0 if l == zero_layer else min(q, m)
        B.append((rng.standard_normal((m, ql)) / math.sqrt(m)).astype(np.float32))
        sb.append(rng.uniform(-1, 1, ql).astype(np.float32))
    return B, sb


def dev_basis(a, net, B):
    flat = np.concatenate([b.reshape(-1) for b in B]) if B else np.zeros(0, np.float32)
    return a.BiasBasis(net.M, [b.shape[1] for b in B], flat if flat.size else np.zeros(1, np.float32))


def to_dev(w):
    a = api()
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    pts = a.DevicePoints.from_points(w.pts)
    mu = torch.tensor(w.mu[0], device="cuda")
    return net, s, pts, mu


CASES = [("small", lambda: wl.fast_case(2, n=8192), 8, None),
         ("small_zero_layer", lambda: wl.fast_case(2, n=4096), 6, 2),
         ("wide", lambda: wl.big_lrnr(1, 8192), 16, None),
         ("wide_q32", lambda: wl.big_lrnr(1, 2048), 32, None)]


@pytest.mark.parametrize("name,make,q,zero", CASES, ids=[c[0] for c in CASES])
def test_lrnr_factored_bias_matches_oracle(name, make, q, zero):
    a = api()
    w = make()
    B, sb = basis(w.net, q, zero_layer=zero)
    log(f"[case] factored bias {name}: M={w.net.M} r={w.net.r} q={[b.shape[1] for b in B]}")
    net, s, pts, mu = to_dev(w)
    bb = dev_basis(a, w.net, B)
    s_b = torch.tensor(np.concatenate(sb), device="cuda")
    b = a.bias_compose(bb, s_b)
    gs, gsb, loss = a.grad_s_factored(net, bb, s, s_b, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    b_ref = np.concatenate(orc.bias_from_basis(B, sb))
    np.testing.assert_allclose(b.cpu().numpy(), b_ref, rtol=1e-6, atol=1e-7)
    l4, rgs, rgsb = orc.lrnr_loss_factored_bias(w.net, w.net.s, B, sb,
                                                w.mu[0].astype(np.float64), w.pts, {}, True)
    f32 = fp32(lambda: orc.lrnr_loss_factored_bias(w.net, w.net.s, B, sb, w.mu[0], w.pts, {},
                                                   True))
    assert_close(loss.cpu().numpy(), l4, TOL, f"{name} loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, f"{name} grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    assert_close(gsb.cpu().numpy(), rgsb, TOL, f"{name} grad_sb", blocks=[b.shape[1] for b in B],
                 floor=lambda: f32()[2])


def test_bias_grad_is_the_transposed_basis_product():
    a = api()
    w = wl.fast_case(2, n=1024)
    B, _ = basis(w.net, 12, seed=7)
    bb = dev_basis(a, w.net, B)
    rng = np.random.Generator(np.random.PCG64(3))
    g = rng.standard_normal(sum(w.net.M[1:])).astype(np.float32)
    log("[case] bias grad B^T g")
    out = a.bias_grad(bb, torch.tensor(g, device="cuda")).cpu().numpy()
    ref, o = [], 0
    for Bl in B:
        ref.append(Bl.astype(np.float64).T @ g[o:o + Bl.shape[0]].astype(np.float64))
        o += Bl.shape[0]
    np.testing.assert_allclose(out, np.concatenate(ref), rtol=1e-6, atol=1e-7)


def test_fastlrnr_factored_bias_matches_oracle():
    a = api()
    w = wl.fast_case(2, n=8192)
    xs = w.extra["xt_snap"]
    B, sb = basis(w.net, 8, seed=9)
    log("[case] FastLRNR r_hat=8 with factored biases")
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, s.reshape(1, -1), torch.tensor(xs, device="cuda"), 8)
    bb = dev_basis(a, w.net, B)
    red = fast.bias_basis(bb)
    P = fast.indices()
    # the reduced basis is the rows of B at P (hidden layers), B^L as it is
    Bh = red.B.cpu().numpy()
    o = 0
    for l, Bl in enumerate(B):
        rows = Bl[P[l]] if l < len(P) else Bl
        n = rows.size
        assert np.array_equal(Bh[o:o + n], rows.reshape(-1)), l
        o += n
    s_b = torch.tensor(np.concatenate(sb), device="cuda")
    gs, gsb, loss = a.grad_s_factored(fast.net, red, s, s_b, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    ops = fast.operators()
    ops["P"] = P
    l4, rgs, rgsb = orc.fast_loss_factored_bias(w.net, ops, w.net.s, B, sb,
                                                w.mu[0].astype(np.float64), w.pts, {}, True)
    f32 = fp32(lambda: orc.fast_loss_factored_bias(w.net, ops, w.net.s, B, sb, w.mu[0], w.pts,
                                                   {}, True))
    assert_close(loss.cpu().numpy(), l4, TOL, "fast factored loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, "fast factored grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    assert_close(gsb.cpu().numpy(), rgsb, TOL, "fast factored grad_sb",
                 blocks=[b.shape[1] for b in B])
    fast.close()


def test_bias_basis_argument_checks():
    a = api()
    from paper_2410_04001_amd import _clib as cl
    w = wl.fast_case(2, n=1024)
    B, _ = basis(w.net, 4)
    bb = dev_basis(a, w.net, B)
    s_b = torch.zeros(bb.q_total, device="cuda")
    bad = dev_basis(a, w.net, B)
    bad._c.q[1] = 33                                  # above LRNR_MAX_RANK
    with pytest.raises(RuntimeError):
        a.bias_compose(bad, s_b)
    bad = dev_basis(a, w.net, B)
    bad._c.L = 0
    with pytest.raises(RuntimeError):
        a.bias_grad(bad, torch.zeros(bb.b_total, device="cuda"))
    out = torch.empty(bb.b_total, device="cuda")
    assert cl.lib().lrnr_bias_compose(bb.c(), None, out.data_ptr(), None) == cl.EINVAL
    # a basis of another depth does not fit a FastLRNR
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, s.reshape(1, -1), torch.tensor(w.extra["xt_snap"], device="cuda"), 8)
    short = a.BiasBasis(w.net.M[:-1], [b.shape[1] for b in B[:-1]],
                        np.concatenate([b.reshape(-1) for b in B[:-1]]))
    with pytest.raises(RuntimeError):
        fast.bias_basis(short)
    fast.close()
