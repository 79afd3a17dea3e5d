"""GPU parity of the meta-learning kernels (lrnr_hyper_forward,
lrnr_hyper_backward, and the meta gradient built from them and the batched
loss gradient) against the FP64 oracle.  Bar: 1e-4 relative in the 2-norm
and the max-norm (the bar of the loss and s-gradients; the Theta gradient is
a linear image of the s-gradients)."""
import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import assert_close, b_blocks, log, u_blocks, v_blocks

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


def setup(make, B, seed=3):
    a = api()
    w = make()
    R = w.net.r_total
    H = [3, R, R, R]
    theta = wl.hyper_init(H)
    rng = np.random.Generator(np.random.PCG64(seed))
    mus = wl.make_mu(rng, B)
    f = a.Hyper(H, torch.tensor(theta, device="cuda"))
    return a, w, H, theta, mus, f


NETS = [("small", lambda: wl.small_lrnr(0, 2048)), ("wide", lambda: wl.big_lrnr(1, 2048))]


@pytest.mark.parametrize("name,make", NETS, ids=[n for n, _ in NETS])
def test_hyper_forward_backward_match_oracle(name, make):
    a, w, H, theta, mus, f = setup(make, 37)
    log(f"[case] hypernetwork {name}: H={H} B=37")
    mu_d = torch.tensor(mus, device="cuda")
    s = a.hyper_forward(f, mu_d)
    rs, cache = orc.hyper_forward(H, theta, mus.astype(np.float64))
    assert_close(s.cpu().numpy(), rs, TOL, f"{name} s")
    rng = np.random.Generator(np.random.PCG64(8))
    s_bar = rng.standard_normal(rs.shape).astype(np.float32)
    net = a.DeviceNet.from_net(w.net)
    g, r = a.hyper_backward(f, net, mu_d, torch.tensor(s_bar, device="cuda"), 1.5, 0.3)
    g2, _ = a.hyper_backward(f, net, mu_d, torch.tensor(s_bar, device="cuda"), 1.5, 0.3)
    torch.cuda.synchronize()
    B = len(mus)
    sb_ref = s_bar / B + 0.3 * orc.sparse_reg_grad(rs, w.net.r, 1.5) / B
    assert_close(g.cpu().numpy(), orc.hyper_backward(H, cache, sb_ref), TOL, f"{name} grad theta")
    r_ref = orc.sparse_reg_value(rs, w.net.r, 1.5)
    assert abs(float(r[0]) - r_ref) <= TOL * max(1.0, abs(r_ref)), (float(r[0]), r_ref)
    assert torch.equal(g, g2)                      # fixed order: bitwise repeatable


def test_meta_gradient_matches_oracle():
    a, w, H, theta, mus, f = setup(lambda: wl.small_lrnr(0, 2048), 4)
    log("[case] meta gradient, small net, B=4, N=2048")
    net = a.DeviceNet.from_net(w.net)
    pts = a.DevicePoints.from_points(w.pts)
    g, loss, r = a.meta_grad(f, net, torch.tensor(mus, device="cuda"), pts, a.LossCfg(), 1.5, 0.3)
    torch.cuda.synchronize()
    obj, rg = orc.meta_objective(w.net, H, theta.astype(np.float64), mus.astype(np.float64),
                                 w.pts, 1.5, 0.3, {}, with_grad=True)
    got = float(loss[:, 0].double().mean()) + 0.3 * float(r[0])
    assert abs(got - obj) <= TOL * abs(obj), (got, obj)
    assert_close(g.cpu().numpy(), rg, TOL, "meta grad theta")


def test_hyper_argument_checks():
    a, w, H, theta, mus, f = setup(lambda: wl.small_lrnr(0, 256), 2)
    from paper_2410_04001_amd import _clib as cl
    net = a.DeviceNet.from_net(w.net)
    mu_d = torch.tensor(mus, device="cuda")
    bad = a.Hyper([2] + H[1:], f.theta)            # H[0] must be 3
    with pytest.raises(RuntimeError):
        a.hyper_forward(bad, mu_d)
    short = a.Hyper(H[:-1] + [H[-1] - 1], f.theta)  # output is not r_total
    with pytest.raises(RuntimeError):
        a.hyper_backward(short, net, mu_d, torch.zeros((2, H[-1] - 1), device="cuda"), 1.5, 0.1)
    g = torch.empty_like(f.theta)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    rc = cl.lib().lrnr_hyper_backward(f.c(), net.c(), 0, mu_d.data_ptr(), mu_d.data_ptr(),
                                      1.5, 0.1, g.data_ptr(), None, ws.data_ptr(), ws.numel(), None)
    assert rc == cl.EINVAL                          # no samples
    s_bar = torch.zeros((2, H[-1]), device="cuda")
    rc = cl.lib().lrnr_hyper_backward(f.c(), net.c(), 2, mu_d.data_ptr(), s_bar.data_ptr(),
                                      1.5, 0.1, g.data_ptr(), None, ws.data_ptr(), 64, None)
    assert rc == cl.ENOMEM                          # workspace too small
    assert cl.lib().lrnr_hyper_workspace_size(f.c(), 0) == 0
    empty = a.hyper_forward(f, torch.zeros((0, 3), device="cuda"))
    assert empty.shape == (0, H[-1])


@pytest.mark.parametrize("H_mid", [[], [256], [256, 256, 64]], ids=["K1", "wide256", "K4"])
def test_hyper_depths_and_maximum_width(H_mid):
    # one layer (linear + ReLU), the maximum width 256, and a deeper map
    a = api()
    w = wl.big_lrnr(1, 256)
    R = w.net.r_total
    H = [3] + H_mid + [R]
    theta = wl.hyper_init(H, seed=11)
    rng = np.random.Generator(np.random.PCG64(12))
    mus = wl.make_mu(rng, 9)
    log(f"[case] hypernetwork H={H} B=9")
    f = a.Hyper(H, torch.tensor(theta, device="cuda"))
    mu_d = torch.tensor(mus, device="cuda")
    s = a.hyper_forward(f, mu_d)
    rs, cache = orc.hyper_forward(H, theta, mus.astype(np.float64))
    assert_close(s.cpu().numpy(), rs, TOL, f"H={H} s")
    s_bar = rng.standard_normal(rs.shape).astype(np.float32)
    net = a.DeviceNet.from_net(w.net)
    g, r = a.hyper_backward(f, net, mu_d, torch.tensor(s_bar, device="cuda"), 2.0, 0.5)
    sb_ref = s_bar / 9 + 0.5 * orc.sparse_reg_grad(rs, w.net.r, 2.0) / 9
    assert_close(g.cpu().numpy(), orc.hyper_backward(H, cache, sb_ref), TOL, f"H={H} grad theta")


def test_meta_step_with_biases_matches_oracle():
    # Theta and bias gradients through a task table of GRAD tasks
    a, w, H, theta, mus, f = setup(lambda: wl.small_lrnr(0, 2048), 5)
    log("[case] meta step with biases, small net, B=5, N=2048")
    net = a.DeviceNet.from_net(w.net)
    pts = a.DevicePoints.from_points(w.pts)
    step = a.MetaStep(f, net, torch.tensor(mus, device="cuda"), pts)
    g, gb, loss, r = step(a.LossCfg(), 1.5, 0.3)
    torch.cuda.synchronize()
    obj, rg, rgb = orc.meta_objective(w.net, H, theta.astype(np.float64), mus.astype(np.float64),
                                      w.pts, 1.5, 0.3, {}, with_grad=True, with_b=True)
    got = float(loss[:, 0].double().mean()) + 0.3 * float(r[0])
    assert abs(got - obj) <= TOL * abs(obj), (got, obj)
    assert_close(g.cpu().numpy(), rg, TOL, "meta step grad theta")
    assert_close(gb.cpu().numpy(), rgb, TOL, "meta step grad b", blocks=b_blocks(w.net))
    # the mean over samples is a fixed-order sum
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.standard_normal((37, 1001)).astype(np.float32)
    m1 = a.rows_mean(torch.tensor(x, device="cuda"))
    m2 = a.rows_mean(torch.tensor(x, device="cuda"))
    assert torch.equal(m1, m2)
    np.testing.assert_allclose(m1.cpu().numpy(), x.astype(np.float64).mean(axis=0),
                               rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("name,make", NETS, ids=[n for n, _ in NETS])
def test_orth_reg_matches_oracle(name, make):
    import copy
    a = api()
    w = make()
    rng = np.random.Generator(np.random.PCG64(13))
    n2 = copy.copy(w.net)          # bases pulled off orthonormality
    n2.U = [(u * (1 + 0.2 * rng.standard_normal(u.shape))).astype(np.float32) for u in w.net.U]
    n2.V = [(v * (1 + 0.2 * rng.standard_normal(v.shape))).astype(np.float32) for v in w.net.V]
    log(f"[case] R_orth {name}")
    v, gU, gV = a.orth_reg(a.DeviceNet.from_net(n2))
    rv, rgU, rgV = orc.orth_reg(n2.U, n2.V, with_grad=True)
    assert abs(float(v[0]) - rv) <= TOL * rv, (float(v[0]), rv)
    assert_close(gU.cpu().numpy(), np.concatenate([g.ravel() for g in rgU]), TOL, f"{name} grad U",
                 blocks=u_blocks(n2))
    assert_close(gV.cpu().numpy(), np.concatenate([g.ravel() for g in rgV]), TOL, f"{name} grad V",
                 blocks=v_blocks(n2))
    # the generated bases are orthonormal up to FP32 rounding
    v0, _, _ = a.orth_reg(a.DeviceNet.from_net(w.net), with_grad=False)
    assert float(v0[0]) < 1e-9


def rank16_case():
    # ranks in (8, 16]: the middle rank tile of the per-point kernels
    rng = np.random.Generator(np.random.PCG64(17))
    M = [2, 96, 80, 1]
    net = wl.make_net(rng, M, wl.ranks(M, 13))
    return wl.Workload(net, wl.make_points(rng, 700, 90, 70), wl.make_mu(rng, 1))


@pytest.mark.parametrize("name,make,form", [("small", lambda: wl.small_lrnr(0, 2048), 0),
                                            ("small_l1", lambda: wl.small_lrnr(0, 1500), 1),
                                            ("rank13", rank16_case, 0),
                                            ("wide", lambda: wl.big_lrnr(1, 512), 0)],
                         ids=["small", "small_l1", "rank13", "wide"])
def test_basis_grad_matches_oracle(name, make, form):
    a = api()
    w = make()
    log(f"[case] basis gradient {name}: M={w.net.M} r={w.net.r} form={form}")
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    pts = a.DevicePoints.from_points(w.pts)
    mu = torch.tensor(w.mu[0], device="cuda")
    cfg = a.LossCfg(form=form, w_0=0.7, w_b=1.3)
    gU, gV = a.basis_grad(net, s, mu, pts, cfg)
    gU2, gV2 = a.basis_grad(net, s, mu, pts, cfg)
    torch.cuda.synchronize()
    rU, rV = orc.lrnr_basis_grad(w.net, w.net.s, w.mu[0].astype(np.float64), w.pts,
                                 {"form": form, "w_r": 1.0, "w_0": 0.7, "w_b": 1.3})
    assert_close(gU.cpu().numpy(), rU, TOL, f"{name} grad U", blocks=u_blocks(w.net))
    assert_close(gV.cpu().numpy(), rV, TOL, f"{name} grad V", blocks=v_blocks(w.net))
    assert torch.equal(gU, gU2) and torch.equal(gV, gV2)


@pytest.mark.parametrize("name,make", [("small", lambda: wl.small_lrnr(0, 3000)),
                                       ("rank13", rank16_case)], ids=["small", "rank13"])
def test_basis_grad_batched_is_the_mean_over_samples(name, make):
    """lrnr_basis_grad_batched over B = 5 samples (own s and mu, shared
    points) against the mean of the oracle's per-sample gradients, and its
    B = 1 case bitwise equal to lrnr_basis_grad."""
    a = api()
    w = make()
    rng = np.random.Generator(np.random.PCG64(23))
    B = 5
    s0 = w.net.s_flat()
    S = np.stack([(s0 * rng.uniform(0.5, 1.5, s0.shape)).astype(np.float32) for _ in range(B)])
    mus = wl.make_mu(rng, B)
    log(f"[case] batched basis gradient {name}: M={w.net.M} r={w.net.r} B={B}")
    net = a.DeviceNet.from_net(w.net)
    pts = a.DevicePoints.from_points(w.pts)
    cfg = a.LossCfg()
    Sd, Md = torch.tensor(S, device="cuda"), torch.tensor(mus, device="cuda")
    gU, gV = a.basis_grad_batched(net, Sd, Md, pts, cfg)
    g1U, g1V = a.basis_grad_batched(net, Sd[:1].contiguous(), Md[:1].contiguous(), pts, cfg)
    h1U, h1V = a.basis_grad(net, Sd[0].contiguous(), Md[0].contiguous(), pts, cfg)
    torch.cuda.synchronize()
    assert torch.equal(g1U, h1U) and torch.equal(g1V, h1V)
    rU, rV = 0.0, 0.0
    for b in range(B):
        u, v = orc.lrnr_basis_grad(w.net, w.net.split_s(S[b]), mus[b].astype(np.float64), w.pts,
                                   {})
        rU, rV = rU + u / B, rV + v / B
    assert_close(gU.cpu().numpy(), rU, TOL, f"{name} mean grad U", blocks=u_blocks(w.net))
    assert_close(gV.cpu().numpy(), rV, TOL, f"{name} mean grad V", blocks=v_blocks(w.net))


def _trunc_theta(w, H, dead_idx, seed=7):
    """A hypernetwork whose last layer sends the outputs dead_idx to a
    pre-activation of -5 at every mu (zero row of W_K, c_K = -5) and keeps
    the others at least 2 (decisions far from the ReLU's kink)."""
    theta = wl.hyper_init(H, seed=seed).astype(np.float64)
    layers = orc.hyper_unpack(H, theta)
    WK, cK = layers[-1]
    dead = np.zeros(H[-1], bool)
    dead[dead_idx] = True
    WK[dead, :] = 0.0
    cK[dead] = -5.0
    cK[~dead] = np.abs(cK[~dead]) + 2.0
    return np.concatenate([np.concatenate([W.ravel(), c]) for W, c in layers]).astype(np.float32)


TRUNC = [("small", lambda: wl.small_lrnr(0, 2048), [3, 5, 6, 9, 10, 11, 12, 13, 14, 15, 16, 17]),
         ("wide", lambda: wl.big_lrnr(1, 2048), list(range(2, 22, 3)) + list(range(22, 42)))]


@pytest.mark.parametrize("name,make,dead", TRUNC, ids=[c[0] for c in TRUNC])
def test_truncate_matches_oracle(name, make, dead):
    """Truncation after meta-learning (lrnr_truncate): the kept set and ranks
    equal the oracle's, the truncated U, V and Theta are the oracle's gathers
    bitwise, and the truncated net at f'(mu) reproduces the full net's loss
    and kept s-gradients (the dropped coefficients are zero)."""
    a = api()
    w = make()
    R = w.net.r_total
    H = [3, 16, 16, R]
    theta = _trunc_theta(w, H, dead)
    mus = wl.make_mu(np.random.Generator(np.random.PCG64(11)), 6)
    f = a.Hyper(H, torch.tensor(theta, device="cuda"))
    net = a.DeviceNet.from_net(w.net)
    mu_d = torch.tensor(mus, device="cuda")
    tnet, tf, keep = a.truncate(net, f, mu_d)
    torch.cuda.synchronize()
    ref = orc.truncate(w.net, H, theta.astype(np.float64), mus.astype(np.float64))
    log(f"[case] truncate {name}: r {w.net.r} -> {tnet.r} (oracle {ref['r']})")
    assert tnet.r == ref["r"] and np.array_equal(keep, ref["keep"])
    assert tf.H == ref["H"]
    assert np.array_equal(tnet.U.cpu().numpy(), np.concatenate([u.ravel() for u in ref["U"]]))
    assert np.array_equal(tnet.V.cpu().numpy(), np.concatenate([v.ravel() for v in ref["V"]]))
    assert np.array_equal(tf.theta.cpu().numpy(), ref["theta"].astype(np.float32))
    # the truncated net and map against the full ones, through the device path
    pts = a.DevicePoints.from_points(w.pts)
    s_full = a.hyper_forward(f, mu_d)
    s_tr = a.hyper_forward(tf, mu_d)
    torch.cuda.synchronize()
    assert torch.equal(s_tr, s_full[:, torch.tensor(keep, device="cuda")])
    for b in (0, 5):
        gs, _, loss = a.grad_s(tnet, s_tr[b].contiguous(), mu_d[b].contiguous(), pts, a.LossCfg(),
                               with_b=False)
        torch.cuda.synchronize()
        sf = w.net.split_s(s_full[b].cpu().numpy())
        lf, gf, _ = orc.lrnr_loss(w.net, sf, mus[b].astype(np.float64), w.pts, {},
                                  with_grad=True)
        assert_close(loss.cpu().numpy(), lf, TOL, f"truncated {name} loss (mu {b})")
        assert_close(gs.cpu().numpy(), gf[keep], TOL, f"truncated {name} kept grad_s (mu {b})")
