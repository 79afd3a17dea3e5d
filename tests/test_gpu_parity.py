"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded FP32 inputs.

Bar: loss, grad_s, grad_b and the u, u_x, u_t jets within 1e-4 relative, the
u_xx jet within 1e-3, as relative errors in the 2-norm and in the max-norm
(tests/_util.assert_close).
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import LOSS_BLOCKS, assert_close, b_blocks, fp32, log, s_blocks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-4
TOL_XX = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "the gpu tests need the MI355X"
    from paper_2410_04001_amd import _clib
    _clib.lib()


def api():
    from paper_2410_04001_amd import api as a
    return a


def to_dev(w, mu_row=0):
    a = api()
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    pts = a.DevicePoints.from_points(w.pts)
    mu = torch.tensor(np.asarray(w.mu[mu_row], np.float32), device="cuda")
    return net, s, pts, mu


def cfg_dict(form=0, w_r=1.0, w_0=1.0, w_b=1.0, lam=0.0, sref=None):
    return {"form": form, "w_r": w_r, "w_0": w_0, "w_b": w_b, "lambda_loc": lam, "s_ref": sref}


def gpu_cfg(d):
    a = api()
    sref = None if d["s_ref"] is None else torch.tensor(np.asarray(d["s_ref"], np.float32),
                                                         device="cuda")
    return a.LossCfg(d["form"], d["w_r"], d["w_0"], d["w_b"], d["lambda_loc"], sref)


def check_loss_grad(w, mu_row=0, cfg=None, with_b=True, tag=""):
    a = api()
    cfg = cfg or cfg_dict()
    log(f"[case] {tag} M={w.net.M} r={w.net.r} n=({len(w.pts.xt_r)},{len(w.pts.x_0)},"
        f"{len(w.pts.t_b)}) mu={w.mu[mu_row]} form={cfg['form']}")
    net, s, pts, mu = to_dev(w, mu_row)
    gc = gpu_cfg(cfg)
    gs, gb, loss = a.grad_s(net, s, mu, pts, gc, with_b=with_b)
    loss_only = a.residual_loss(net, s, mu, pts, gc)
    torch.cuda.synchronize()
    ref_cfg = dict(cfg)
    if ref_cfg["s_ref"] is not None:
        ref_cfg["s_ref"] = np.asarray(ref_cfg["s_ref"], np.float32).astype(np.float64)
    l4, rgs, rgb = orc.lrnr_loss(w.net, w.net.s, w.mu[mu_row].astype(np.float64), w.pts,
                                 ref_cfg, with_grad=True)
    f32 = fp32(lambda: orc.lrnr_loss(w.net, w.net.s, w.mu[mu_row], w.pts, ref_cfg,
                                     with_grad=True))
    assert_close(loss.cpu().numpy(), l4, TOL, f"{tag} loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(loss_only.cpu().numpy(), l4, TOL, f"{tag} loss (loss-only entry)",
                 blocks=LOSS_BLOCKS, floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, f"{tag} grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    if with_b:
        assert_close(gb.cpu().numpy(), rgb, TOL, f"{tag} grad_b", blocks=b_blocks(w.net),
                     floor=lambda: f32()[2])
    return gs, gb, loss


def check_jets(w, xt=None, tag=""):
    a = api()
    xt = w.pts.xt_r if xt is None else xt
    log(f"[case] jets {tag} M={w.net.M} r={w.net.r} n={len(xt)}")
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    xtd = torch.tensor(xt, device="cuda")
    jets = a.forward_jets(net, s, xtd).cpu().numpy()
    val = a.forward_value(net, s, xtd).cpu().numpy()
    ref = orc.lrnr_forward_jets(w.net, w.net.s, xt)
    for c, name, tol in ((0, "u", TOL), (1, "u_x", TOL), (2, "u_t", TOL), (3, "u_xx", TOL_XX)):
        assert_close(jets[c], ref[c], tol, f"{tag} {name}")
    assert_close(val, ref[0], TOL, f"{tag} value-only u")
    return jets


def custom(seed, M, rank, n_r, n_0, n_b, mu=(3.0, 0.7, 1.3)):
    rng = np.random.Generator(np.random.PCG64(seed))
    M = list(M)
    r = wl.ranks(M, rank) if np.isscalar(rank) else list(rank)
    net = wl.make_net(rng, M, r)
    pts = wl.make_points(rng, n_r, n_0, n_b)
    return wl.Workload(net, pts, np.array([mu], np.float32))


# --------------------------------------------------------------- LRNR -------

def test_forward_jets_small_lrnr():
    check_jets(wl.small_lrnr(0), tag="small")


def test_loss_grad_small_lrnr_convection():
    check_loss_grad(wl.small_lrnr(0), tag="small beta=10")


def test_loss_grad_small_net_full_cdr_params():
    w = wl.small_lrnr(0)
    w.mu = wl.make_mu(np.random.default_rng(9), 3)
    for i in range(3):
        check_loss_grad(w, mu_row=i, cfg=cfg_dict(w_r=1.0, w_0=2.0, w_b=0.5), tag=f"small cdr{i}")


def test_l1_form_and_locality_term():
    w = wl.small_lrnr(0, 2048)
    w.mu = np.array([[7.0, 0.3, 0.8]], np.float32)
    sref = w.net.s_flat() + np.float32(0.05) * np.sin(np.arange(w.net.r_total, dtype=np.float32))
    check_loss_grad(w, cfg=cfg_dict(form=1, lam=0.01, sref=sref), tag="l1+loc")


# width 64 at rank tile 8 runs the single-role kernel for the gradient, width
# 128 at rank tile 16 the four-role kernel
NETS = pytest.mark.parametrize("width,rank", [(64, 8), (128, 16)])


@NETS
@pytest.mark.parametrize("n_r,n_0,n_b", [(1, 1, 1), (63, 0, 0), (65, 77, 33), (300, 1, 129),
                                         (0, 50, 0), (0, 0, 40), (257, 256, 128),
                                         (130, 600, 300), (0, 1025, 385)])
def test_ragged_and_empty_point_sets(n_r, n_0, n_b, width, rank):
    w = custom(21, (2, width, width, width, 1), rank, n_r, n_0, n_b)
    check_loss_grad(w, tag=f"ragged {n_r},{n_0},{n_b} width {width} rank {rank}")


@NETS
def test_ragged_value_tiles_beyond_the_cus(width, rank):
    """151 IC and 121 BC tiles (272 > 256 CUs); in the four-role kernel the
    IC/BC workgroups take two tiles each, with a trailing workgroup that has
    one."""
    w = custom(23, (2, width, width, width, 1), rank, 130, 151 * 256 - 179, 121 * 128 - 95)
    check_loss_grad(w, tag=f"value tiles beyond the CUs, width {width} rank {rank}")


def test_all_sets_empty_gives_zero():
    a = api()
    w = custom(22, (2, 32, 32, 1), 8, 0, 0, 0)
    net, s, pts, mu = to_dev(w)
    gs, gb, loss = a.grad_s(net, s, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    assert np.all(loss.cpu().numpy() == 0) and np.all(gs.cpu().numpy() == 0)
    assert np.all(gb.cpu().numpy() == 0)
    empty = torch.empty((0, 2), device="cuda")
    assert a.forward_jets(net, s, empty).shape == (4, 0)


@pytest.mark.parametrize("M,rank", [
    ((2, 40, 1), 3),                        # one hidden layer, rank tile 4
    ((2, 37, 50, 1), 13),                   # widths not a multiple of 4, tile 16
    ((2, 100, 90, 80, 1), (2, 24, 17, 1)),  # mixed ranks, tile 24
    ((2, 64, 64, 64, 1), 32),               # tile 32
    ((2, 48, 48, 48, 48, 48, 48, 48, 1), 5),  # depth 8, tile 8 (all layers resident in LDS)
    ((2, 160, 160, 160, 1), 8),             # tile 8 too wide for resident layers
    ((2, 256, 256, 1), 20),                 # widest, tile 20
    ((2, 256, 256, 256, 1), 32),            # compiled maxima: width 256, tile 32
])
def test_net_shapes(M, rank):
    w = custom(31, M, rank, 700, 90, 70, mu=(11.0, 2.0, 3.5))
    check_jets(w, tag=f"shape {M}")
    check_loss_grad(w, tag=f"shape {M}")


@NETS
def test_large_preactivations_take_the_accurate_path(width, rank):
    """Four neurons of layer 1 get zero U-rows and bias 2^25, so their
    pre-activation is exactly 2^25 at every point (and the oracle exact).  The
    fast sin/cos reduction is not valid there (its quadrant index passes
    2^24); parity holds only if the accurate path is taken."""
    w = custom(51, (2, width, width, width, 1), rank, 600, 70, 70)
    w.net.U[0][:4, :] = 0.0
    w.net.b[0][:4] = np.float32(2.0 ** 25)
    check_jets(w, tag="large |a|")
    check_loss_grad(w, tag="large |a|")


def test_nan_point_stays_local():
    """A NaN input makes the running |a| maximum of its wave NaN (IEEE
    maximum propagates it), which fails the range test, so that wave takes
    the accurate sin/cos path.  The NaN point's jets are NaN; every other
    point's jets, including its wave neighbours on the accurate path, match
    the oracle."""
    a = api()
    w = wl.small_lrnr(0, 300)
    xt = w.pts.xt_r[:300].copy()
    xt[77, 0] = np.nan
    log("[case] jets with one NaN point (index 77 of 300)")
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    jets = a.forward_jets(net, s, torch.tensor(xt, device="cuda")).cpu().numpy()
    assert np.all(np.isnan(jets[:, 77]))
    ok = np.ones(len(xt), bool)
    ok[77] = False
    assert np.all(np.isfinite(jets[:, ok]))
    ref = orc.lrnr_forward_jets(w.net, w.net.s, xt[ok])
    for c, name, tol in ((0, "u", TOL), (1, "u_x", TOL), (2, "u_t", TOL), (3, "u_xx", TOL_XX)):
        assert_close(jets[c][ok], ref[c], tol, f"NaN neighbours {name}")


def test_big_net_reduced_points():
    w = wl.big_lrnr(1, 2048)
    check_jets(w, tag="big 2048")
    for i in (0, 3):
        check_loss_grad(w, mu_row=i, tag=f"big 2048 mu{i}")


def test_big_net_full_size():
    """Working size (N = 262144, the benchmarked launch): forward jets on a
    sample of points against the oracle, and the gradient by additivity over
    8 disjoint point blocks, one of which is checked against the oracle."""
    a = api()
    w = wl.big_lrnr(1)
    log("[case] big full size N=262144")
    net, s, pts, mu = to_dev(w, 0)
    gc = a.LossCfg()
    gs, gb, loss = a.grad_s(net, s, mu, pts, gc)
    torch.cuda.synchronize()
    # sampled jets at the working size
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(len(w.pts.xt_r), 2048, replace=False))
    jets = a.forward_jets(net, s, pts.xt_r).cpu().numpy()[:, idx]
    ref = orc.lrnr_forward_jets(w.net, w.net.s, w.pts.xt_r[idx])
    for c, tol in ((0, TOL), (1, TOL), (2, TOL), (3, TOL_XX)):
        assert_close(jets[c], ref[c], tol, f"full-size jets[{c}]")
    # additivity: each block with weights scaled by its share of the points
    n_r, n_0, n_b = pts.counts
    K = 8
    acc_s = np.zeros(net.r_total)
    acc_b = np.zeros(net.b_total)
    acc_l = np.zeros(4)
    for k in range(K):
        sl = lambda n: slice(k * n // K, (k + 1) * n // K)
        sub = wl.Points(w.pts.xt_r[sl(n_r)], w.pts.x_0[sl(n_0)], w.pts.t_b[sl(n_b)])
        dsub = a.DevicePoints.from_points(sub)
        c = cfg_dict(w_r=len(sub.xt_r) / n_r, w_0=len(sub.x_0) / n_0, w_b=len(sub.t_b) / n_b)
        g1, b1, l1 = a.grad_s(net, s, mu, dsub, gpu_cfg(c))
        acc_s += g1.cpu().numpy()
        acc_b += b1.cpu().numpy()
        acc_l += l1.cpu().numpy()
        if k == 3:
            l4, rgs, rgb = orc.lrnr_loss_chunked(w.net, w.net.s, w.mu[0].astype(np.float64), sub, c)
            f32 = fp32(lambda: orc.lrnr_loss_chunked(w.net, w.net.s, w.mu[0], sub, c))
            assert_close(l1.cpu().numpy(), l4, TOL, "block loss", blocks=LOSS_BLOCKS,
                         floor=lambda: f32()[0])
            assert_close(g1.cpu().numpy(), rgs, TOL, "block grad_s", blocks=s_blocks(w.net),
                         floor=lambda: f32()[1])
            assert_close(b1.cpu().numpy(), rgb, TOL, "block grad_b", blocks=b_blocks(w.net),
                         floor=lambda: f32()[2])
    assert_close(gs.cpu().numpy(), acc_s, 1e-5, "full grad_s vs sum of blocks")
    assert_close(gb.cpu().numpy(), acc_b, 1e-5, "full grad_b vs sum of blocks")
    assert_close(loss.cpu().numpy(), acc_l, 1e-5, "full loss vs sum of blocks")


@NETS
def test_determinism_bitwise(width, rank):
    a = api()
    w = custom(24, (2, width, width, width, width, 1), rank, 4096, 512, 512)
    net, s, pts, mu = to_dev(w)
    outs = [a.grad_s(net, s, mu, pts, a.LossCfg()) for _ in range(3)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert torch.equal(x, y)


@NETS
@pytest.mark.parametrize("n_r", [1000, 30000])
def test_batched_equals_single_bitwise(width, rank, n_r):
    """With 30,000 points the five-instance launch has 815 workgroups (more
    than two per CU: the three-wave fast pass and relaunch at rank tile 8)
    while each single-instance launch has 163 (two waves, redo in place)."""
    a = api()
    w = custom(25, (2, width, width, width, width, 1), rank, n_r, n_r // 8, n_r // 8)
    net, s, pts, _ = to_dev(w)
    rng = np.random.default_rng(4)
    B = 5
    S = torch.tensor(np.stack([w.net.s_flat() * rng.uniform(0.8, 1.2, w.net.r_total).astype(np.float32)
                               for _ in range(B)]), device="cuda")
    MU = torch.tensor(wl.make_mu(rng, B), device="cuda")
    gsb, lb = a.grad_s_batched(net, S, MU, pts, a.LossCfg())
    for i in range(B):
        gs, _, loss = a.grad_s(net, S[i].contiguous(), MU[i].contiguous(), pts, a.LossCfg(),
                               with_b=False)
        assert torch.equal(gs, gsb[i]) and torch.equal(loss, lb[i])
    # and one instance against the oracle
    s_list = w.net.split_s(S[2].cpu().numpy())
    l4, rgs, _ = orc.lrnr_loss(w.net, s_list, MU[2].cpu().numpy().astype(np.float64), w.pts, {},
                               with_grad=True)
    mu2 = MU[2].cpu().numpy()
    f32 = fp32(lambda: orc.lrnr_loss(w.net, s_list, mu2, w.pts, {}, with_grad=True))
    assert_close(gsb[2].cpu().numpy(), rgs, TOL, "batched grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    assert_close(lb[2].cpu().numpy(), l4, TOL, "batched loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])


def test_adam_step_matches_oracle():
    a = api()
    rng = np.random.default_rng(5)
    n = 1000
    s0, g0 = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    s = torch.tensor(s0, device="cuda")
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    g = torch.tensor(g0, device="cuda")
    rs, rm, rv = s0.astype(np.float64), np.zeros(n), np.zeros(n)
    for k in range(1, 4):
        a.adam_step(s, m, v, g, k)
        rs, rm, rv = orc.adam_step(rs, g0, rm, rv, k)
    torch.cuda.synchronize()
    assert_close(s.cpu().numpy(), rs, 1e-6, "adam s")


# ----------------------------------------------------------- FastLRNR -------

def resolved_modes(net, xt_snap, thresh=1e-8):
    """Per hidden layer, the number of snapshot singular values above thresh
    times the largest (FP64): the POD modes that rounding does not blur."""
    out = []
    for z in orc.lrnr_hidden_values(net, net.s, xt_snap):
        sv = np.linalg.svd(z.T, compute_uv=False)
        out.append(int(np.sum(sv >= thresh * sv[0])))
    return out


def test_fastlrnr_build_matches_oracle_at_resolved_rank():
    """r_hat = 8 lies inside the resolved snapshot spectrum of every layer, so
    the device construction (FP64 snapshots, Jacobi SVD, DEIM) must pick the
    oracle's indices and reproduce its FastLRNR loss and gradient."""
    a = api()
    w = wl.fast_case(2, n=8192)
    xs = w.extra["xt_snap"]
    k = resolved_modes(w.net, xs)
    log(f"[case] fastlrnr r_hat=8, resolved modes per layer {k}")
    assert min(k) >= 8
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, s.reshape(1, -1), torch.tensor(xs, device="cuda"), 8)
    P = fast.indices()
    ref = orc.fastlrnr_build(w.net, [w.net.s], xs, 8)
    for p, q in zip(P, ref["P"]):
        assert np.array_equal(p, q), (p, q)
    gs, loss = fast.grad_s(s, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    l4, rgs = orc.fast_loss(w.net, ref, w.net.s, w.mu[0].astype(np.float64), w.pts, {},
                            with_grad=True)
    f32 = fp32(lambda: orc.fast_loss(w.net, ref, w.net.s, w.mu[0], w.pts, {}, with_grad=True))
    assert_close(loss.cpu().numpy(), l4, TOL, "fast r8 loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, "fast r8 grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    jets = a.forward_jets(fast.net, s, pts.xt_r[:512].contiguous()).cpu().numpy()
    rj = orc.fast_forward_jets(w.net, ref, w.net.s, w.pts.xt_r[:512])
    for c, tol in ((0, TOL), (1, TOL), (2, TOL), (3, TOL_XX)):
        assert_close(jets[c], rj[c], tol, f"fast r8 jets[{c}]")
    fast.close()


def test_fastlrnr_build_from_perturbed_snapshots_matches_oracle():
    """Snapshots at s and at 3 perturbed copies of s (the fidelity sweep's
    second set): at r_hat = 8 the device picks the oracle's indices on the
    resolved spectrum of the joint snapshot matrix, and the FastLRNR loss and
    gradient match the oracle's eq. 2.8 chain on the device's operators."""
    a = api()
    w = wl.fast_case(2, n=8192)
    xs = w.extra["xt_snap"]
    rng = np.random.Generator(np.random.PCG64(9))
    s0 = w.net.s_flat()
    snaps = [s0] + [(s0 * (1.0 + 0.1 * rng.standard_normal(s0.shape))).astype(np.float32)
                    for _ in range(3)]
    s_lists = [w.net.split_s(v) for v in snaps]
    Z = [np.concatenate(zs, axis=0) for zs in
         zip(*[orc.lrnr_hidden_values(w.net, sl, xs) for sl in s_lists])]
    k = []
    for z in Z:
        sv = np.linalg.svd(z.T, compute_uv=False)
        k.append(int(np.sum(sv >= 1e-8 * sv[0])))
    log(f"[case] fastlrnr r_hat=8 from 4 snapshot sets, resolved modes per layer {k}")
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, torch.tensor(np.stack(snaps), device="cuda"),
                      torch.tensor(xs, device="cuda"), 8)
    P = fast.indices()
    ref = orc.fastlrnr_build(w.net, s_lists, xs, 8)
    for p, q, kl in zip(P, ref["P"], k):
        n_eq = int(np.argmin(np.append(p == q, False)))
        assert n_eq >= min(kl, 8), (n_eq, kl, p, q)
    ops = fast.operators()
    gs, loss = fast.grad_s(s, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    l4, rgs = orc.fast_loss(w.net, ops, w.net.s, w.mu[0].astype(np.float64), w.pts, {},
                            with_grad=True)
    f32 = fp32(lambda: orc.fast_loss(w.net, ops, w.net.s, w.mu[0], w.pts, {}, with_grad=True))
    assert_close(loss.cpu().numpy(), l4, TOL, "fast r8 (4 snapshot sets) loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, "fast r8 (4 snapshot sets) grad_s",
                 blocks=s_blocks(w.net), floor=lambda: f32()[1])
    fast.close()


@pytest.mark.parametrize("n_sets", [1, 4])
def test_fastlrnr_qdeim_matches_oracle(n_sets):
    """Q-DEIM selection (fastlrnr_build_sel) at r_hat = 8, from snapshots at
    s alone and at s plus 3 perturbed copies: the device picks the oracle's
    indices on the resolved spectrum, and the FastLRNR loss and gradient
    match the oracle's eq. 2.8 chain on the device's operators."""
    a = api()
    w = wl.fast_case(2, n=8192)
    xs = w.extra["xt_snap"]
    rng = np.random.Generator(np.random.PCG64(9))
    s0 = w.net.s_flat()
    snaps = [s0] + [(s0 * (1.0 + 0.1 * rng.standard_normal(s0.shape))).astype(np.float32)
                    for _ in range(n_sets - 1)]
    s_lists = [w.net.split_s(v) for v in snaps]
    Z = [np.concatenate(zs, axis=0) for zs in
         zip(*[orc.lrnr_hidden_values(w.net, sl, xs) for sl in s_lists])]
    k = []
    for z in Z:
        sv = np.linalg.svd(z.T, compute_uv=False)
        k.append(int(np.sum(sv >= 1e-8 * sv[0])))
    log(f"[case] fastlrnr Q-DEIM r_hat=8, {n_sets} snapshot sets, resolved modes {k}")
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, torch.tensor(np.stack(snaps), device="cuda"),
                      torch.tensor(xs, device="cuda"), 8, selection="qdeim")
    P = fast.indices()
    ref = orc.fastlrnr_build(w.net, s_lists, xs, 8, selection="qdeim")
    for p, q, kl in zip(P, ref["P"], k):
        n_eq = int(np.argmin(np.append(p == q, False)))
        assert n_eq >= min(kl, 8), (n_eq, kl, p, q)
        assert len(set(p.tolist())) == 8
    ops = fast.operators()
    gs, loss = fast.grad_s(s, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    l4, rgs = orc.fast_loss(w.net, ops, w.net.s, w.mu[0].astype(np.float64), w.pts, {},
                            with_grad=True)
    f32 = fp32(lambda: orc.fast_loss(w.net, ops, w.net.s, w.mu[0], w.pts, {}, with_grad=True))
    assert_close(loss.cpu().numpy(), l4, TOL, "fast Q-DEIM r8 loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, "fast Q-DEIM r8 grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    fast.close()


@pytest.mark.parametrize("which", ["small", "wide"])
def test_fastlrnr_r32_prefix_operators_and_chain(which):
    """r_hat = 32 on the 64-wide rank-8 net, and on the 256-wide rank-20 net
    (reduced widths 32 at rank tile 20: the four-role kernel), runs past the
    resolved snapshot spectrum, where POD modes are rounding noise in any
    precision and later DEIM picks are arbitrary.  Checked: the picks on the
    resolved prefix equal the oracle's; U_hat = P^T U and b_hat = P^T b
    exactly; the EIM reduction reproduces the projected snapshot states
    V^{(l+1)T} z^l; and the device FastLRNR loss and gradient equal the
    oracle's eq. 2.8 chain run on the device's own reduced operators."""
    a = api()
    if which == "small":
        w = wl.fast_case(2, n=8192)
    else:
        w = wl.equal_accuracy_case(big=True, n=8192)
    xs = w.extra["xt_snap"]
    k = resolved_modes(w.net, xs)
    log(f"[case] fastlrnr {which} r_hat=32, resolved modes per layer {k}")
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, s.reshape(1, -1), torch.tensor(xs, device="cuda"), 32)
    P = fast.indices()
    ref = orc.fastlrnr_build(w.net, [w.net.s], xs, 32)
    agree = []
    for p, q, kl in zip(P, ref["P"], k):
        n_eq = int(np.argmin(np.append(p == q, False)))
        agree.append(n_eq)
        assert n_eq >= min(kl, 32), (n_eq, kl, p, q)
        assert len(set(p.tolist())) == 32 and p.min() >= 0 and p.max() < max(w.net.M)
    log(f"  picks equal to the oracle's: {agree} (resolved prefix {k})")
    ops = fast.operators()
    Z = orc.lrnr_hidden_values(w.net, w.net.s, xs)
    for l, p in enumerate(P):
        assert np.array_equal(ops["U_hat"][l], w.net.U[l][p]), l
        assert np.array_equal(ops["b_hat"][l], w.net.b[l][p]), l
        proj = Z[l] @ w.net.V[l + 1].astype(np.float64)          # V^{(l+1)T} z
        red = Z[l][:, p] @ ops["V_hat"][l].astype(np.float64)    # V_hat^T P^T z
        e = np.linalg.norm(red - proj) / np.linalg.norm(proj)
        log(f"  layer {l + 1}: EIM reduced state vs projected state rel err {e:.2e}")
        assert e < 1e-4, (l, e)
    gs, loss = fast.grad_s(s, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    l4, rgs = orc.fast_loss(w.net, ops, w.net.s, w.mu[0].astype(np.float64), w.pts, {},
                            with_grad=True)
    f32 = fp32(lambda: orc.fast_loss(w.net, ops, w.net.s, w.mu[0], w.pts, {}, with_grad=True))
    assert_close(loss.cpu().numpy(), l4, TOL, f"fast {which} r32 loss (device operators)",
                 blocks=LOSS_BLOCKS, floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, f"fast {which} r32 grad_s (device operators)",
                 blocks=s_blocks(w.net), floor=lambda: f32()[1])
    fast.close()


def test_fastlrnr_full_index_set_equals_lrnr():
    a = api()
    w = custom(41, (2, 32, 32, 32, 1), 8, 2000, 200, 200)
    log("[case] fastlrnr full index set r_hat=M=32")
    net, s, pts, mu = to_dev(w)
    xt_snap = torch.tensor(wl.uniform_points(np.random.default_rng(3), 256), device="cuda")
    fast = a.FastLRNR(net, s.reshape(1, -1), xt_snap, [32, 32, 32])
    for p in fast.indices():
        assert sorted(p.tolist()) == list(range(32))
    gf, lf = fast.grad_s(s, mu, pts, a.LossCfg())
    gl, _, ll = a.grad_s(net, s, mu, pts, a.LossCfg(), with_b=False)
    torch.cuda.synchronize()
    assert_close(gf.cpu().numpy(), gl.cpu().numpy(), TOL, "full-set fast vs lrnr grad_s",
                 blocks=s_blocks(w.net))
    assert_close(lf.cpu().numpy(), ll.cpu().numpy(), TOL, "full-set fast vs lrnr loss")
    fast.close()


@pytest.mark.parametrize("which,r_hat", [("small", 4), ("wide", 5)])
def test_fastlrnr_reduced_width_below_rank(which, r_hat):
    """The paper's own regime (Section 2.2 eq. 2.6-2.8, Section 4): reduced
    widths r_hat_l below the ranks r_l, so U_hat^l = P^T U^l is r_hat x r and
    V_hat^{l+1} is r_hat x r_{l+1}.  At r_hat = 4 on the rank-8 net and
    r_hat = 5 on the rank-20 working-size net (both inside the resolved
    snapshot spectrum) the device picks the oracle's indices, and the FastLRNR
    loss, gradient and jets match the oracle's eq. 2.8 chain."""
    a = api()
    if which == "small":
        w = wl.fast_case(2, n=8192)
        xs = w.extra["xt_snap"]
    else:
        w = wl.big_lrnr(1, 8192)
        xs = wl.uniform_points(np.random.Generator(np.random.PCG64(2)), 2048)
    k = resolved_modes(w.net, xs)
    log(f"[case] fastlrnr {which} r_hat={r_hat} < r={max(w.net.r)}, resolved modes {k}")
    assert min(k) >= r_hat
    net, s, pts, mu = to_dev(w)
    fast = a.FastLRNR(net, s.reshape(1, -1), torch.tensor(xs, device="cuda"), r_hat)
    P = fast.indices()
    ref = orc.fastlrnr_build(w.net, [w.net.s], xs, r_hat)
    for p, q in zip(P, ref["P"]):
        assert np.array_equal(p, q), (p, q)
    ops = fast.operators()
    for l in range(len(P)):
        assert ops["U_hat"][l].shape == (r_hat, w.net.r[l])
        assert ops["V_hat"][l].shape == (r_hat, w.net.r[l + 1])
    gs, loss = fast.grad_s(s, mu, pts, a.LossCfg())
    torch.cuda.synchronize()
    l4, rgs = orc.fast_loss(w.net, ref, w.net.s, w.mu[0].astype(np.float64), w.pts, {},
                            with_grad=True)
    tag = f"fast {which} r_hat={r_hat}"
    f32 = fp32(lambda: orc.fast_loss(w.net, ref, w.net.s, w.mu[0], w.pts, {}, with_grad=True))
    assert_close(loss.cpu().numpy(), l4, TOL, f"{tag} loss", blocks=LOSS_BLOCKS,
                 floor=lambda: f32()[0])
    assert_close(gs.cpu().numpy(), rgs, TOL, f"{tag} grad_s", blocks=s_blocks(w.net),
                 floor=lambda: f32()[1])
    jets = a.forward_jets(fast.net, s, pts.xt_r[:512].contiguous()).cpu().numpy()
    rj = orc.fast_forward_jets(w.net, ref, w.net.s, w.pts.xt_r[:512])
    for c, tol in ((0, TOL), (1, TOL), (2, TOL), (3, TOL_XX)):
        assert_close(jets[c], rj[c], tol, f"{tag} jets[{c}]")
    fast.close()
