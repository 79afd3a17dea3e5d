"""Task tables (lrnr_tasks_run): many instances with their own nets, s, mu,
points and outputs in one persistent launch.

Checked: every mode against the FP64 oracle (tolerances of test_gpu_parity);
a task's results are bitwise identical alone and inside any mix of other
tasks (different nets, sizes and positions); results agree with the
single-instance entry points; ragged, empty and many-task tables.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import LOSS_BLOCKS, assert_close, b_blocks, log, s_blocks, fp32

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


def dev(x):
    return torch.tensor(np.asarray(x, np.float32), device="cuda").contiguous()


class Inst:
    """One instance: host data for the oracle and device copies for the tasks."""

    def __init__(self, net_id, net, seed, n_r, n_0, n_b, s_scale=1.0):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.net_id, self.net = net_id, net
        self.pts = wl.make_points(rng, n_r, n_0, n_b)
        self.mu = wl.make_mu(rng, 1)[0]
        self.s_host = (net.s_flat() * np.float32(s_scale)).astype(np.float32)
        self.s = dev(self.s_host)
        self.mu_d = dev(self.mu)
        self.xt = dev(self.pts.xt_r.reshape(-1, 2))
        self.x0 = dev(self.pts.x_0)
        self.tb = dev(self.pts.t_b)
        rt, bt = net.r_total, sum(net.M[1:])
        self.gs = torch.full((rt,), np.nan, device="cuda")
        self.gb = torch.full((bt,), np.nan, device="cuda")
        self.loss = torch.full((4,), np.nan, device="cuda")
        self.jets = torch.full((4, n_r), np.nan, device="cuda")
        self.val = torch.full((n_r,), np.nan, device="cuda")
        self.cot_host = rng.standard_normal((4, n_r)).astype(np.float32)
        self.cot = dev(self.cot_host)

    def s_list(self):
        return self.net.split_s(self.s_host)

    def add(self, tab):
        tab.add(self.net_id, s=self.s, mu=self.mu_d, xt_r=self.xt, x_0=self.x0, t_b=self.tb,
                grad_s=self.gs, grad_b=self.gb, loss=self.loss, out=None, cot=self.cot)

    def outputs(self):
        return [x.detach().cpu().numpy().copy() for x in (self.gs, self.gb, self.loss)]


def nets(kind="narrow"):
    """Two nets per table.  narrow: widest layer 64 at rank tile 8 (the
    reverse modes run the single-role kernel); wide: widest layer 128 at rank
    tile 16 (the four-role kernel)."""
    rng = np.random.Generator(np.random.PCG64(21))
    if kind == "narrow":
        n0 = wl.small_lrnr(0, 16).net                               # (2,64,64,64,64,1), r 8
        M, rank = [2, 48, 40, 1], 8
    else:
        M0 = [2, 128, 128, 128, 1]
        n0 = wl.make_net(rng, M0, wl.ranks(M0, 16))
        M, rank = [2, 120, 100, 1], 13
    n1 = wl.make_net(rng, M, wl.ranks(M, rank))                     # other widths, depth
    return [n0, n1]


KINDS = pytest.mark.parametrize("kind", ["narrow", "wide"])


def run(mode, dnets, insts, cfg=None, out_attr=None):
    a = api()
    tab = a.TaskTable(dnets)
    for it in insts:
        if out_attr is None:
            it.add(tab)
        else:
            tab.add(it.net_id, s=it.s, xt_r=it.xt, out=getattr(it, out_attr),
                    cot=it.cot, grad_s=it.gs, grad_b=it.gb)
    tab.run(mode, cfg)
    torch.cuda.synchronize()


@KINDS
def test_tasks_grad_loss_vs_oracle_and_single_path(kind):
    a = api()
    hn = nets(kind)
    dn = [a.DeviceNet.from_net(n) for n in hn]
    shapes = [(0, 4096, 512, 512), (1, 1000, 77, 33), (0, 300, 0, 129), (1, 257, 256, 128)]
    insts = [Inst(sh[0], hn[sh[0]], 100 + i, *sh[1:]) for i, sh in enumerate(shapes)]
    cfg = a.LossCfg()
    log(f"[case] task table GRAD ({kind} nets), {len(insts)} tasks, shapes {shapes}")
    run(a.MODE_GRAD, dn, insts, cfg)
    for i, it in enumerate(insts):
        gs, gb, loss = it.outputs()
        l4, rgs, rgb = orc.lrnr_loss(it.net, it.s_list(), it.mu.astype(np.float64), it.pts, {},
                                     with_grad=True)
        f32 = fp32(lambda: orc.lrnr_loss(it.net, it.s_list(), it.mu, it.pts, {}, with_grad=True))
        assert_close(loss, l4, TOL, f"task {i} loss", blocks=LOSS_BLOCKS, floor=lambda: f32()[0])
        assert_close(gs, rgs, TOL, f"task {i} grad_s", blocks=s_blocks(it.net),
                     floor=lambda: f32()[1])
        assert_close(gb, rgb, TOL, f"task {i} grad_b", blocks=b_blocks(it.net),
                     floor=lambda: f32()[2])
        # the single-instance entry point on the same data
        pts = a.DevicePoints(it.pts.xt_r, it.pts.x_0, it.pts.t_b)
        sgs, sgb, sl = a.grad_s(dn[it.net_id], it.s, it.mu_d, pts, cfg)
        torch.cuda.synchronize()
        for name, x, y in (("grad_s", gs, sgs), ("grad_b", gb, sgb), ("loss", loss, sl)):
            y = y.cpu().numpy()
            assert_close(x, y, 1e-6, f"task {i} {name} vs lrnr_grad_s")
            log(f"  task {i} {name}: bitwise equal to lrnr_grad_s: {np.array_equal(x, y)}")
    # loss-only mode
    for it in insts:
        it.loss.fill_(np.nan)
    run(a.MODE_LOSS, dn, insts, cfg)
    for i, it in enumerate(insts):
        l4, _, _ = orc.lrnr_loss(it.net, it.s_list(), it.mu.astype(np.float64), it.pts, {})
        assert_close(it.loss.cpu().numpy(), l4, TOL, f"task {i} loss (LOSS mode)")


@KINDS
def test_tasks_alone_equals_mix_bitwise(kind):
    """Each task's outputs do not depend on the other tasks of the launch."""
    a = api()
    hn = nets(kind)
    dn = [a.DeviceNet.from_net(n) for n in hn]
    mk = lambda: [Inst(0, hn[0], 200, 3000, 300, 300), Inst(1, hn[1], 201, 700, 90, 50),
                  Inst(0, hn[0], 202, 64, 8, 8, 0.9), Inst(1, hn[1], 203, 5000, 600, 600, 1.1)]
    cfg = a.LossCfg(form=1, lambda_loc=0.01, s_ref=None)
    for mode, name in ((a.MODE_GRAD, "grad"), (a.MODE_LOSS, "loss")):
        pool = mk()
        # lambda_loc needs a reference: a scaled copy of each task's s
        for it in pool:
            it.s_ref = (it.s * 0.95).contiguous()
        tab_cfg = cfg

        def run_set(sel):
            tab = a.TaskTable(dn)
            for it in sel:
                tab.add(it.net_id, s=it.s, mu=it.mu_d, xt_r=it.xt, x_0=it.x0, t_b=it.tb,
                        s_ref=it.s_ref, grad_s=it.gs, grad_b=it.gb, loss=it.loss)
            tab.run(mode, tab_cfg)
            torch.cuda.synchronize()
            return [it.outputs() for it in sel]

        alone = [run_set([it])[0] for it in pool]
        mixes = [pool, pool[::-1], [pool[2], pool[0], pool[3], pool[1]]]
        for m in mixes:
            got = run_set(m)
            for it, o in zip(m, got):
                ref = alone[pool.index(it)]
                for x, y in zip(o, ref):
                    # (LOSS mode leaves the gradient buffers at their NaN fill)
                    assert np.array_equal(x, y, equal_nan=True), (name, pool.index(it))
        log(f"  {name}: alone == mix bitwise over {len(mixes)} orderings of {len(pool)} tasks")


@KINDS
def test_tasks_jets_value_vjp_vs_oracle(kind):
    a = api()
    hn = nets(kind)
    dn = [a.DeviceNet.from_net(n) for n in hn]
    insts = [Inst(0, hn[0], 300, 1500, 0, 0), Inst(1, hn[1], 301, 777, 0, 0),
             Inst(0, hn[0], 302, 1, 0, 0)]
    log(f"[case] task table JETS / VALUE / VJP ({kind} nets), 3 tasks")
    run(a.MODE_JETS, dn, insts, out_attr="jets")
    run(a.MODE_VALUE, dn, insts, out_attr="val")
    run(a.MODE_VJP, dn, insts, out_attr="jets")
    for i, it in enumerate(insts):
        xt = it.pts.xt_r.astype(np.float64)
        rj = orc.lrnr_forward_jets(it.net, it.s_list(), xt)
        j = it.jets.cpu().numpy()
        for c, tol in ((0, TOL), (1, TOL), (2, TOL), (3, TOL_XX)):
            assert_close(j[c], rj[c], tol, f"task {i} jets[{c}]")
        assert_close(it.val.cpu().numpy(), rj[0], TOL, f"task {i} value")
        rgs, rgb = orc.lrnr_jets_vjp(it.net, it.s_list(), xt, it.cot_host.astype(np.float64))
        assert_close(it.gs.cpu().numpy(), rgs, TOL, f"task {i} vjp grad_s", blocks=s_blocks(it.net))
        assert_close(it.gb.cpu().numpy(), rgb, TOL, f"task {i} vjp grad_b", blocks=b_blocks(it.net))
        # the single-instance jets entry point
        sj = a.forward_jets(dn[it.net_id], it.s, it.xt).cpu().numpy()
        assert_close(j, sj, 1e-6, f"task {i} jets vs lrnr_forward_jets")


@KINDS
def test_tasks_empty_and_many(kind):
    """Tasks with no points give zero loss and gradient; 150 tasks exercise
    the task search past one wave of candidates."""
    a = api()
    hn = nets(kind)
    dn = [a.DeviceNet.from_net(n) for n in hn]
    insts = []
    for i in range(150):
        k = i % 2
        n = 0 if i % 37 == 5 else 40 + 13 * (i % 11)
        insts.append(Inst(k, hn[k], 400 + i, n, n // 8, (n // 8) * (i % 3 != 0)))
    log(f"[case] 150 tasks, sizes up to {max(len(it.pts.xt_r) for it in insts)}, "
        f"{sum(len(it.pts.xt_r) == 0 for it in insts)} empty")
    run(a.MODE_GRAD, dn, insts, a.LossCfg())
    for i, it in enumerate(insts):
        gs, gb, loss = it.outputs()
        if len(it.pts.xt_r) == 0:
            assert np.all(gs == 0) and np.all(gb == 0) and np.all(loss == 0), i
            continue
        if i % 10 == 0:
            l4, rgs, rgb = orc.lrnr_loss(it.net, it.s_list(), it.mu.astype(np.float64), it.pts,
                                         {}, with_grad=True)
            f32 = fp32(lambda: orc.lrnr_loss(it.net, it.s_list(), it.mu, it.pts, {},
                                             with_grad=True))
            assert_close(loss, l4, TOL, f"task {i} loss", blocks=LOSS_BLOCKS,
                         floor=lambda: f32()[0])
            assert_close(gs, rgs, TOL, f"task {i} grad_s", blocks=s_blocks(it.net),
                         floor=lambda: f32()[1])
        assert np.all(np.isfinite(gs)) and np.all(np.isfinite(loss)), i


@KINDS
def test_tasks_persistent_workgroups_keep_and_switch_nets(kind):
    """More tiles than persistent workgroups: each workgroup runs several
    tiles in a row, of one net or of alternating nets (resident factors kept
    or restaged).  Every task's outputs equal its one-task table bitwise, and
    the jets agree with the single-instance entry point's."""
    a = api()
    hn = nets(kind)
    dn = [a.DeviceNet.from_net(n) for n in hn]
    ids = [0, 1, 0, 0, 1]
    pool = [Inst(k, hn[k], 500 + i, 65536, 8192, 8192, 0.9 + 0.05 * i)
            for i, k in enumerate(ids)]
    cfg = a.LossCfg()
    log(f"[case] {len(pool)} tasks of 65,536 + 8192 + 8192 points, nets {ids} ({kind})")

    def run_set(sel, mode):
        tab = a.TaskTable(dn)
        for it in sel:
            tab.add(it.net_id, s=it.s, mu=it.mu_d, xt_r=it.xt, x_0=it.x0, t_b=it.tb,
                    grad_s=it.gs, grad_b=it.gb, loss=it.loss)
        tab.run(mode, cfg)
        torch.cuda.synchronize()
        return [it.outputs() for it in sel]

    for mode, name in ((a.MODE_GRAD, "grad"), (a.MODE_LOSS, "loss")):
        alone = [run_set([it], mode)[0] for it in pool]
        for order in (pool, pool[::-1]):
            got = run_set(order, mode)
            for it, o in zip(order, got):
                ref = alone[pool.index(it)]
                for x, y in zip(o, ref):
                    assert np.array_equal(x, y, equal_nan=True), (name, pool.index(it))
    it = pool[3]
    l4, rgs, _ = orc.lrnr_loss(it.net, it.s_list(), it.mu.astype(np.float64), it.pts, {},
                               with_grad=True)
    f32 = fp32(lambda: orc.lrnr_loss(it.net, it.s_list(), it.mu, it.pts, {}, with_grad=True))
    gs, _, loss = alone[3]
    assert_close(loss, l4, TOL, "task 3 loss", blocks=LOSS_BLOCKS, floor=lambda: f32()[0])
    assert_close(gs, rgs, TOL, "task 3 grad_s", blocks=s_blocks(it.net), floor=lambda: f32()[1])
    # forward-only modes over the same tables
    for it in pool:
        it.jets.fill_(np.nan)
    run(a.MODE_JETS, dn, pool, out_attr="jets")
    for i, it in enumerate(pool):
        sj = a.forward_jets(dn[it.net_id], it.s, it.xt)
        torch.cuda.synchronize()
        assert_close(it.jets.cpu().numpy(), sj.cpu().numpy(), 1e-6,
                     f"task {i} jets vs lrnr_forward_jets")
    log("  alone == mix bitwise (grad, loss); jets agree with lrnr_forward_jets")


def test_tasks_large_preactivations_take_the_accurate_path():
    """Four neurons of layer 1 of one net get zero U-rows and bias 2^25, so
    their pre-activation is exactly 2^25 (the fast sin/cos reduction is not
    valid there): every tile of its tasks is flagged and recomputed by the
    accurate relaunch, which scans the flags a workgroup-width at a time.
    Tasks of the other net are not flagged and keep the fast pass's
    results."""
    a = api()
    hn = nets("narrow")
    big = wl.make_net(np.random.Generator(np.random.PCG64(52)), [2, 64, 64, 64, 1],
                      wl.ranks([2, 64, 64, 64, 1], 8))
    big.U[0][:4, :] = 0.0
    big.b[0][:4] = np.float32(2.0 ** 25)
    hn = [hn[0], big]
    dn = [a.DeviceNet.from_net(n) for n in hn]
    ids = [0, 1, 0, 1]
    pool = [Inst(k, hn[k], 600 + i, 40000, 4000, 4000) for i, k in enumerate(ids)]
    cfg = a.LossCfg()
    log(f"[case] task table GRAD with |a| = 2^25 in net 1, tasks {ids}")
    run(a.MODE_GRAD, dn, pool, cfg)
    for i in (0, 1):
        it = pool[i]
        gs, gb, loss = it.outputs()
        l4, rgs, rgb = orc.lrnr_loss(it.net, it.s_list(), it.mu.astype(np.float64), it.pts, {},
                                     with_grad=True)
        f32 = fp32(lambda: orc.lrnr_loss(it.net, it.s_list(), it.mu, it.pts, {}, with_grad=True))
        assert_close(loss, l4, TOL, f"task {i} loss", blocks=LOSS_BLOCKS, floor=lambda: f32()[0])
        assert_close(gs, rgs, TOL, f"task {i} grad_s", blocks=s_blocks(it.net),
                     floor=lambda: f32()[1])
        assert_close(gb, rgb, TOL, f"task {i} grad_b", blocks=b_blocks(it.net),
                     floor=lambda: f32()[2])


def test_tasks_invalid_arguments():
    a = api()
    from paper_2410_04001_amd import _clib as cl
    hn = nets()
    dn = [a.DeviceNet.from_net(n) for n in hn]
    it = Inst(0, hn[0], 500, 100, 10, 10)
    tab = a.TaskTable(dn)
    tab.add(5, s=it.s, mu=it.mu_d, xt_r=it.xt, grad_s=it.gs)      # net index out of range
    with pytest.raises(cl.LrnrError):
        tab.run(a.MODE_GRAD, a.LossCfg())
    tab = a.TaskTable(dn)
    tab.add(0, s=it.s, mu=it.mu_d, xt_r=it.xt)                      # GRAD without grad_s
    with pytest.raises(cl.LrnrError):
        tab.run(a.MODE_GRAD, a.LossCfg())
