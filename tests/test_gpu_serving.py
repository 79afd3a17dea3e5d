"""Serving engine (lrnr_srv_*): continuous batching of new-mu requests.

Checked: a request's tuned s, last loss and grid values are bitwise identical
alone and in a mix with other requests arriving while it runs, with graph
replay or direct launches, and with several steps per launch, for FastLRNR
models and for wider LRNR models (the two gradient kernels); they equal a
plain loop of the task entry point and Adam; the grid values match the FP64
oracle's FastLRNR forward at the tuned s; admission by arena footprint
bounds the requests in flight.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import assert_close, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-4
K = 100


@pytest.fixture(scope="module")
def models():
    assert torch.cuda.is_available(), "the gpu tests need the MI355X"
    from paper_2410_04001_amd import api
    w = wl.fast_case(2, n=16)
    net = api.DeviceNet.from_net(w.net)
    s0 = torch.tensor(w.net.s_flat(), device="cuda")
    xs = torch.tensor(w.extra["xt_snap"], device="cuda")
    fasts = [api.FastLRNR(net, s0.reshape(1, -1), xs, rh) for rh in (16, 32, 48)]
    yield w, net, s0, fasts
    for f in fasts:
        f.close()


def make_server(models, **kw):
    from paper_2410_04001_amd import serving
    w, net, s0, fasts = models
    return serving.Server([(f.net, s0) for f in fasts], K=K, **kw)


def requests(srv, specs):
    """specs: (id, model, n, seed)."""
    out = []
    for rid, model, n, seed in specs:
        pts = wl.request_points(seed, n)
        mu = wl.make_mu(np.random.Generator(np.random.PCG64(seed + 7)), 1)[0]
        out.append(srv.request(rid, model, mu, pts))
    return out


SPECS = [(0, 1, 5000, 11), (1, 0, 1024, 12), (2, 2, 20000, 13), (3, 1, 3001, 14),
         (4, 0, 65536, 15), (5, 2, 777, 16)]


def outputs(r):
    return r.u.copy(), r.s.copy(), r.loss.copy()


def run_alone(models, spec, **kw):
    srv = make_server(models, **kw)
    (r,) = requests(srv, [spec])
    srv.submit(r)
    srv.run_until_done()
    srv.close()
    return outputs(r)


def test_serving_alone_equals_mix_bitwise(models):
    alone = {sp[0]: run_alone(models, sp) for sp in SPECS}
    for kw in ({}, {"steps_per_launch": 1}, {"steps_per_launch": 4},
               {"use_graph": False, "max_inflight": 3}):
        srv = make_server(models, **kw)
        reqs = requests(srv, SPECS)
        # staggered arrivals: two now, the rest while those run
        srv.submit(reqs[0])
        srv.submit(reqs[1])
        for _ in range(5):
            srv.poll()
        for r in reqs[2:4]:
            srv.submit(r)
        for _ in range(20):
            srv.poll()
        for r in reqs[4:]:
            srv.submit(r)
        done = srv.run_until_done()
        st = srv.stats()
        srv.close()
        log(f"  {kw}: {len(done)} done, peak active {st['peak_active']}, launches "
            f"{st['launches']}, table uploads {st['table_uploads']}")
        assert len(done) == len(SPECS)
        for r in reqs:
            for x, y in zip(outputs(r), alone[r.id]):
                assert np.all(np.isfinite(x))
                assert np.array_equal(x, y), (kw, r.id)
    log("  every request bitwise equal alone and in the mixes")


def test_serving_equals_plain_loop_and_oracle(models):
    """K steps of lrnr_tasks_run(GRAD) + lrnr_adam_step on one request give the
    engine's tuned s; the engine's grid values match the oracle's FastLRNR
    forward at that s."""
    from paper_2410_04001_amd import api
    w, net, s0, fasts = models
    spec = (0, 1, 5000, 11)
    u, s_eng, loss_eng = run_alone(models, spec)
    fast = fasts[spec[1]]
    pts = wl.request_points(spec[3], spec[2])
    mu = wl.make_mu(np.random.Generator(np.random.PCG64(spec[3] + 7)), 1)[0]
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda").contiguous()
    s = s0.clone()
    m = torch.zeros_like(s)
    v = torch.zeros_like(s)
    g = torch.empty_like(s)
    loss = torch.empty(4, device="cuda")
    xt, x0, tb, mud = dev(pts.xt_r), dev(pts.x_0), dev(pts.t_b), dev(mu)
    tab = api.TaskTable([fast.net])
    tab.add(0, s=s, mu=mud, xt_r=xt, x_0=x0, t_b=tb, grad_s=g, loss=loss)
    for k in range(1, K + 1):
        tab.run(api.MODE_GRAD, api.LossCfg())
        api.adam_step(s, m, v, g, k)
    torch.cuda.synchronize()
    s_loop = s.cpu().numpy()
    assert_close(s_eng, s_loop, 1e-6, "engine s vs plain loop")
    assert_close(loss_eng, loss.cpu().numpy(), 1e-6, "engine last loss vs plain loop")
    log(f"  engine s bitwise equal to the plain loop: {np.array_equal(s_eng, s_loop)}")
    ops = fast.operators()
    nx, nt = 256, 100
    grid = wl.grid_points(nx, nt)
    ref = orc.fast_forward_jets(w.net, ops, w.net.split_s(s_eng), grid.astype(np.float64))[0]
    assert_close(u, ref, TOL, "grid values vs oracle FastLRNR forward")
    # the tuning lowered the request's loss
    l0 = orc.fast_loss(w.net, ops, w.net.s, mu.astype(np.float64), pts, {})[0][0]
    l1 = orc.fast_loss(w.net, ops, w.net.split_s(s_eng), mu.astype(np.float64), pts, {})[0][0]
    log(f"  request loss {l0:.5f} -> {l1:.5f} after {K} steps")
    assert l1 < l0


def test_serving_admission_by_memory(models):
    from paper_2410_04001_amd import _clib as cl
    probe = make_server(models)
    fps = [probe.footprint(sp[1], sp[2], sp[2] // 8, sp[2] // 8) for sp in SPECS]
    probe.close()
    big = max(fps)
    arena = int(1.1 * big)
    assert sum(fps) > arena
    log(f"[case] arena {arena} bytes = 1.1 x largest request footprint {big} "
        f"(all six need {sum(fps)})")
    srv = make_server(models, arena_bytes=arena)
    reqs = requests(srv, SPECS)
    for r in reqs:
        srv.submit(r)
    done = srv.run_until_done()
    st = srv.stats()
    log(f"  peak active {st['peak_active']}, arena peak {st['arena_peak']}")
    assert len(done) == len(SPECS)
    assert st["arena_peak"] <= arena
    assert st["peak_active"] < len(SPECS)
    too_big = srv.request(99, 0, [1.0, 0.0, 0.0], wl.request_points(1, 200000))
    with pytest.raises(cl.LrnrError) as ei:
        srv.submit(too_big)
    assert ei.value.status == cl.ENOMEM
    srv.close()
    alone = run_alone(models, SPECS[2])
    for x, y in zip(outputs(reqs[2]), alone):
        assert np.array_equal(x, y)


@pytest.fixture(scope="module")
def wide_models():
    """Two LRNRs of widest layer 128 at rank tile 16: their gradient runs the
    four-role kernel (the FastLRNR models above run the single-role one)."""
    from paper_2410_04001_amd import api
    out = []
    for seed, M in ((61, [2, 128, 128, 128, 1]), (62, [2, 120, 100, 1])):
        rng = np.random.Generator(np.random.PCG64(seed))
        net = wl.make_net(rng, M, wl.ranks(M, 16))
        out.append((api.DeviceNet.from_net(net), torch.tensor(net.s_flat(), device="cuda")))
    return out


def test_serving_alone_equals_mix_bitwise_wide_models(wide_models):
    from paper_2410_04001_amd import serving
    specs = [(0, 0, 3000, 21), (1, 1, 900, 22), (2, 0, 12000, 23), (3, 1, 700, 24)]
    alone = {}
    for sp in specs:
        srv = serving.Server(wide_models, K=K)
        (r,) = requests(srv, [sp])
        srv.submit(r)
        srv.run_until_done()
        srv.close()
        alone[sp[0]] = outputs(r)
    for kw in ({}, {"use_graph": False, "max_inflight": 3}):
        srv = serving.Server(wide_models, K=K, **kw)
        reqs = requests(srv, specs)
        srv.submit(reqs[0])
        srv.submit(reqs[1])
        for _ in range(5):
            srv.poll()
        for r in reqs[2:]:
            srv.submit(r)
        done = srv.run_until_done()
        srv.close()
        assert len(done) == len(specs)
        for r in reqs:
            for x, y in zip(outputs(r), alone[r.id]):
                assert np.all(np.isfinite(x))
                assert np.array_equal(x, y), (kw, r.id)
    log(f"  wide models: every request bitwise equal alone and in the mixes")


def test_serving_rejects_nonfinite_mu(models):
    from paper_2410_04001_amd import _clib as cl
    srv = make_server(models)
    (r,) = requests(srv, [(0, 1, 1024, 11)])
    r.mu = np.array([np.nan, 1.0, 1.0], np.float32)
    rc = r.c(0.0)
    import ctypes as C
    assert cl.lib().lrnr_srv_submit(srv._h, C.byref(rc)) == cl.EINVAL
    r.mu = np.array([1.0, np.inf, 1.0], np.float32)
    rc = r.c(0.0)
    assert cl.lib().lrnr_srv_submit(srv._h, C.byref(rc)) == cl.EINVAL
    assert srv.stats()["submitted"] == 0
    srv.close()


def test_serving_failure_isolation_and_cancellation(models):
    """A request with a non-finite point (an input value) completes alone with
    status NONFINITE after 0 steps (s left at s_init, grid written); one
    request cancelled while waiting and one cancelled while tuning complete
    with status CANCELLED and no outputs; every other request in the mix is
    bitwise equal to its solo run."""
    from paper_2410_04001_amd import _clib as cl
    w, net, s0, fasts = models
    specs = SPECS[:4]
    alone = {sp[0]: run_alone(models, sp) for sp in specs}
    srv = make_server(models)
    reqs = requests(srv, specs)
    pts = wl.request_points(21, 4000)
    pts.xt_r[17, 0] = np.nan
    mu = wl.make_mu(np.random.Generator(np.random.PCG64(28)), 1)[0]
    bad = srv.request(100, 1, mu, pts)
    c_wait, c_run = requests(srv, [(101, 0, 2000, 22), (102, 2, 9000, 23)])
    srv.submit(reqs[0])
    srv.submit(bad)
    srv.submit(c_run)
    for _ in range(6):
        srv.poll()
    srv.submit(c_wait)
    srv.cancel(101)             # still waiting: completes at once
    srv.cancel(102)             # tuning: leaves the table before the next launch
    for r in reqs[1:]:
        srv.submit(r)
    done = srv.run_until_done()
    st = srv.stats()
    srv.close()
    rec = {r.id: r.record for r in done}
    log(f"  statuses { {k: (v['status'], v['steps']) for k, v in rec.items()} }, stats "
        f"failed {st['failed']} cancelled {st['cancelled']} completed {st['completed']}")
    assert len(done) == len(specs) + 3
    assert st["failed"] == 1 and st["cancelled"] == 2 and st["completed"] == len(specs) + 3
    assert rec[100]["status"] == cl.SRV_NONFINITE and rec[100]["steps"] == 0
    assert not np.isfinite(bad.loss[0])
    fast = fasts[1]
    assert np.array_equal(bad.s, s0.cpu().numpy()[:fast.net.r_total])
    assert np.all(np.isfinite(bad.u))
    for c in (c_wait, c_run):
        assert rec[c.id]["status"] == cl.SRV_CANCELLED
        assert np.all(np.isnan(c.u)) and np.all(np.isnan(c.s)) and np.all(np.isnan(c.loss))
    assert rec[101]["admitted"] == 0.0
    for r in reqs:
        assert rec[r.id]["status"] == cl.SRV_OK and rec[r.id]["steps"] == K
        for x, y in zip(outputs(r), alone[r.id]):
            assert np.array_equal(x, y), r.id
    srv2 = make_server(models)
    try:
        with pytest.raises(cl.LrnrError):
            srv2.cancel(12345)          # unknown id
    finally:
        srv2.close()
