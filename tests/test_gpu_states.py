"""GPU parity of lrnr_reduced_states (y^{l+1} = V^{(l+1)T} z^l per hidden
layer) against the FP64 oracle: on the LRNR, on a FastLRNR with the full
index set (whose reduced states are the LRNR's), and on a FastLRNR at
r_hat = 8 against the oracle's eq. 2.8 chain on the device's operators.
Bar: 1e-4 relative in the 2-norm and the max-norm, as the other parity tests."""
import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import assert_close, log

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


def oracle_states(net, xt):
    z = orc.lrnr_hidden_values(net, net.s, xt.astype(np.float64))
    return [zl @ net.V[l + 1].astype(np.float64) for l, zl in enumerate(z)]


@pytest.mark.parametrize("name,make", [("small", lambda: wl.small_lrnr(0, 16)),
                                       ("wide", lambda: wl.big_lrnr(1, 16))],
                         ids=["small", "wide"])
def test_reduced_states_match_oracle(name, make):
    a = api()
    w = make()
    rng = np.random.Generator(np.random.PCG64(4))
    xt = wl.uniform_points(rng, 3001)          # several blocks and a ragged tail
    log(f"[case] reduced states {name}: M={w.net.M} n=3001")
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    ys = a.reduced_states(net, s, torch.tensor(xt, device="cuda"))
    for l, (g, r) in enumerate(zip(ys, oracle_states(w.net, xt)), start=1):
        assert_close(g.cpu().numpy().T, r, TOL, f"{name} y^{l + 1}")
    empty = a.reduced_states(net, s, torch.zeros((0, 2), device="cuda"))
    assert all(e.numel() == 0 for e in empty)


def test_fastlrnr_reduced_states():
    a = api()
    w = wl.fast_case(2, n=1024)
    xs = torch.tensor(w.extra["xt_snap"], device="cuda")
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    rng = np.random.Generator(np.random.PCG64(6))
    xt = wl.uniform_points(rng, 2000)
    xt_d = torch.tensor(xt, device="cuda")
    y_full = a.reduced_states(net, s, xt_d)
    # the full index set reproduces the LRNR's states
    log("[case] FastLRNR r_hat = M reduced states")
    full = a.FastLRNR(net, s.reshape(1, -1), xs, w.net.M[1])
    for l, (g, r) in enumerate(zip(a.reduced_states(full.net, s, xt_d), y_full), start=1):
        assert_close(g.cpu().numpy(), r.cpu().numpy(), TOL, f"full index set y^{l + 1}")
    full.close()
    # r_hat = 8: the oracle's eq. 2.8 chain on the device's operators
    log("[case] FastLRNR r_hat = 8 reduced states")
    fast = a.FastLRNR(net, s.reshape(1, -1), xs, 8)
    ops = fast.operators()
    _, cache = orc.fast_forward(w.net, ops, w.net.s, xt.astype(np.float64))
    ref = [cache[l][0]["v"] for l in range(1, w.net.L)]
    for l, (g, r) in enumerate(zip(a.reduced_states(fast.net, s, xt_d), ref), start=1):
        assert_close(g.cpu().numpy().T, r, TOL, f"r_hat 8 z_hat^{l}")
    fast.close()
