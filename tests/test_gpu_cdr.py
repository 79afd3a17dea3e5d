"""GPU parity of the CDR reference solver (lrnr_cdr_reference) and of the L1
relative error (lrnr_l1_error) against the FP64 oracle
(oracle/cdr_reference.py), through the C ABI.

Bar: both sides compute in FP64 with different transforms (the device's own
radix-2 FFT pair against numpy's FFT), so finite outputs agree to rounding:
|gpu - ref| <= 1e-9 max(1, |ref|) elementwise (near a blow-up the flow
amplifies rounding differences, hence the relative part); the blow-up step
(status) is an integer decision and must be equal; NaN exactly where the
oracle has NaN.  The L1 sums agree with numpy's to 1e-12 relative and are
bitwise reproducible.
"""
import numpy as np
import pytest

from oracle import cdr_reference as cdr

from _util import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RTOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "the gpu tests need the MI355X"
    from paper_2410_04001_amd import _clib
    _clib.lib()


def api():
    from paper_2410_04001_amd import api as a
    return a


def mu_cases(seed=0, n1=10, n2=10):
    """mu drawn uniformly from the two parameter domains of Section 4."""
    import workloads as wl
    return wl.cdr_test_cases(seed, n1, n2)


def check(u_gpu, st_gpu, u_ref, st_ref, what):
    assert np.array_equal(st_gpu, st_ref), (what, st_gpu, st_ref)
    nan_g, nan_r = np.isnan(u_gpu), np.isnan(u_ref)
    assert np.array_equal(nan_g, nan_r), what
    fin = ~nan_r
    err = np.abs(u_gpu[fin] - u_ref[fin]) / np.maximum(1.0, np.abs(u_ref[fin]))
    worst = float(err.max()) if err.size else 0.0
    log(f"  {what}: max scaled err {worst:.2e}, statuses {st_ref.tolist()}")
    assert worst <= RTOL, (what, worst)


def run(mus, n_x, n_t, n_out, t_end=1.0):
    a = api()
    mu = torch.tensor(np.asarray(mus, np.float64), device="cuda")
    u, st = a.cdr_reference(mu, n_x, n_t, n_out, t_end)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st.cpu().numpy()


# n_x = 4^m runs the radix-4 kernel (16: outer and span-4 stages only), the
# other powers of two the radix-2 kernel
@pytest.mark.parametrize("n_x,n_t,n_out", [(8, 20, 5), (16, 40, 5), (32, 30, 4), (64, 200, 11),
                                           (128, 60, 4), (256, 500, 2), (512, 100, 101),
                                           (1024, 200, 21)])
def test_solver_matches_oracle_across_grid_sizes(n_x, n_t, n_out):
    mus = np.concatenate([mu_cases(1, 3, 5), [[0, 0, 0], [0, 0, 2.0], [2.0, 2.0, 0.0]]])
    log(f"[case] cdr n_x={n_x} n_t={n_t} n_out={n_out} B={len(mus)}")
    ug, sg = run(mus, n_x, n_t, n_out)
    ur, sr = cdr.cdr_solve_batch(mus, n_x, n_t, n_out)
    check(ug, sg, ur, sr, f"n_x={n_x}")


def test_solver_test_cases_at_working_size():
    # 10 + 10 test cases of the Section 4 comparison, 256 x 1000 steps, 101 outputs
    mus = mu_cases()
    log("[case] cdr 20 test cases, n_x=256 n_t=1000 n_out=101")
    ug, sg = run(mus, 256, 1000, 101)
    ur, sr = cdr.cdr_solve_batch(mus, 256, 1000, 101)
    check(ug, sg, ur, sr, "20 test cases")
    assert np.all(sr[:10] == 0)          # D1 never blows up
    x = 2 * np.pi * np.arange(256) / 256
    for i in range(10):                   # D1: u = sin(x - beta t)
        t = np.arange(101) / 100.0
        exact = np.sin(x[None, :] - mus[i, 0] * t[:, None])
        assert np.abs(ug[i] - exact).max() < 1e-11


def test_solver_t_end_blow_up_and_determinism():
    mus = [[0.0, 0.0, 2.0], [1.0, 0.0, 1.5], [3.0, 1.0, 0.5]]
    log("[case] cdr t_end=0.5, blow-up, repeat")
    ug, sg = run(mus, 128, 400, 9, t_end=0.5)
    ur, sr = cdr.cdr_solve_batch(mus, 128, 400, 9, t_end=0.5)
    check(ug, sg, ur, sr, "t_end 0.5")
    assert sg[0] == int(np.ceil(np.log(2.0) / 2.0 / (0.5 / 400)))
    ug2, sg2 = run(mus, 128, 400, 9, t_end=0.5)
    assert np.array_equal(sg, sg2)
    assert np.array_equal(ug.view(np.int64), ug2.view(np.int64))


def test_solver_argument_checks():
    a = api()
    from paper_2410_04001_amd import _clib as cl
    mu = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
    for n_x, n_t, n_out in [(100, 10, 2), (4, 10, 2), (2048, 10, 2), (64, 10, 4), (64, 0, 2),
                            (64, 10, 1)]:
        with pytest.raises(RuntimeError):
            a.cdr_reference(mu, n_x, n_t, n_out)
    u = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = cl.lib().lrnr_cdr_reference(None, 0, 64, 10, 2, 1.0, None, None, None)
    assert rc == cl.OK                      # B = 0: nothing to do
    rc = cl.lib().lrnr_cdr_reference(None, 1, 64, 10, 2, 1.0, u.data_ptr(), None, None)
    assert rc == cl.EINVAL


@pytest.mark.parametrize("n", [0, 1, 1025, 300_000])
def test_l1_error_sums(n):
    a = api()
    rng = np.random.Generator(np.random.PCG64(n))
    ref = rng.standard_normal(n)
    pred = (ref + 0.1 * rng.standard_normal(n)).astype(np.float32)
    log(f"[case] l1 error n={n}")
    out = a.l1_error_sums(torch.tensor(pred, device="cuda"), torch.tensor(ref, device="cuda"))
    out2 = a.l1_error_sums(torch.tensor(pred, device="cuda"), torch.tensor(ref, device="cuda"))
    g = out.cpu().numpy()
    d_ref = np.sum(np.abs(pred.astype(np.float64) - ref))
    r_ref = np.sum(np.abs(ref))
    assert g[0] == pytest.approx(d_ref, rel=1e-12, abs=0)
    assert g[1] == pytest.approx(r_ref, rel=1e-12, abs=0)
    assert np.array_equal(g.view(np.int64), out2.cpu().numpy().view(np.int64))
    if n:
        assert g[0] / g[1] == pytest.approx(cdr.l1_relative_error(pred, ref), rel=1e-12)


def test_l1_error_of_the_lrnr_on_the_reference_grid():
    # the evaluation of the Section 4 comparison: u of an LRNR on the output
    # grid of the reference, L1 relative error on the device and in the oracle
    import workloads as wl
    from oracle import lrnr_oracle as orc
    a = api()
    w = wl.fast_case(2, n=1024)
    net = a.DeviceNet.from_net(w.net)
    s = torch.tensor(w.net.s_flat(), device="cuda")
    mus = mu_cases(3, 1, 1)
    ug, sg = run(mus, 64, 200, 11)
    xt = cdr.grid_points(64, 11).astype(np.float32)
    u_net = a.forward_value(net, s, torch.tensor(xt, device="cuda"))
    u_orc = orc.lrnr_forward_jets(w.net, w.net.s, xt.astype(np.float64))[0]
    for i in range(len(mus)):
        if sg[i]:
            continue
        ref = torch.tensor(ug[i].reshape(-1), device="cuda")
        sums = a.l1_error_sums(u_net, ref).cpu().numpy()
        got = sums[0] / sums[1]
        assert got == pytest.approx(cdr.l1_relative_error(u_net.cpu().numpy(), ug[i]), rel=1e-12)
        assert got == pytest.approx(cdr.l1_relative_error(u_orc, ug[i]), rel=1e-4)
