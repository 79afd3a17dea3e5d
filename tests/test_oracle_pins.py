"""Pins of the FP64 oracle against things other than itself.

Each test fixes one part of the oracle by a route that does not reuse its
code: complex-step and finite-difference derivatives (Squire & Trapp 1998),
PyTorch float64 autograd on a textbook MLP (eq. 2.1 with the product of
eq. 2.2 formed explicitly), closed-form solutions of eq. 4.1, exact
properties of EIM/DEIM (eq. 2.7), the full-index-set reduction of eq. 2.8
to the LRNR, and the closed form of Adam's first steps.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny_case(seed=11, M=(2, 12, 10, 9, 1), rank=4, n=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    M = list(M)
    net = wl.make_net(rng, M, wl.ranks(M, rank))
    pts = wl.make_points(rng, n, 7, 5)
    mu = np.array([3.0, 0.7, 1.3])
    return net, pts, mu


# ---------------------------------------------------------------- jets -----

def test_jets_complex_step_x_t():
    net, pts, _ = tiny_case()
    xt = pts.xt_r.astype(np.float64)
    jets = orc.lrnr_forward_jets(net, net.s, xt)
    h = 1e-30
    for comp, col in (("x", 0), ("t", 1)):
        z = xt.astype(np.complex128)
        z[:, col] += 1j * h
        d = orc.lrnr_forward_jets(net, net.s, z)[0].imag / h
        ref = jets[1 if comp == "x" else 2]
        np.testing.assert_allclose(ref, d, rtol=1e-12, atol=1e-14)


def test_jets_uxx_difference_of_complex_step():
    net, pts, _ = tiny_case()
    xt = pts.xt_r.astype(np.float64)
    uxx = orc.lrnr_forward_jets(net, net.s, xt)[3]
    h, d = 1e-4, 1e-30

    def ux_cs(shift):
        z = xt.astype(np.complex128)
        z[:, 0] += shift + 1j * d
        return orc.lrnr_forward_jets(net, net.s, z)[0].imag / d

    fd = (ux_cs(h) - ux_cs(-h)) / (2 * h)
    scale = np.abs(uxx).max()
    np.testing.assert_allclose(uxx, fd, rtol=0, atol=1e-7 * scale)


def _torch_case(net, pts, mu, cfg):
    torch = pytest.importorskip("torch")
    dt = torch.float64
    U = [torch.tensor(u, dtype=dt) for u in net.U]
    V = [torch.tensor(v, dtype=dt) for v in net.V]
    b = [torch.tensor(x, dtype=dt, requires_grad=True) for x in net.b]
    s = [torch.tensor(x, dtype=dt, requires_grad=True) for x in net.s]
    L = len(U)

    def u_of(x, t):
        z = torch.stack([x, t], dim=-1)
        for l in range(L):
            W = U[l] @ torch.diag(s[l]) @ V[l].T
            z = z @ W.T + b[l]
            if l < L - 1:
                z = torch.sin(z)
        return z[..., 0]

    x = torch.tensor(pts.xt_r[:, 0], dtype=dt, requires_grad=True)
    t = torch.tensor(pts.xt_r[:, 1], dtype=dt, requires_grad=True)
    u = u_of(x, t)
    ux, = torch.autograd.grad(u.sum(), x, create_graph=True)
    ut, = torch.autograd.grad(u.sum(), t, create_graph=True)
    uxx, = torch.autograd.grad(ux.sum(), x, create_graph=True)
    beta, nu, rho = (float(m) for m in mu)
    res = ut + beta * ux - nu * uxx - rho * u * (1 - u)
    x0 = torch.tensor(pts.x_0, dtype=dt)
    tb = torch.tensor(pts.t_b, dtype=dt)
    e0 = u_of(x0, torch.zeros_like(x0)) - torch.sin(x0)
    eb = u_of(torch.zeros_like(tb), tb) - u_of(torch.full_like(tb, 2 * math.pi), tb)
    loss = (cfg["w_r"] * (res ** 2).mean() + cfg["w_0"] * (e0 ** 2).mean()
            + cfg["w_b"] * (eb ** 2).mean())
    loss.backward()
    jets = np.stack([u.detach().numpy(), ux.detach().numpy(), ut.detach().numpy(),
                     uxx.detach().numpy()])
    return (float(loss), jets, np.concatenate([x.grad.numpy() for x in s]),
            np.concatenate([x.grad.numpy() for x in b]))


def test_oracle_matches_torch_autograd_textbook_mlp():
    net, pts, mu = tiny_case()
    cfg = {"form": 0, "w_r": 1.0, "w_0": 2.0, "w_b": 0.5}
    tl, tj, tgs, tgb = _torch_case(net, pts, mu, cfg)
    jets = orc.lrnr_forward_jets(net, net.s, pts.xt_r)
    np.testing.assert_allclose(jets, tj, rtol=1e-11, atol=1e-13)
    l4, gs, gb = orc.lrnr_loss(net, net.s, mu, pts, cfg, with_grad=True)
    assert abs(l4[0] - tl) <= 1e-12 * abs(tl)
    np.testing.assert_allclose(gs, tgs, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(gb, tgb, rtol=1e-10, atol=1e-13)


# ------------------------------------------------------------ residual -----

def test_exact_zero_convection_residual():
    """u = h(x - beta t) solves u_t + beta u_x = 0 whatever h is: a net whose
    first layer sees only x - beta t must give a zero interior residual."""
    beta = 10.0
    rng = np.random.Generator(np.random.PCG64(5))
    M = [2, 16, 16, 16, 1]
    r = [1, 6, 6, 1]
    net = wl.convection_net(rng, M, r, beta)
    pts = wl.make_points(rng, 200, 10, 10)
    jets = orc.lrnr_forward_jets(net, net.s, pts.xt_r)
    res = orc.residual(jets[0], jets[1], jets[2], jets[3], [beta, 0.0, 0.0])
    rms = math.sqrt(np.mean((beta * jets[1]) ** 2))
    assert rms > 1e-3
    assert np.abs(res).max() <= 1e-12 * rms


def test_residual_closed_forms():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 2 * math.pi, 100)
    t = rng.uniform(0, 1, 100)
    beta, nu = 4.0, 0.7
    # u = exp(-nu t) sin(x - beta t) solves u_t + beta u_x - nu u_xx = 0
    e = np.exp(-nu * t)
    u = e * np.sin(x - beta * t)
    ux = e * np.cos(x - beta * t)
    ut = -nu * u - beta * ux
    uxx = -u
    assert np.abs(orc.residual(u, ux, ut, uxx, [beta, nu, 0.0])).max() < 1e-13
    # logistic u(t) solves u_t = rho u (1 - u), no x dependence
    rho, u0 = 2.5, 0.3
    u = 1.0 / (1.0 + (1 - u0) / u0 * np.exp(-rho * t))
    ut = rho * (1 - u0) / u0 * np.exp(-rho * t) * u * u
    z = np.zeros_like(u)
    assert np.abs(orc.residual(u, z, ut, z, [beta, 0.0, rho])).max() < 1e-13
    # a wrong sign anywhere must show: the same data with mu_2 flipped fails
    e = np.exp(-nu * t)
    u = e * np.sin(x - beta * t)
    ux = e * np.cos(x - beta * t)
    assert np.abs(orc.residual(u, ux, -nu * u - beta * ux, -u, [beta, -nu, 0.0])).max() > 1e-2


def test_loss_terms_brute_force_fsum():
    """The interior/initial/boundary means, assembled point by point with
    math.fsum from separately evaluated u at (x,0), (0,t) and (2 pi, t)."""
    net, pts, mu = tiny_case()
    cfg = {"form": 0, "w_r": 1.5, "w_0": 0.25, "w_b": 3.0}
    l4, _, _ = orc.lrnr_loss(net, net.s, mu, pts, cfg)
    jets = orc.lrnr_forward_jets(net, net.s, pts.xt_r)
    res = orc.residual(jets[0], jets[1], jets[2], jets[3], mu)
    interior = cfg["w_r"] * math.fsum(float(r) ** 2 for r in res) / len(res)
    ic = []
    for x in pts.x_0:
        u = orc.lrnr_forward_jets(net, net.s, np.array([[x, 0.0]]))[0, 0]
        ic.append((u - math.sin(float(x))) ** 2)
    bc = []
    for t in pts.t_b:
        ul = orc.lrnr_forward_jets(net, net.s, np.array([[0.0, t]]))[0, 0]
        ur = orc.lrnr_forward_jets(net, net.s, np.array([[2 * math.pi, t]]))[0, 0]
        bc.append((ul - ur) ** 2)
    ic_t = cfg["w_0"] * math.fsum(ic) / len(ic)
    bc_t = cfg["w_b"] * math.fsum(bc) / len(bc)
    np.testing.assert_allclose(l4[1:], [interior, ic_t, bc_t], rtol=1e-12)
    assert abs(l4[0] - (interior + ic_t + bc_t)) <= 1e-12 * l4[0]


# ------------------------------------------------------------ gradients ----

def _complex_step_grad(fun, x0, h=1e-30):
    g = np.zeros(len(x0))
    for k in range(len(x0)):
        z = x0.astype(np.complex128)
        z[k] += 1j * h
        g[k] = fun(z).imag / h
    return g


def test_grad_s_b_complex_step():
    net, pts, mu = tiny_case(n=25)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    _, gs, gb = orc.lrnr_loss(net, net.s, mu, pts, cfg, with_grad=True)
    s0 = net.s_flat().astype(np.float64)
    cs = _complex_step_grad(lambda z: orc.lrnr_loss(net, net.split_s(z), mu, pts, cfg)[0][0], s0)
    np.testing.assert_allclose(gs, cs, rtol=1e-11, atol=1e-14)
    b0 = np.concatenate(net.b).astype(np.float64)

    def lb(z):
        import copy
        n2 = copy.copy(net)
        out, o = [], 0
        for x in net.b:
            out.append(z[o:o + len(x)])
            o += len(x)
        n2.b = out
        return orc.lrnr_loss(n2, net.s, mu, pts, cfg)[0][0]

    cb = _complex_step_grad(lb, b0)
    np.testing.assert_allclose(gb, cb, rtol=1e-11, atol=1e-14)


def test_jets_vjp_complex_step():
    """The oracle's vector-Jacobian product of the jets (used by the
    differentiation form) against complex-step derivatives of the contracted
    jets, in s and in b."""
    net, pts, _ = tiny_case(n=30)
    xt = pts.xt_r.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(5))
    cot = rng.standard_normal((4, len(xt)))
    gs, gb = orc.lrnr_jets_vjp(net, net.s, xt, cot)
    s0 = net.s_flat().astype(np.float64)
    cs = _complex_step_grad(
        lambda z: np.sum(cot * orc.lrnr_forward_jets(net, net.split_s(z), xt)), s0)
    np.testing.assert_allclose(gs, cs, rtol=1e-11, atol=1e-13)
    b0 = np.concatenate(net.b).astype(np.float64)

    def lb(z):
        import copy
        n2 = copy.copy(net)
        out, o = [], 0
        for x in net.b:
            out.append(z[o:o + len(x)])
            o += len(x)
        n2.b = out
        return np.sum(cot * orc.lrnr_forward_jets(n2, net.s, xt))

    np.testing.assert_allclose(gb, _complex_step_grad(lb, b0), rtol=1e-11, atol=1e-13)


def test_grad_l1_form_and_locality_fd():
    net, pts, mu = tiny_case(n=25)
    s0 = net.s_flat().astype(np.float64)
    sref = s0 + np.linspace(-0.2, 0.2, len(s0)) + 0.013
    cfg = {"form": 1, "w_r": 1.0, "w_0": 0.5, "w_b": 2.0, "lambda_loc": 0.3, "s_ref": sref}
    _, gs, _ = orc.lrnr_loss(net, net.s, mu, pts, cfg, with_grad=True)
    h = 1e-7
    fd = np.zeros_like(s0)
    for k in range(len(s0)):
        sp, sm = s0.copy(), s0.copy()
        sp[k] += h
        sm[k] -= h
        fd[k] = (orc.lrnr_loss(net, net.split_s(sp), mu, pts, cfg)[0][0]
                 - orc.lrnr_loss(net, net.split_s(sm), mu, pts, cfg)[0][0]) / (2 * h)
    np.testing.assert_allclose(gs, fd, rtol=1e-6, atol=1e-7)


def test_chunked_oracle_equals_unchunked():
    net, pts, mu = tiny_case(n=50)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    a = orc.lrnr_loss(net, net.s, mu, pts, cfg, with_grad=True)
    b = orc.lrnr_loss_chunked(net, net.s, mu, pts, cfg, chunk=16)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------ FastLRNR -----

def test_deim_hand_worked_example():
    g = json.load(open(os.path.join(GOLD, "deim_4x2.json")))
    Xi = np.array(g["Xi"])
    assert list(orc.deim_indices(Xi)) == g["P"]


def test_deim_permuted_identity_picks_the_permutation():
    perm = [5, 2, 7, 0, 3]
    Xi = np.zeros((8, 5))
    for j, p in enumerate(perm):
        Xi[p, j] = 1.0 + 0.1 * j
    Xi[:, 1] += 0.3 * Xi[:, 0]        # lower-triangular mixing keeps the picks
    Xi[:, 4] += 0.2 * Xi[:, 2] - 0.1 * Xi[:, 3]
    assert list(orc.deim_indices(Xi)) == perm


def test_deim_interpolation_and_error_bound():
    rng = np.random.default_rng(7)
    Z = rng.standard_normal((30, 12)) @ rng.standard_normal((12, 200))
    Z += 1e-3 * rng.standard_normal(Z.shape)
    Xi = orc.pod_basis(Z, 8)
    P = orc.deim_indices(Xi)
    assert len(set(P.tolist())) == 8
    proj = Xi @ np.linalg.inv(Xi[P, :])
    f = rng.standard_normal(30)
    # interpolation: exact at the selected indices
    np.testing.assert_allclose((proj @ f[P])[P], f[P], rtol=1e-12, atol=1e-12)
    # reproduction: exact on span(Xi)
    g = Xi @ rng.standard_normal(8)
    np.testing.assert_allclose(proj @ g[P], g, rtol=1e-10, atol=1e-12)
    # error bound of DEIM for orthonormal Xi
    err = np.linalg.norm(f - proj @ f[P])
    bound = np.linalg.norm(np.linalg.inv(Xi[P, :]), 2) * np.linalg.norm(f - Xi @ (Xi.T @ f))
    assert err <= bound * (1 + 1e-10)
    # Xi is orthonormal and spans the leading left singular subspace
    np.testing.assert_allclose(Xi.T @ Xi, np.eye(8), atol=1e-12)


def test_qdeim_equals_pivoted_qr_of_xi_transposed():
    """Q-DEIM's picks are the first r pivots of LAPACK's column-pivoted QR
    of Xi^T (scipy.linalg.qr, geqp3), an independent implementation."""
    from scipy.linalg import qr
    rng = np.random.default_rng(11)
    for M, r in ((30, 8), (64, 32), (40, 20)):
        Z = rng.standard_normal((M, 3 * M))
        Xi = orc.pod_basis(Z, r)
        P = orc.qdeim_indices(Xi)
        piv = qr(Xi.T, pivoting=True)[2][:r]
        assert list(P) == list(piv), (M, r, P, piv)
        assert len(set(P.tolist())) == r


def test_qdeim_permuted_diagonal_picks_rows_by_norm():
    """Rows of distinct norms along distinct coordinates: the pivots are the
    rows in decreasing norm, whatever their order in Xi."""
    Xi = np.zeros((9, 4))
    for p, v, k in ((6, 5.0, 0), (1, 4.0, 1), (8, 3.0, 2), (3, 2.0, 3)):
        Xi[p, k] = v
    assert list(orc.qdeim_indices(Xi)) == [6, 1, 8, 3]


def test_qdeim_interpolation_and_error_bound():
    rng = np.random.default_rng(12)
    Z = rng.standard_normal((30, 12)) @ rng.standard_normal((12, 200))
    Z += 1e-3 * rng.standard_normal(Z.shape)
    Xi = orc.pod_basis(Z, 8)
    P = orc.qdeim_indices(Xi)
    proj = Xi @ np.linalg.inv(Xi[P, :])
    f = rng.standard_normal(30)
    np.testing.assert_allclose((proj @ f[P])[P], f[P], rtol=1e-12, atol=1e-12)
    err = np.linalg.norm(f - proj @ f[P])
    bound = np.linalg.norm(np.linalg.inv(Xi[P, :]), 2) * np.linalg.norm(f - Xi @ (Xi.T @ f))
    assert err <= bound * (1 + 1e-10)
    # Q-DEIM's guarantee: ||(P^T Xi)^{-1}||_2 <= sqrt(M - r + 1) * sqrt(4^r + 6 r - 1) / 3
    M, r = Xi.shape
    g = np.linalg.norm(np.linalg.inv(Xi[P, :]), 2)
    assert g <= np.sqrt(M - r + 1) * np.sqrt(4.0 ** r + 6 * r - 1) / 3


def test_fastlrnr_full_index_set_is_lrnr():
    net, pts, mu = tiny_case(M=(2, 12, 10, 9, 1), n=30)
    rng = np.random.default_rng(1)
    xt_snap = wl.uniform_points(rng, 64)
    fast = orc.fastlrnr_build(net, [net.s], xt_snap, [12, 10, 9])
    for P, M in zip(fast["P"], (12, 10, 9)):
        assert sorted(P.tolist()) == list(range(M))
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    l_a, g_a, _ = orc.lrnr_loss(net, net.s, mu, pts, cfg, with_grad=True)
    l_b, g_b = orc.fast_loss(net, fast, net.s, mu, pts, cfg, with_grad=True)
    np.testing.assert_allclose(l_b, l_a, rtol=1e-10)
    np.testing.assert_allclose(g_b, g_a, rtol=1e-9, atol=1e-12)
    ja = orc.lrnr_forward_jets(net, net.s, pts.xt_r)
    jb = orc.fast_forward_jets(net, fast, net.s, pts.xt_r)
    np.testing.assert_allclose(jb, ja, rtol=1e-9, atol=1e-11)


def test_fastlrnr_grad_complex_step():
    net, pts, mu = tiny_case(n=20)
    rng = np.random.default_rng(2)
    fast = orc.fastlrnr_build(net, [net.s], wl.uniform_points(rng, 64), [6, 5, 4])
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    _, gs = orc.fast_loss(net, fast, net.s, mu, pts, cfg, with_grad=True)
    s0 = net.s_flat().astype(np.float64)
    cs = _complex_step_grad(
        lambda z: orc.fast_loss(net, fast, net.split_s(z), mu, pts, cfg)[0][0], s0)
    np.testing.assert_allclose(gs, cs, rtol=1e-11, atol=1e-14)


def test_fastlrnr_jets_complex_step():
    net, pts, _ = tiny_case(n=20)
    rng = np.random.default_rng(2)
    fast = orc.fastlrnr_build(net, [net.s], wl.uniform_points(rng, 64), [6, 5, 4])
    xt = pts.xt_r.astype(np.float64)
    j = orc.fast_forward_jets(net, fast, net.s, xt)
    z = xt.astype(np.complex128)
    z[:, 0] += 1e-30j
    np.testing.assert_allclose(j[1], orc.fast_forward_jets(net, fast, net.s, z)[0].imag / 1e-30,
                               rtol=1e-12, atol=1e-14)


# ------------------------------------------------------ factored biases -----

def _bias_basis(net, q, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    B = [rng.standard_normal((m, min(q, m))) / math.sqrt(m) for m in net.M[1:]]
    sb = [rng.uniform(-1, 1, b.shape[1]) for b in B]
    return B, sb


def test_factored_bias_identity_basis_is_the_plain_bias():
    # B^l = I, s_b^l = b^l: same loss, and grad_sb equals grad_b
    net, pts, mu = tiny_case(n=25)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    B = [np.eye(len(b)) for b in net.b]
    l_a, gs_a, gb_a = orc.lrnr_loss(net, net.s, mu, pts, cfg, with_grad=True)
    l_b, gs_b, gsb = orc.lrnr_loss_factored_bias(net, net.s, B, net.b, mu, pts, cfg, True)
    np.testing.assert_allclose(l_b, l_a, rtol=1e-14)
    np.testing.assert_allclose(gs_b, gs_a, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(gsb, gb_a, rtol=1e-13, atol=1e-15)


def test_factored_bias_grad_complex_step():
    net, pts, mu = tiny_case(n=25)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    B, sb = _bias_basis(net, 3)
    _, gs, gsb = orc.lrnr_loss_factored_bias(net, net.s, B, sb, mu, pts, cfg, True)
    q = [len(x) for x in sb]
    sb0 = np.concatenate(sb)
    c = _complex_step_grad(lambda z: orc.lrnr_loss_factored_bias(
        net, net.s, B, orc._split(z, q), mu, pts, cfg)[0][0], sb0)
    np.testing.assert_allclose(gsb, c, rtol=1e-11, atol=1e-14)
    cs = _complex_step_grad(lambda z: orc.lrnr_loss_factored_bias(
        net, net.split_s(z), B, sb, mu, pts, cfg)[0][0], net.s_flat().astype(np.float64))
    np.testing.assert_allclose(gs, cs, rtol=1e-11, atol=1e-14)


def test_fastlrnr_factored_bias_full_index_set_and_complex_step():
    net, pts, mu = tiny_case(M=(2, 12, 10, 9, 1), n=30)
    rng = np.random.default_rng(1)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    B, sb = _bias_basis(net, 4)
    q = [len(x) for x in sb]
    # the index set of every neuron: FastLRNR with factored biases is the LRNR's
    full = orc.fastlrnr_build(net, [net.s], wl.uniform_points(rng, 64), [12, 10, 9])
    l_a, gs_a, gsb_a = orc.lrnr_loss_factored_bias(net, net.s, B, sb, mu, pts, cfg, True)
    l_b, gs_b, gsb_b = orc.fast_loss_factored_bias(net, full, net.s, B, sb, mu, pts, cfg, True)
    np.testing.assert_allclose(l_b, l_a, rtol=1e-10)
    np.testing.assert_allclose(gs_b, gs_a, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gsb_b, gsb_a, rtol=1e-9, atol=1e-12)
    # a reduced FastLRNR: analytic grad_sb against complex step
    fast = orc.fastlrnr_build(net, [net.s], wl.uniform_points(rng, 64), [6, 5, 4])
    _, _, gsb = orc.fast_loss_factored_bias(net, fast, net.s, B, sb, mu, pts, cfg, True)
    c = _complex_step_grad(lambda z: orc.fast_loss_factored_bias(
        net, fast, net.s, B, orc._split(z, q), mu, pts, cfg)[0][0], np.concatenate(sb))
    np.testing.assert_allclose(gsb, c, rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------- Adam -----

def test_adam_closed_form_constant_gradient():
    s = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr, eps = 1e-3, 1e-8
    for k in range(1, 6):
        s, m, v = orc.adam_step(s, g, m, v, k, lr=lr, eps=eps)
        # bias correction makes m_hat = g and v_hat = g^2 for a constant g
        expect = np.array([1.0, -2.0, 0.5]) - k * lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(s, expect, rtol=1e-12, atol=1e-15)


# ------------------------------------------------------- meta-learning -----

def _hyper_case(net, width=8, seed=21):
    rng = np.random.Generator(np.random.PCG64(seed))
    H = [3, width, width, net.r_total]
    theta = []
    for k in range(1, len(H)):
        theta.append(rng.standard_normal(H[k] * H[k - 1]) / math.sqrt(H[k - 1]))
        theta.append(rng.uniform(0.2, 0.8, H[k]) if k == len(H) - 1 else rng.uniform(-0.5, 0.5, H[k]))
    mus = np.stack([rng.uniform(1, 3, 3), rng.uniform(0, 2, 3), rng.uniform(0, 2, 3)], axis=1)
    return H, np.concatenate(theta), mus


def test_hyper_forward_backward_match_torch_autograd():
    import torch
    net, _, _ = tiny_case()
    H, theta, mus = _hyper_case(net)
    s, cache = orc.hyper_forward(H, theta, mus)
    rng = np.random.default_rng(4)
    s_bar = rng.standard_normal(s.shape)
    g = orc.hyper_backward(H, cache, s_bar)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    h = torch.tensor(mus, dtype=torch.float64)
    o = 0
    for k in range(1, len(H)):
        W = th[o:o + H[k] * H[k - 1]].reshape(H[k], H[k - 1])
        o += H[k] * H[k - 1]
        c = th[o:o + H[k]]
        o += H[k]
        h = torch.nn.functional.linear(h, W, c)
        if k < len(H) - 1:
            h = torch.sin(h)
    st = torch.relu(h)
    np.testing.assert_allclose(s, st.detach().numpy(), rtol=1e-13, atol=1e-14)
    (st * torch.tensor(s_bar)).sum().backward()
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_sparse_reg_zero_on_geometric_decay_and_hand_values():
    # R_sparse vanishes when s_{i+1} < s_i / gamma (the decay it promotes)
    r = [4, 3]
    gamma = 2.0
    s = np.array([[1.0, 0.4, 0.15, 0.05, 2.0, 0.9, 0.3]])
    assert orc.sparse_reg_value(s, r, gamma) == 0.0
    assert np.all(orc.sparse_reg_grad(s, r, gamma) == 0.0)
    # flat coefficients: every term is (gamma - 1) s
    s = np.array([[1.0, 1.0, 1.0, 1.0, 0.5, 0.5, 0.5]])
    assert orc.sparse_reg_value(s, r, gamma) == pytest.approx(3 * 1.0 + 2 * 0.5)
    np.testing.assert_allclose(orc.sparse_reg_grad(s, r, gamma)[0],
                               [-1, 1, 1, 2, -1, 1, 2])
    # the layers do not couple: the last entry of one layer and the first of
    # the next form no term
    s = np.array([[1.0, 0.1, 0.01, 0.001, 100.0, 1.0, 0.01]])
    assert orc.sparse_reg_value(s, r, gamma) == 0.0


def test_meta_objective_grad_complex_step():
    net, pts, _ = tiny_case(n=15)
    H, theta, mus = _hyper_case(net)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 1.0, "w_b": 1.0}
    obj, g = orc.meta_objective(net, H, theta, mus, pts, 1.5, 0.3, cfg, with_grad=True)
    c = _complex_step_grad(lambda z: orc.meta_objective(net, H, z, mus, pts, 1.5, 0.3, cfg)[0],
                           theta)
    np.testing.assert_allclose(g, c, rtol=1e-10, atol=1e-13)
    # the bias gradient of the same objective, against complex steps in b
    _, _, gb = orc.meta_objective(net, H, theta, mus, pts, 1.5, 0.3, cfg, with_grad=True,
                                  with_b=True)
    import copy
    sizes = [len(x) for x in net.b]

    def ob(z):
        n2 = copy.copy(net)
        n2.b = orc._split(z, sizes)
        return orc.meta_objective(n2, H, theta, mus, pts, 1.5, 0.3, cfg)[0]

    cb = _complex_step_grad(ob, np.concatenate(net.b).astype(np.float64))
    np.testing.assert_allclose(gb, cb, rtol=1e-10, atol=1e-13)
    # the objective is the mean of the per-sample losses plus the weighted term
    s, _ = orc.hyper_forward(H, theta, mus)
    per = [orc.lrnr_loss(net, net.split_s(s[b]), mus[b], pts, cfg)[0][0] for b in range(len(mus))]
    assert obj == pytest.approx(np.mean(per) + 0.3 * orc.sparse_reg_value(s, net.r, 1.5), rel=1e-14)


def test_orth_reg_zero_on_orthonormal_bases_and_complex_step():
    net, _, _ = tiny_case()
    # the generators column-orthonormalise U and V: R_orth vanishes (to FP32
    # rounding of the stored factors)
    assert orc.orth_reg(net.U, net.V) < 1e-11
    # a hand value: U = 2 I (2 x 2) gives ||4 I - I||^2 = 18, V = [1, 1]^T gives (2 - 1)^2 = 1
    assert orc.orth_reg([2 * np.eye(2)], [np.ones((2, 1))]) == pytest.approx(19.0)
    rng = np.random.default_rng(3)
    U = [rng.standard_normal((5, 3)), rng.standard_normal((4, 2))]
    V = [rng.standard_normal((3, 3)), rng.standard_normal((5, 2))]
    _, gU, gV = orc.orth_reg(U, V, with_grad=True)
    flat = np.concatenate([a.ravel() for a in U + V])
    shapes = [a.shape for a in U + V]

    def f(z):
        out, o = [], 0
        for sh in shapes:
            n = sh[0] * sh[1]
            out.append(z[o:o + n].reshape(sh))
            o += n
        return orc.orth_reg(out[:2], out[2:])

    c = _complex_step_grad(f, flat)
    np.testing.assert_allclose(np.concatenate([a.ravel() for a in gU + gV]), c, rtol=1e-12,
                               atol=1e-13)


def test_basis_grad_complex_step():
    net, pts, mu = tiny_case(n=20)
    cfg = {"form": 0, "w_r": 1.0, "w_0": 0.7, "w_b": 1.3}
    gU, gV = orc.lrnr_basis_grad(net, net.s, mu, pts, cfg)
    import copy
    for attr, g in (("U", gU), ("V", gV)):
        mats = getattr(net, attr)
        shapes = [m.shape for m in mats]

        def f(z, attr=attr, shapes=shapes):
            n2 = copy.copy(net)
            out, o = [], 0
            for sh in shapes:
                k = sh[0] * sh[1]
                out.append(z[o:o + k].reshape(sh))
                o += k
            setattr(n2, attr, out)
            return orc.lrnr_loss(n2, net.s, mu, pts, cfg)[0][0]

        c = _complex_step_grad(f, np.concatenate([m.ravel() for m in mats]).astype(np.float64))
        np.testing.assert_allclose(g, c, rtol=1e-10, atol=1e-13)


# ------------------------------------------- snapshot states and POD basis --

def _torch_hidden(net, s_list, xt, drop_bias=None):
    """Hidden states of eq. 2.1 with W^l = U^l diag(s^l) V^lT (eq. 2.2) in
    PyTorch float64; drop_bias = l leaves out b^l (a planted mistake)."""
    torch = pytest.importorskip("torch")
    dt = torch.float64
    z = torch.tensor(np.asarray(xt, np.float64), dtype=dt)
    out = []
    for l in range(net.L - 1):
        W = (torch.tensor(net.U[l], dtype=dt) @ torch.diag(torch.tensor(s_list[l], dtype=dt))
             @ torch.tensor(net.V[l], dtype=dt).T)
        a = torch.nn.functional.linear(z, W)
        if l != drop_bias:
            a = a + torch.tensor(net.b[l], dtype=dt)
        z = torch.sin(a)
        out.append(z.numpy())
    return out


def test_hidden_values_match_torch_textbook_mlp():
    """lrnr_hidden_values (the snapshot states of eq. 2.7) against PyTorch's
    float64 forward of the textbook network, at s and at a perturbed s; the
    comparison separates the oracle from the same forward with any one bias
    left out, so a dropped or misplaced bias fails it."""
    net, pts, _ = tiny_case(seed=13)
    rng = np.random.default_rng(3)
    for s_list in (net.s, [x * (1 + 0.2 * rng.standard_normal(x.shape)) for x in net.s]):
        Z = orc.lrnr_hidden_values(net, s_list, pts.xt_r)
        T = _torch_hidden(net, s_list, pts.xt_r)
        assert len(Z) == net.L - 1
        for z, t in zip(Z, T):
            np.testing.assert_allclose(z, t, rtol=0, atol=1e-13)
        for l in range(net.L - 1):
            Tb = _torch_hidden(net, s_list, pts.xt_r, drop_bias=l)
            assert max(np.abs(z - t).max() for z, t in zip(Z, Tb)) > 1e-3, l


def test_hidden_values_feed_the_output_layer():
    """The last hidden state through the linear output layer of eq. 2.1 is
    the u of the forward jets (which the autograd and complex-step pins fix)."""
    net, pts, _ = tiny_case(seed=14)
    z = orc.lrnr_hidden_values(net, net.s, pts.xt_r)[-1]
    L = net.L
    W = (net.U[L - 1].astype(np.float64) * net.s[L - 1].astype(np.float64)) @ \
        net.V[L - 1].astype(np.float64).T
    u = z @ W.T + net.b[L - 1].astype(np.float64)
    np.testing.assert_allclose(u[:, 0], orc.lrnr_forward_jets(net, net.s, pts.xt_r)[0],
                               rtol=0, atol=1e-13)


def test_pod_basis_is_the_leading_singular_subspace_in_order():
    """Eckart-Young: the projection on the leading r_hat left singular
    vectors leaves exactly the trailing singular values, ||Z - Xi Xi^T Z||_F^2
    = sum_{j > r_hat} sigma_j^2, and column j alone carries sigma_j
    (||xi_j^T Z|| = sigma_j, descending), with the singular values from
    scipy's svdvals.  Trailing or reordered vectors fail both checks."""
    from scipy.linalg import svdvals
    rng = np.random.default_rng(21)
    # distinct, decaying singular values (as the snapshot matrices have)
    A = np.linalg.qr(rng.standard_normal((40, 40)))[0]
    B = np.linalg.qr(rng.standard_normal((300, 40)))[0]
    Z = (A * np.geomspace(10.0, 1e-3, 40)) @ B.T
    Z += 1e-6 * rng.standard_normal(Z.shape)
    sv = svdvals(Z)

    def check(Xi, r):
        res = np.linalg.norm(Z - Xi @ (Xi.T @ Z)) ** 2
        ok_tail = abs(res - np.sum(sv[r:] ** 2)) <= 1e-9 * np.sum(sv ** 2)
        ok_cols = np.allclose(np.linalg.norm(Xi.T @ Z, axis=1), sv[:r], rtol=1e-9)
        return ok_tail and ok_cols

    for r in (1, 5, 16, 40):
        Xi = orc.pod_basis(Z, r)
        assert Xi.shape == (40, r)
        np.testing.assert_allclose(Xi.T @ Xi, np.eye(r), atol=1e-12)
        assert check(Xi, r), r
    # planted mistakes: trailing singular vectors, or the leading ones out of order
    u = np.linalg.svd(Z, full_matrices=False)[0]
    assert not check(u[:, -8:], 8)
    assert not check(u[:, [1, 0, 2, 3, 4, 5, 6, 7]], 8)


# ----------------------------------------------------- truncation (Section 4)

def _trunc_case(seed=11):
    """Small net, a hypernetwork whose last layer sends some outputs to
    clearly negative pre-activations for every mu (row of W_K zero, c_K = -5):
    those coefficients are zero at every parameter, the others positive."""
    w = wl.small_lrnr(0, 512)
    H = [3, 16, 16, sum(w.net.r)]
    theta = wl.hyper_init(H, seed=7).astype(np.float64)
    layers = orc.hyper_unpack(H, theta)
    WK, cK = layers[-1]
    dead = np.zeros(H[-1], bool)
    dead[[3, 5, 6, 9, 10, 11, 12, 13, 14, 15, 16, 17]] = True   # layer 2 keeps 1 (index 2)
    # (layer blocks of the flat s: [0,2) [2,10) [10,18) [18,26) [26,27))
    WK[dead, :] = 0.0
    cK[dead] = -5.0
    cK[~dead] = np.abs(cK[~dead]) + 2.0
    theta = np.concatenate([np.concatenate([W.ravel(), c]) for W, c in layers])
    mus = wl.make_mu(np.random.Generator(np.random.PCG64(seed)), 6).astype(np.float64)
    return w, H, theta, mus, dead


def test_truncate_drops_the_zero_coefficients_and_keeps_one_per_layer():
    w, H, theta, mus, dead = _trunc_case()
    t = orc.truncate(w.net, H, theta, mus)
    # hand count per layer (r = 2, 8, 8, 8, 1): layer 1 keeps 2; layer 2 drops
    # indices 3, 5, 6, 9 -> keeps 2, 4, 7, 8; layer 3 (10..17) loses all and
    # keeps its first; layer 4 and the output keep everything
    assert t["r"] == [2, 4, 1, 8, 1]
    expect = ~dead
    expect[10] = True
    assert np.array_equal(t["keep"], expect)
    assert t["H"] == H[:-1] + [16]
    for l, (u, v) in enumerate(zip(t["U"], t["V"])):
        assert u.shape == (w.net.M[l + 1], t["r"][l]) and v.shape == (w.net.M[l], t["r"][l])


def test_truncated_net_and_hypernetwork_reproduce_the_full_ones():
    """Exactness: the dropped coefficients are zero at every sampled mu, so
    U^l diag(s^l) V^lT is unchanged and the truncated hypernetwork's outputs
    are the full one's kept outputs: loss and jets agree to rounding."""
    w, H, theta, mus, dead = _trunc_case()
    t = orc.truncate(w.net, H, theta, mus)
    s_full, _ = orc.hyper_forward(H, theta, mus)
    s_tr, _ = orc.hyper_forward(t["H"], t["theta"], mus)
    assert np.array_equal(s_tr, s_full[:, t["keep"]])
    assert np.all(s_full[:, ~t["keep"]] == 0.0)
    net_t = wl.Net(M=w.net.M, r=t["r"], U=t["U"], V=t["V"], b=t["b"], s=[])
    for b in range(len(mus)):
        sf = w.net.split_s(s_full[b])
        st = net_t.split_s(s_tr[b])
        lf, gf, _ = orc.lrnr_loss(w.net, sf, mus[b], w.pts, {}, with_grad=True)
        lt, gt, _ = orc.lrnr_loss(net_t, st, mus[b], w.pts, {}, with_grad=True)
        np.testing.assert_allclose(lt, lf, rtol=1e-12, atol=0)
        # the kept coefficients' gradients are the full net's at those indices
        np.testing.assert_allclose(gt, gf[t["keep"]], rtol=1e-10, atol=1e-12 * np.abs(gf).max())
        jf = orc.lrnr_forward_jets(w.net, sf, w.pts.xt_r[:64])
        jt = orc.lrnr_forward_jets(net_t, st, w.pts.xt_r[:64])
        np.testing.assert_allclose(jt, jf, rtol=1e-11, atol=1e-12 * np.abs(jf).max())


def test_truncate_keeps_everything_when_no_output_vanishes():
    w = wl.small_lrnr(0, 64)
    H = [3, 8, sum(w.net.r)]
    theta = wl.hyper_init(H, seed=3).astype(np.float64)
    layers = orc.hyper_unpack(H, theta)
    layers[-1][0][:] = 0.0          # outputs = c_K in [0.5, 1.5): all positive
    theta = np.concatenate([np.concatenate([W.ravel(), c]) for W, c in layers])
    t = orc.truncate(w.net, H, theta, np.array([[1.0, 0.5, 0.5]]))
    assert t["r"] == list(w.net.r) and t["keep"].all()
    assert np.array_equal(t["theta"], theta)
