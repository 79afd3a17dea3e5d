"""FP64 CPU oracle for the LRNR / FastLRNR physics-informed hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports or calls this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` do.  It shares no code with the HIP path: its inputs come
from the seeded generators in ``workloads`` (FP32 arrays, upcast here).

Everything is plain numpy in float64 (or complex128 when a test feeds complex
inputs for complex-step differentiation: every function below is written so
that it stays analytic in its inputs).

Paper passages followed (arXiv 2410.04001):
  * Section 2.1, eq. (2.1): feed-forward network z^l = sigma(W^l z^{l-1} + b^l),
    linear last layer.
  * Section 2.1, eq. (2.2): W^l = U^l diag(s^l) V^lT.  V^l is read as
    [M_{l-1}][r_l] so that the product has the shape of W^l.
  * Section 2.2, eq. (2.6)-(2.8): FastLRNR, z_hat^l = zeta^l(s^l * z_hat^{l-1}),
    zeta^l(y) = V_hat^{(l+1)T} sigma(U_hat^l y + b_hat^l), output
    U^L (s^L * z_hat^{L-1}) + b^L; the input layer is reduced trivially by V^1.
  * Section 2.2, eq. (2.7): EIM/DEIM, U_hat = P^T U, V_hat^{l+1} read as
    (V^{(l+1)T} Xi (P^T Xi)^{-1})^T, b_hat = P^T b.
  * Section 3.2, eq. (3.5): mean-squared physics-informed loss; eq. (3.6): the
    l1 form; eq. (3.7): locality term lambda * sum |s - s_ref|.
  * Section 4, eq. (4.1): N[u; mu] = u_t + mu_1 u_x - mu_2 u_xx - mu_3 u (1 - u),
    u(x, 0) = sin x, u(0, t) = u(2 pi, t).
  * sigma = sin (the paper leaves sigma open; the workload fixes it).
  * Section 2.1 (remark on the biases): factored biases b^l = B^l s_b^l.
  * Section 3.1, eq. (3.1)-(3.4): hypernetwork s = f_hyper(mu; Theta), meta
    loss over parameter samples, R_sparse (bases held fixed).
  * Section 4 (meta-learning run): truncation of the coefficients that the
    hypernetwork sets to zero, with the matching columns of U and V.

The two networks are computed by two different routes on purpose: LRNR by the
dense route (form W^l explicitly, run eq. 2.1), FastLRNR by the reduced chain
of eq. 2.8.  With the full index set the two must agree, which pins both.
"""
from __future__ import annotations

import contextlib
import math

import numpy as np

TWO_PI = 2.0 * math.pi
JETS = ("v", "x", "t", "xx")


# Real type of the oracle's arithmetic: float64.  ``working_precision`` can
# switch it for a test that needs the rounding floor of the same chain in
# float32 (how far an FP32 evaluation of these formulas lands from the
# float64 one); the oracle proper never runs in anything but float64.
_REAL = np.float64


@contextlib.contextmanager
def working_precision(dtype):
    """Run the oracle's real arithmetic in ``dtype`` inside the block."""
    global _REAL
    old, _REAL = _REAL, np.dtype(dtype).type
    try:
        yield
    finally:
        _REAL = old


def _f(a):
    """Upcast an FP32 input to float64 (complex inputs stay complex)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return a.astype(np.complex128)
    return a.astype(_REAL)


def _sgn(x):
    """Subgradient of |x| with sign(0) = 0."""
    return np.sign(x)


# --------------------------------------------------------------------------
# Activation jets: z = sigma(a) with sigma = sin, differentiated by the chain
# rule for the x-, t- and xx-components of a point's jet.
# --------------------------------------------------------------------------

def sigma_jets(a):
    """a: dict of jet components -> z jets (eq. 2.1 with sigma = sin)."""
    sn, cs = np.sin(a["v"]), np.cos(a["v"])
    return {
        "v": sn,
        "x": cs * a["x"],
        "t": cs * a["t"],
        "xx": -sn * a["x"] * a["x"] + cs * a["xx"],
    }


def sigma_jets_adjoint(a, zbar):
    """Reverse of ``sigma_jets``: adjoints of the a-jets from those of the z-jets."""
    sn, cs = np.sin(a["v"]), np.cos(a["v"])
    ax, at, axx = a["x"], a["t"], a["xx"]
    return {
        "v": cs * zbar["v"] - sn * ax * zbar["x"] - sn * at * zbar["t"]
             + (-cs * ax * ax - sn * axx) * zbar["xx"],
        "x": cs * zbar["x"] - 2.0 * sn * ax * zbar["xx"],
        "t": cs * zbar["t"],
        "xx": cs * zbar["xx"],
    }


def input_jets(xt):
    """Jets of z^0 = (x, t): value, d/dx = (1, 0), d/dt = (0, 1), d2/dx2 = 0."""
    xt = _f(xt)
    n = xt.shape[0]
    one = np.zeros((n, 2), dtype=xt.dtype)
    ex, et = one.copy(), one.copy()
    ex[:, 0] = 1.0
    et[:, 1] = 1.0
    return {"v": xt, "x": ex, "t": et, "xx": one.copy()}


# --------------------------------------------------------------------------
# LRNR: dense route (eq. 2.1 with W^l = U^l diag(s^l) V^lT from eq. 2.2)
# --------------------------------------------------------------------------

def dense_weights(U, s, V):
    """W^l = U^l diag(s^l) V^lT for every layer (eq. 2.2)."""
    return [_f(u) @ np.diag(_f(sl)) @ _f(v).T for u, sl, v in zip(U, s, V)]


def mlp_forward(W, b, xt):
    """Run eq. 2.1 with jets; returns the output jets and the per-layer caches."""
    L = len(W)
    z = input_jets(xt)
    cache = []
    for l in range(L - 1):
        a = {c: z[c] @ W[l].T for c in JETS}
        a["v"] = a["v"] + _f(b[l])[None, :]
        cache.append((z, a))
        z = sigma_jets(a)
    u = {c: z[c] @ W[L - 1].T for c in JETS}
    u["v"] = u["v"] + _f(b[L - 1])[None, :]
    cache.append((z, None))
    return {c: u[c][:, 0] for c in JETS}, cache


def mlp_backward(W, cache, ubar):
    """Hand reverse mode of ``mlp_forward``: dL/dW^l and dL/db^l from the
    per-point adjoints of the output jets."""
    L = len(W)
    gW, gb = [None] * L, [None] * L
    zprev, _ = cache[L - 1]
    ub = {c: _f(ubar[c])[:, None] for c in JETS}
    gW[L - 1] = sum(ub[c].T @ zprev[c] for c in JETS)
    gb[L - 1] = ub["v"].sum(axis=0)
    zbar = {c: ub[c] @ W[L - 1] for c in JETS}
    for l in range(L - 2, -1, -1):
        zprev, a = cache[l]
        abar = sigma_jets_adjoint(a, zbar)
        gW[l] = sum(abar[c].T @ zprev[c] for c in JETS)
        gb[l] = abar["v"].sum(axis=0)
        zbar = {c: abar[c] @ W[l] for c in JETS}
    return gW, gb


def grad_s_from_dense(gW, U, V):
    """Chain rule through eq. 2.2: dL/ds^l_k = sum_mn dL/dW_mn U_mk V_nk."""
    return [np.einsum("mn,mk,nk->k", g, _f(u), _f(v)) for g, u, v in zip(gW, U, V)]


# --------------------------------------------------------------------------
# PDE residual, boundary terms and loss (eq. 4.1, 3.5-3.7)
# --------------------------------------------------------------------------

def residual(u, ux, ut, uxx, mu):
    """N[u; mu] = u_t + mu_1 u_x - mu_2 u_xx - mu_3 u (1 - u)  (eq. 4.1)."""
    b_, n_, r_ = (_f(m) for m in mu)
    return ut + b_ * ux - n_ * uxx - r_ * u * (1.0 - u)


def residual_adjoint(u, mu, g):
    """Adjoints of the output jets for a residual adjoint g (per point)."""
    b_, n_, r_ = (_f(m) for m in mu)
    return {"v": -r_ * (1.0 - 2.0 * u) * g, "x": b_ * g, "t": g, "xx": -n_ * g}


def _phi(x, form):
    return x * x if form == 0 else np.abs(x)


def _dphi(x, form):
    return 2.0 * x if form == 0 else _sgn(x)


def loss_points(pts):
    """Evaluation points of one loss: interior, initial line t = 0, and the
    two periodic boundary lines x = 0 and x = 2 pi (eq. 4.1)."""
    xt_r = _f(pts.xt_r)
    x0 = _f(pts.x_0)
    tb = _f(pts.t_b)
    ic = np.stack([x0, np.zeros_like(x0)], axis=1)
    bl = np.stack([np.zeros_like(tb), tb], axis=1)
    br = np.stack([np.full_like(tb, TWO_PI), tb], axis=1)
    return xt_r, ic, bl, br


def _loss_and_ubar(jets, n_r, n_0, n_b, x0, mu, cfg):
    """Loss terms (means, eq. 3.5 / 3.6) and per-point output adjoints."""
    form = cfg.get("form", 0)
    w_r, w_0, w_b = cfg.get("w_r", 1.0), cfg.get("w_0", 1.0), cfg.get("w_b", 1.0)
    u = jets["v"]
    ur, ic, bl, br = (slice(0, n_r), slice(n_r, n_r + n_0),
                      slice(n_r + n_0, n_r + n_0 + n_b), slice(n_r + n_0 + n_b, None))
    res = residual(u[ur], jets["x"][ur], jets["t"][ur], jets["xx"][ur], mu)
    e0 = u[ic] - np.sin(x0)
    eb = u[bl] - u[br]
    terms = [
        w_r / max(n_r, 1) * _phi(res, form).sum() if n_r else 0.0,
        w_0 / max(n_0, 1) * _phi(e0, form).sum() if n_0 else 0.0,
        w_b / max(n_b, 1) * _phi(eb, form).sum() if n_b else 0.0,
    ]
    n_all = u.shape[0]
    dt = np.result_type(u, _REAL)
    ubar = {c: np.zeros(n_all, dt) for c in JETS}
    if n_r:
        g = w_r / n_r * _dphi(res, form)
        ra = residual_adjoint(u[ur], mu, g)
        for c in JETS:
            ubar[c][ur] = ra[c]
    if n_0:
        ubar["v"][ic] = w_0 / n_0 * _dphi(e0, form)
    if n_b:
        gb = w_b / n_b * _dphi(eb, form)
        ubar["v"][bl] = gb
        ubar["v"][br] = -gb
    return terms, ubar


def _loc_term(s_list, cfg):
    lam = cfg.get("lambda_loc", 0.0)
    sref = cfg.get("s_ref", None)
    if lam == 0.0 or sref is None:
        return 0.0, [np.zeros(len(x)) for x in s_list]
    val, grad, o = 0.0, [], 0
    for sl in s_list:
        d = _f(sl) - _f(sref[o:o + len(sl)])
        val = val + lam * np.abs(d).sum()
        grad.append(lam * _sgn(d))
        o += len(sl)
    return val, grad


def _all_points(pts):
    xt_r, ic, bl, br = loss_points(pts)
    return np.concatenate([xt_r, ic, bl, br], axis=0), len(xt_r), len(ic), len(bl)


# --------------------------------------------------------------------------
# LRNR public functions
# --------------------------------------------------------------------------

def lrnr_forward_jets(net, s_list, xt):
    """u, u_x, u_t, u_xx at the points xt ([n][2]); returns [4][n]."""
    W = dense_weights(net.U, s_list, net.V)
    jets, _ = mlp_forward(W, net.b, xt)
    return np.stack([jets[c] for c in JETS])


def lrnr_jets_vjp(net, s_list, xt, cot):
    """Vector-Jacobian product of the forward jets: the gradients w.r.t. s
    (flat) and b (flat) of sum_i sum_c cot[c][i] * jet_c(x_i), with cot [4][n]
    in the order u, u_x, u_t, u_xx (chain rule through eq. 2.1-2.2)."""
    W = dense_weights(net.U, s_list, net.V)
    jets, cache = mlp_forward(W, net.b, xt)
    cot = _f(np.asarray(cot))
    ubar = {c: cot[k] for k, c in enumerate(JETS)}
    gW, gb = mlp_backward(W, cache, ubar)
    gs = grad_s_from_dense(gW, net.U, net.V)
    return np.concatenate(gs), np.concatenate(gb)


def lrnr_hidden_values(net, s_list, xt):
    """Post-activation hidden states z^l (values only) at the points: list of
    [n][M_l] for l = 1..L-1 (snapshot data of eq. 2.7)."""
    W = dense_weights(net.U, s_list, net.V)
    z = _f(xt)
    out = []
    for l in range(len(W) - 1):
        z = np.sin(z @ W[l].T + _f(net.b[l])[None, :])
        out.append(z)
    return out


def lrnr_loss(net, s_list, mu, pts, cfg=None, with_grad=False):
    """Physics-informed loss of the LRNR (eq. 3.5 / 3.6 / 3.7) and, when
    ``with_grad``, its gradients w.r.t. s (flat) and b (flat).

    Returns (loss4, grad_s, grad_b) with loss4 = [total, interior, ic, bc]."""
    cfg = cfg or {}
    W = dense_weights(net.U, s_list, net.V)
    X, n_r, n_0, n_b = _all_points(pts)
    jets, cache = mlp_forward(W, net.b, X)
    terms, ubar = _loss_and_ubar(jets, n_r, n_0, n_b, _f(pts.x_0), mu, cfg)
    loc, gloc = _loc_term(s_list, cfg)
    loss4 = np.array([terms[0] + terms[1] + terms[2] + loc] + terms)
    if not with_grad:
        return loss4, None, None
    gW, gb = mlp_backward(W, cache, ubar)
    gs = grad_s_from_dense(gW, net.U, net.V)
    gs = [g + h for g, h in zip(gs, gloc)]
    return loss4, np.concatenate(gs), np.concatenate(gb)


def lrnr_loss_chunked(net, s_list, mu, pts, cfg=None, chunk=16384):
    """``lrnr_loss(with_grad=True)`` for large point sets: the loss and its
    gradients are sums over points, so they are accumulated over point chunks
    (interior, initial and boundary points chunked alike)."""
    from workloads import Points  # generator container only
    cfg = dict(cfg or {})
    n_r, n_0, n_b = len(pts.xt_r), len(pts.x_0), len(pts.t_b)
    nchunks = max(1, math.ceil(max(n_r, n_0, n_b) / chunk))
    tot4, tgs, tgb = None, None, None
    lam = cfg.get("lambda_loc", 0.0)
    for i in range(nchunks):
        def sl(n):
            per = math.ceil(n / nchunks)
            return slice(i * per, min(n, (i + 1) * per))
        sub = Points(pts.xt_r[sl(n_r)], pts.x_0[sl(n_0)], pts.t_b[sl(n_b)])
        m_r, m_0, m_b = len(sub.xt_r), len(sub.x_0), len(sub.t_b)
        c2 = dict(cfg)
        c2["lambda_loc"] = 0.0
        # weights rescaled so that every chunk's means add up to the full means
        c2["w_r"] = cfg.get("w_r", 1.0) * (m_r / n_r if n_r else 0.0)
        c2["w_0"] = cfg.get("w_0", 1.0) * (m_0 / n_0 if n_0 else 0.0)
        c2["w_b"] = cfg.get("w_b", 1.0) * (m_b / n_b if n_b else 0.0)
        l4, gs, gb = lrnr_loss(net, s_list, mu, sub, c2, with_grad=True)
        tot4 = l4 if tot4 is None else tot4 + l4
        tgs = gs if tgs is None else tgs + gs
        tgb = gb if tgb is None else tgb + gb
    if lam != 0.0:
        loc, gloc = _loc_term(s_list, cfg)
        tot4[0] += loc
        tgs = tgs + np.concatenate(gloc)
    return tot4, tgs, tgb


# --------------------------------------------------------------------------
# FastLRNR construction (eq. 2.7) and reduced chain (eq. 2.8)
# --------------------------------------------------------------------------

def pod_basis(Z, r_hat):
    """Xi: the leading r_hat left singular vectors of the snapshot matrix Z
    ([M][n_snap]), in descending singular-value order."""
    u, _, _ = np.linalg.svd(_f(Z), full_matrices=False)
    return u[:, :r_hat]


def deim_indices(Xi):
    """Greedy DEIM selection (Chaturantabut & Sorensen 2010): the first index
    maximises |xi_1|; each next index maximises the residual of interpolating
    the next basis vector at the indices chosen so far.  Ties go to the
    smallest index."""
    Xi = _f(Xi)
    m = Xi.shape[1]
    P = [int(np.argmax(np.abs(Xi[:, 0])))]
    for j in range(1, m):
        c = np.linalg.solve(Xi[P, :j], Xi[P, j])
        res = Xi[:, j] - Xi[:, :j] @ c
        P.append(int(np.argmax(np.abs(res))))
    return np.array(P, dtype=np.int64)


def qdeim_indices(Xi):
    """Q-DEIM (Drmac & Gugercin 2016): the first r indices of a column-pivoted
    QR factorisation of Xi^T.  Written as modified Gram-Schmidt on the rows of
    Xi: each step takes the row of largest remaining 2-norm (ties to the
    smallest index) and removes its direction from every row."""
    W = _f(Xi).copy()
    M, r = W.shape
    picked = np.zeros(M, dtype=bool)
    P = []
    for _ in range(r):
        nrm = np.where(picked, 0.0, np.sum(W * W, axis=1))
        p = int(np.argmax(nrm))
        if not nrm[p] > 0.0:
            raise np.linalg.LinAlgError("Q-DEIM: no row with a nonzero remaining norm")
        q = W[p] / np.sqrt(nrm[p])
        W -= np.outer(W @ q, q)
        picked[p] = True
        P.append(p)
    return np.array(P, dtype=np.int64)


def fast_operators(net, P_list, Xi_list):
    """Reduced operators of eq. 2.7 for every hidden layer l = 1..L-1:
    U_hat^l = P^T U^l, b_hat^l = P^T b^l,
    V_hat^{l+1} = (V^{(l+1)T} Xi^l (P^T Xi^l)^{-1})^T  ([r_hat_l][r_{l+1}])."""
    Uh, bh, Vh = [], [], []
    for l, (P, Xi) in enumerate(zip(P_list, Xi_list)):
        Xi = _f(Xi)
        Uh.append(_f(net.U[l])[P, :])
        bh.append(_f(net.b[l])[P])
        Vt = _f(net.V[l + 1]).T @ Xi @ np.linalg.inv(Xi[P, :])
        Vh.append(Vt.T)
    return Uh, bh, Vh


def fastlrnr_build(net, s_snap_list, xt_snap, r_hat, P_override=None, selection="deim"):
    """Snapshots of the hidden states at the snapshot points, POD basis, DEIM
    (or, with selection="qdeim", Q-DEIM) indices and reduced operators.
    ``s_snap_list`` is a list of coefficient vectors (each a per-layer list).
    ``P_override`` replaces the picks (used to compare against a selection
    made elsewhere)."""
    L = net.L
    if np.isscalar(r_hat):
        r_hat = [int(r_hat)] * (L - 1)
    Zs = [[] for _ in range(L - 1)]
    for s_list in s_snap_list:
        for l, z in enumerate(lrnr_hidden_values(net, s_list, xt_snap)):
            Zs[l].append(z.T)
    Xi_list, P_list = [], []
    for l in range(L - 1):
        Z = np.concatenate(Zs[l], axis=1)
        Xi = pod_basis(Z, r_hat[l])
        if P_override is not None:
            P = np.asarray(P_override[l])
        else:
            P = qdeim_indices(Xi) if selection == "qdeim" else deim_indices(Xi)
        Xi_list.append(Xi)
        P_list.append(P)
    Uh, bh, Vh = fast_operators(net, P_list, Xi_list)
    return {"P": P_list, "Xi": Xi_list, "U_hat": Uh, "b_hat": bh, "V_hat": Vh}


def fast_forward(net, fast, s_list, xt):
    """Eq. 2.8 with jets: z_hat^0 = V^1T z^0, then
    z_hat^l = V_hat^{(l+1)T} sigma(U_hat^l (s^l * z_hat^{l-1}) + b_hat^l),
    output U^L (s^L * z_hat^{L-1}) + b^L."""
    L = net.L
    z0 = input_jets(xt)
    zh = {c: z0[c] @ _f(net.V[0]) for c in JETS}
    cache = []
    for l in range(L - 1):
        w = {c: _f(s_list[l])[None, :] * zh[c] for c in JETS}
        a = {c: w[c] @ _f(fast["U_hat"][l]).T for c in JETS}
        a["v"] = a["v"] + _f(fast["b_hat"][l])[None, :]
        h = sigma_jets(a)
        cache.append((zh, a))
        zh = {c: h[c] @ _f(fast["V_hat"][l]) for c in JETS}
    w = {c: _f(s_list[L - 1])[None, :] * zh[c] for c in JETS}
    u = {c: w[c] @ _f(net.U[L - 1]).T for c in JETS}
    u["v"] = u["v"] + _f(net.b[L - 1])[None, :]
    cache.append((zh, None))
    return {c: u[c][:, 0] for c in JETS}, cache


def fast_backward(net, fast, s_list, cache, ubar):
    """Hand reverse mode of ``fast_forward`` to s (per layer) and b_hat."""
    L = net.L
    gs, gb = [None] * L, [None] * L
    zh, _ = cache[L - 1]
    UL = _f(net.U[L - 1])
    wbar = {c: _f(ubar[c])[:, None] @ UL for c in JETS}
    gs[L - 1] = sum((wbar[c] * zh[c]).sum(axis=0) for c in JETS)
    gb[L - 1] = _f(ubar["v"]).sum(keepdims=True)
    zhbar = {c: _f(s_list[L - 1])[None, :] * wbar[c] for c in JETS}
    for l in range(L - 2, -1, -1):
        zh_prev, a = cache[l]
        hbar = {c: zhbar[c] @ _f(fast["V_hat"][l]).T for c in JETS}
        abar = sigma_jets_adjoint(a, hbar)
        gb[l] = abar["v"].sum(axis=0)
        wbar = {c: abar[c] @ _f(fast["U_hat"][l]) for c in JETS}
        gs[l] = sum((wbar[c] * zh_prev[c]).sum(axis=0) for c in JETS)
        zhbar = {c: _f(s_list[l])[None, :] * wbar[c] for c in JETS}
    return gs, gb


def fast_forward_jets(net, fast, s_list, xt):
    jets, _ = fast_forward(net, fast, s_list, xt)
    return np.stack([jets[c] for c in JETS])


def fast_loss(net, fast, s_list, mu, pts, cfg=None, with_grad=False):
    """FastLRNR physics-informed loss and gradient w.r.t. s (flat)."""
    cfg = cfg or {}
    X, n_r, n_0, n_b = _all_points(pts)
    jets, cache = fast_forward(net, fast, s_list, X)
    terms, ubar = _loss_and_ubar(jets, n_r, n_0, n_b, _f(pts.x_0), mu, cfg)
    loc, gloc = _loc_term(s_list, cfg)
    loss4 = np.array([terms[0] + terms[1] + terms[2] + loc] + terms)
    if not with_grad:
        return loss4, None
    gs, _ = fast_backward(net, fast, s_list, cache, ubar)
    gs = [g + h for g, h in zip(gs, gloc)]
    return loss4, np.concatenate(gs)


# --------------------------------------------------------------------------
# Factored biases (the variant the paper notes in Section 2.1 and does not
# use: the bias treated like the weights, so that it is driven by
# coefficients too).  Reading: b^l = B^l s_b^l with a basis B^l [M_l][q_l]
# and coefficients s_b^l [q_l]; the rest of the network is unchanged, so the
# gradient to s_b follows from the bias gradient by the chain rule.
# --------------------------------------------------------------------------

def bias_from_basis(B_list, sb_list):
    """b^l = B^l s_b^l for every layer."""
    return [_f(B) @ _f(sb) for B, sb in zip(B_list, sb_list)]


def _split(v, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(v[o:o + n])
        o += n
    return out


def lrnr_loss_factored_bias(net, s_list, B_list, sb_list, mu, pts, cfg=None, with_grad=False):
    """LRNR loss with factored biases; returns (loss4, grad_s, grad_sb) with
    grad_sb^l = B^lT (dL/db^l), flat over layers."""
    import copy
    n2 = copy.copy(net)
    n2.b = bias_from_basis(B_list, sb_list)
    loss4, gs, gb = lrnr_loss(n2, s_list, mu, pts, cfg, with_grad)
    if not with_grad:
        return loss4, None, None
    gbl = _split(gb, [len(x) for x in n2.b])
    gsb = np.concatenate([_f(B).T @ g for B, g in zip(B_list, gbl)])
    return loss4, gs, gsb


def fast_loss_factored_bias(net, fast, s_list, B_list, sb_list, mu, pts, cfg=None,
                            with_grad=False):
    """FastLRNR loss with factored biases: the reduced bias of hidden layer l
    is P^lT B^l s_b^l (the rows of the basis at the interpolation indices,
    eq. 2.7 applied to b = B s_b), the output bias B^L s_b^L; returns
    (loss4, grad_s, grad_sb)."""
    import copy
    L = net.L
    Bh = [_f(B_list[l])[np.asarray(fast["P"][l]), :] for l in range(L - 1)] + [_f(B_list[L - 1])]
    bh = bias_from_basis(Bh, sb_list)
    f2 = dict(fast)
    f2["b_hat"] = bh[:L - 1]
    n2 = copy.copy(net)
    n2.b = list(net.b[:L - 1]) + [bh[L - 1]]
    cfg = cfg or {}
    X, n_r, n_0, n_b = _all_points(pts)
    jets, cache = fast_forward(n2, f2, s_list, X)
    terms, ubar = _loss_and_ubar(jets, n_r, n_0, n_b, _f(pts.x_0), mu, cfg)
    loc, gloc = _loc_term(s_list, cfg)
    loss4 = np.array([terms[0] + terms[1] + terms[2] + loc] + terms)
    if not with_grad:
        return loss4, None, None
    gs, gb = fast_backward(n2, f2, s_list, cache, ubar)
    gs = [g + h for g, h in zip(gs, gloc)]
    gsb = np.concatenate([B.T @ g for B, g in zip(Bh, gb)])
    return loss4, np.concatenate(gs), gsb


# --------------------------------------------------------------------------
# Meta-learning of the coefficient map and the biases (Section 3.1,
# eq. 3.1-3.4) with the bases U, V held fixed: the hypernetwork
# s = f_hyper(mu; Theta), the meta loss averaged over parameter samples and
# the sparsity term R_sparse.
# Readings: f_hyper is a network of the form of eq. 2.1 with the same
# activation sigma = sin and a ReLU on its output; Theta is packed per layer
# as W_k [H_k][H_{k-1}] row-major, then c_k [H_k]; the sigma inside R_sparse is
# the ReLU; expectations over mu are means over the sample.
# --------------------------------------------------------------------------

def _relu(x):
    return np.where(np.real(x) > 0, x, 0.0 * x)


def hyper_unpack(H, theta):
    """Theta (flat) -> [(W_k, c_k)] for k = 1..K, widths H[0..K]."""
    out, o = [], 0
    for k in range(1, len(H)):
        W = theta[o:o + H[k] * H[k - 1]].reshape(H[k], H[k - 1])
        o += H[k] * H[k - 1]
        c = theta[o:o + H[k]]
        o += H[k]
        out.append((W, c))
    return out


def hyper_forward(H, theta, mu):
    """s = ReLU(NN(mu)) for mu [B][3]; returns (s [B][H_K], cache)."""
    layers = hyper_unpack(H, _f(theta))
    h = _f(mu)
    pre = []
    for k, (W, c) in enumerate(layers):
        a = h @ W.T + c[None, :]
        pre.append((h, a))
        h = np.sin(a) if k < len(layers) - 1 else a
    return _relu(h), (layers, pre)


def sparse_reg_value(s, r, gamma):
    """Mean over the sample rows of sum_l sum_i ReLU(-s_i^l + gamma s_{i+1}^l)."""
    s = _f(s)
    tot, o = 0.0, 0
    for rl in r:
        sl = s[:, o:o + rl]
        t = -sl[:, :-1] + gamma * sl[:, 1:]
        tot = tot + _relu(t).sum(axis=1)
        o += rl
    return np.mean(tot)


def sparse_reg_grad(s, r, gamma):
    """Per-row gradient of sum_l sum_i ReLU(-s_i + gamma s_{i+1}) w.r.t. s."""
    s = _f(s)
    g = np.zeros_like(s)
    o = 0
    for rl in r:
        sl = s[:, o:o + rl]
        act = (np.real(-sl[:, :-1] + gamma * sl[:, 1:]) > 0).astype(np.float64)
        g[:, o:o + rl - 1] -= act
        g[:, o + 1:o + rl] += gamma * act
        o += rl
    return g


def hyper_backward(H, cache, s_bar):
    """Theta gradient of sum_b <s_bar[b], s[b]> through the ReLU and the network."""
    layers, pre = cache
    K = len(layers)
    h_in, a = pre[K - 1]
    g = _f(s_bar) * (np.real(a) > 0)
    grads = [None] * K
    for k in range(K - 1, -1, -1):
        h_in, a = pre[k]
        W, _ = layers[k]
        if k < K - 1:
            g = g * np.cos(a)
        grads[k] = (g.T @ h_in, g.sum(axis=0))
        g = g @ W
    return np.concatenate([np.concatenate([gW.ravel(), gc]) for gW, gc in grads])


def truncate(net, H, theta, mus):
    """Truncation after meta-learning (Section 4): a coefficient s^l_k whose
    hypernetwork output is zero for every parameter of the sample ``mus``
    ([B][3]) is dropped, with column k of U^l and of V^l and the matching
    output of f_hyper (row k of the last layer's W_K and entry k of c_K); the
    ranks shrink accordingly.  A layer that would lose every coefficient keeps
    its first one (which is zero, so the network is unchanged).  The biases
    and the widths stay.  Returns a dict with the kept mask ``keep``
    ([r_total] bool), the new ranks ``r``, the factor lists ``U``, ``V``,
    ``b``, the hypernetwork widths ``H`` and parameters ``theta``."""
    s, _ = hyper_forward(H, theta, mus)
    alive = np.any(s != 0.0, axis=0)
    keep, o = [], 0
    for rl in net.r:
        k = alive[o:o + rl].copy()
        if not k.any():
            k[0] = True
        keep.append(k)
        o += rl
    U = [np.asarray(u)[:, k] for u, k in zip(net.U, keep)]
    V = [np.asarray(v)[:, k] for v, k in zip(net.V, keep)]
    keep_all = np.concatenate(keep)
    layers = hyper_unpack(H, np.asarray(theta))
    WK, cK = layers[-1]
    layers[-1] = (WK[keep_all, :], cK[keep_all])
    theta_t = np.concatenate([np.concatenate([W.ravel(), c]) for W, c in layers])
    H_t = list(H[:-1]) + [int(keep_all.sum())]
    return {"keep": keep_all, "r": [int(k.sum()) for k in keep], "U": U, "V": V,
            "b": [np.asarray(x) for x in net.b], "H": H_t, "theta": theta_t}


def lrnr_basis_grad(net, s_list, mu, pts, cfg=None):
    """Gradient of the loss with respect to U^l and V^l (flat, packed per
    layer): from the dense weight gradient gW^l of eq. 2.1 and W^l =
    U^l diag(s^l) V^lT (eq. 2.2), dL/dU^l = gW^l V^l diag(s^l) and
    dL/dV^l = gW^lT U^l diag(s^l)."""
    cfg = cfg or {}
    W = dense_weights(net.U, s_list, net.V)
    X, n_r, n_0, n_b = _all_points(pts)
    jets, cache = mlp_forward(W, net.b, X)
    _, ubar = _loss_and_ubar(jets, n_r, n_0, n_b, _f(pts.x_0), mu, cfg)
    gW, _ = mlp_backward(W, cache, ubar)
    gU = [g @ _f(V) * _f(s)[None, :] for g, V, s in zip(gW, net.V, s_list)]
    gV = [g.T @ _f(U) * _f(s)[None, :] for g, U, s in zip(gW, net.U, s_list)]
    return np.concatenate([g.ravel() for g in gU]), np.concatenate([g.ravel() for g in gV])


def orth_reg(U_list, V_list, with_grad=False):
    """R_orth of eq. 3.3: sum_l ||U^lT U^l - I||_F^2 + ||V^lT V^l - I||_F^2.
    With ``with_grad`` also its gradients 4 U (U^T U - I) and 4 V (V^T V - I)
    per layer."""
    val = 0.0
    gU, gV = [], []
    for M in (U_list, V_list):
        for A in M:
            A = _f(A)
            D = A.T @ A - np.eye(A.shape[1])
            val = val + np.sum(D * D)
            if with_grad:
                (gU if M is U_list else gV).append(4.0 * A @ D)
    return (val, gU, gV) if with_grad else val


def meta_objective(net, H, theta, mus, pts, gamma, lam_sparse, cfg=None, with_grad=False,
                   with_b=False):
    """Eq. 3.4 with U and V fixed: mean over the samples mu_b of the
    physics-informed loss of the LRNR at s = f_hyper(mu_b; Theta) on the
    shared points, plus lam_sparse * R_sparse.  Returns (objective, grad
    Theta), and with ``with_b`` also the gradient in the biases b (flat), the
    mean over the samples of dL_b/db."""
    s, cache = hyper_forward(H, theta, mus)
    B = s.shape[0]
    tot = 0.0
    s_bar = np.zeros_like(s)
    g_b = 0.0
    for b in range(B):
        l4, gs, gb = lrnr_loss(net, net.split_s(s[b]), mus[b], pts, cfg, with_grad)
        tot = tot + l4[0] / B
        if with_grad:
            s_bar[b] = gs / B
            g_b = g_b + gb / B
    obj = tot + lam_sparse * sparse_reg_value(s, net.r, gamma)
    if not with_grad:
        return (obj, None, None) if with_b else (obj, None)
    s_bar = s_bar + lam_sparse * sparse_reg_grad(s, net.r, gamma) / B
    g_theta = hyper_backward(H, cache, s_bar)
    return (obj, g_theta, g_b) if with_b else (obj, g_theta)


# --------------------------------------------------------------------------
# Adam (Kingma & Ba 2015), the optimiser of Section 4
# --------------------------------------------------------------------------

def adam_step(s, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update; ``step`` counts from 1."""
    s, g, m, v = _f(s), _f(g), _f(m), _f(v)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return s - lr * mh / (np.sqrt(vh) + eps), m, v
