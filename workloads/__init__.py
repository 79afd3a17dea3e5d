"""Seeded synthetic inputs for the LRNR / FastLRNR hot path.

This module only draws numbers: network factors, collocation points and PDE
parameters.  It holds none of the method's arithmetic, so both the FP64 oracle
(``oracle/``) and the HIP path (``paper_2410_04001_amd``) take their inputs from
here and from nowhere else.

Recipe (fixed draw order, numpy ``Generator(PCG64(seed))``, FP64 draws rounded
to FP32):

1. for l = 1..L: U^l with entries N(0, 1/M_l), then V^l with entries
   N(0, 1/M_{l-1}); each is then column-orthonormalised (QR with the signs
   fixed so that diag(R) > 0, i.e. modified Gram-Schmidt in column order);
2. b^1..b^L with entries N(0, 0.1) (variance 0.1);
3. s^1..s^L with entries U(0.5, 1.5);
4. interior points (x, t) = (2 pi U[0,1), U[0,1)), then initial-condition
   abscissae x_j = 2 pi U[0,1), then boundary times t_k = U[0,1);
5. PDE parameters mu = (beta, nu, rho).

Shapes follow the LRNR factorisation W^l = U^l diag(s^l) V^lT of Section 2.1
(eq. 2.2): U^l is [M_l][r_l], V^l is [M_{l-1}][r_l] (the reading under which
the product has the shape of W^l), b^l is [M_l], s^l is [r_l], with
r_l = min(r, M_{l-1}, M_l).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Net:
    """Per-layer factors of an LRNR, FP32.  Index 0 of each list is layer 1."""

    M: list            # widths M_0..M_L
    r: list            # ranks r_1..r_L (len L)
    U: list            # U^l [M_l][r_l]
    V: list            # V^l [M_{l-1}][r_l]
    b: list            # b^l [M_l]
    s: list            # s^l [r_l]  (initial coefficients)

    @property
    def L(self) -> int:
        return len(self.r)

    @property
    def r_total(self) -> int:
        return int(sum(self.r))

    def s_flat(self) -> np.ndarray:
        return np.concatenate([np.asarray(x, np.float32) for x in self.s])

    def packed(self):
        """Row-major per-layer concatenation used across the C ABI."""
        U = np.concatenate([u.reshape(-1) for u in self.U]).astype(np.float32)
        V = np.concatenate([v.reshape(-1) for v in self.V]).astype(np.float32)
        b = np.concatenate([x.reshape(-1) for x in self.b]).astype(np.float32)
        return U, V, b, self.s_flat()

    def split_s(self, s_flat):
        out, o = [], 0
        for rl in self.r:
            out.append(np.asarray(s_flat[o:o + rl]))
            o += rl
        return out


@dataclass
class Points:
    xt_r: np.ndarray   # [n_r][2] interior (x, t)
    x_0: np.ndarray    # [n_0] initial-condition abscissae (t = 0)
    t_b: np.ndarray    # [n_b] periodic-boundary times (x = 0 and x = 2 pi)


@dataclass
class Workload:
    net: Net
    pts: Points
    mu: np.ndarray                 # [n_mu][3]
    extra: dict = field(default_factory=dict)


def widths(n_hidden: int, width: int) -> list:
    return [2] + [width] * n_hidden + [1]


def ranks(M: list, rank: int) -> list:
    return [min(rank, M[l - 1], M[l]) for l in range(1, len(M))]


def _orthonormal_columns(A: np.ndarray) -> np.ndarray:
    q, rr = np.linalg.qr(A)
    sgn = np.sign(np.diag(rr))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def make_net(rng: np.random.Generator, M: list, r: list) -> Net:
    L = len(r)
    U, V = [], []
    for l in range(1, L + 1):
        u = rng.normal(0.0, math.sqrt(1.0 / M[l]), size=(M[l], r[l - 1]))
        v = rng.normal(0.0, math.sqrt(1.0 / M[l - 1]), size=(M[l - 1], r[l - 1]))
        U.append(_orthonormal_columns(u).astype(np.float32))
        V.append(_orthonormal_columns(v).astype(np.float32))
    b = [rng.normal(0.0, math.sqrt(0.1), size=M[l]).astype(np.float32)
         for l in range(1, L + 1)]
    s = [rng.uniform(0.5, 1.5, size=r[l - 1]).astype(np.float32)
         for l in range(1, L + 1)]
    return Net(M=list(M), r=list(r), U=U, V=V, b=b, s=s)


def make_points(rng: np.random.Generator, n_r: int, n_0: int, n_b: int) -> Points:
    X = rng.random((n_r, 2))
    xt = np.empty((n_r, 2), np.float32)
    xt[:, 0] = (TWO_PI * X[:, 0]).astype(np.float32)
    xt[:, 1] = X[:, 1].astype(np.float32)
    x0 = (TWO_PI * rng.random(n_0)).astype(np.float32)
    tb = rng.random(n_b).astype(np.float32)
    return Points(xt_r=xt, x_0=x0, t_b=tb)


def make_mu(rng: np.random.Generator, n: int) -> np.ndarray:
    """(beta, nu, rho) ~ (U[1,20], U[0,5], U[0,5])."""
    mu = np.empty((n, 3), np.float32)
    mu[:, 0] = rng.uniform(1.0, 20.0, n)
    mu[:, 1] = rng.uniform(0.0, 5.0, n)
    mu[:, 2] = rng.uniform(0.0, 5.0, n)
    return mu


def uniform_points(rng: np.random.Generator, n: int) -> np.ndarray:
    X = rng.random((n, 2))
    xt = np.empty((n, 2), np.float32)
    xt[:, 0] = (TWO_PI * X[:, 0]).astype(np.float32)
    xt[:, 1] = X[:, 1].astype(np.float32)
    return xt


def grid_points(nx: int = 256, nt: int = 100) -> np.ndarray:
    """Evaluation grid x_i = 2 pi i / nx, t_j = j / (nt - 1), t-major [nt*nx][2]."""
    x = (TWO_PI * np.arange(nx) / nx)
    t = np.arange(nt) / (nt - 1)
    T, X = np.meshgrid(t, x, indexing="ij")
    return np.stack([X.reshape(-1), T.reshape(-1)], axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def small_lrnr(seed: int = 0, n: int = 4096) -> Workload:
    """Plain LRNR parity case: 4 hidden layers of width 64, rank 8, N points,
    convection residual with beta = 10 (nu = rho = 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = widths(4, 64)
    net = make_net(rng, M, ranks(M, 8))
    pts = make_points(rng, n, n // 8, n // 8)
    mu = np.array([[10.0, 0.0, 0.0]], np.float32)
    return Workload(net, pts, mu)


def big_lrnr(seed: int = 1, n: int = 262144) -> Workload:
    """Full LRNR at working size: 5 hidden layers of width 256, rank 20, N
    points, full CDR residual with 8 parameter draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = widths(5, 256)
    net = make_net(rng, M, ranks(M, 20))
    pts = make_points(rng, n, n // 8, n // 8)
    mu = make_mu(rng, 8)
    return Workload(net, pts, mu)


def fast_case(seed: int = 2, n: int = 65536, n_snap: int = 2048, r_hat: int = 32) -> Workload:
    """FastLRNR comparison: the small LRNR net drawn from seed 0, snapshot
    points and collocation points drawn from ``seed``."""
    net = small_lrnr(0, 16).net
    rng = np.random.Generator(np.random.PCG64(seed))
    xt_snap = uniform_points(rng, n_snap)
    pts = make_points(rng, n, n // 8, n // 8)
    mu = make_mu(rng, 1)
    return Workload(net, pts, mu, extra={"xt_snap": xt_snap, "r_hat": r_hat})


def equal_accuracy_case(big: bool = False, seed: int = 2, n: int = 65536,
                        n_snap: int = 2048, r_hat: int = 32) -> Workload:
    """FastLRNR against LRNR at equal residual accuracy: the small net (or,
    with ``big``, the 256-wide rank-20 net) with snapshot points, training
    points, one parameter draw and a held-out point set of the same size,
    all drawn from ``seed`` in that order."""
    net = (big_lrnr(1, 16) if big else small_lrnr(0, 16)).net
    rng = np.random.Generator(np.random.PCG64(seed))
    xt_snap = uniform_points(rng, n_snap)
    pts = make_points(rng, n, n // 8, n // 8)
    mu = make_mu(rng, 1)
    held = make_points(rng, n, n // 8, n // 8)
    return Workload(net, pts, mu, extra={"xt_snap": xt_snap, "r_hat": r_hat, "heldout": held})


def batched_case(seed: int = 3, n_inst: int = 64, n: int = 16384) -> Workload:
    """Many-instance case: the small net, n_inst parameter draws sharing one
    point set of n interior points."""
    net = small_lrnr(0, 16).net
    rng = np.random.Generator(np.random.PCG64(seed))
    xt_snap = uniform_points(rng, 2048)
    pts = make_points(rng, n, n // 8, n // 8)
    mu = make_mu(rng, n_inst)
    return Workload(net, pts, mu, extra={"xt_snap": xt_snap, "r_hat": 32})


def instances_case(seed: int = 3, n_inst: int = 64, n: int = 16384) -> Workload:
    """Differentiation form: the small net, n_inst parameter draws, each
    instance with its own n interior points and n/8 initial / boundary points.
    extra['pts'] holds the per-instance Points; ``pts`` is instance 0's."""
    net = small_lrnr(0, 16).net
    rng = np.random.Generator(np.random.PCG64(seed))
    xt_snap = uniform_points(rng, 2048)
    mu = make_mu(rng, n_inst)
    per = [make_points(rng, n, n // 8, n // 8) for _ in range(n_inst)]
    return Workload(net, per[0], mu, extra={"xt_snap": xt_snap, "r_hat": 32, "pts": per})


def cdr_test_cases(seed: int = 5, n1: int = 10, n2: int = 10) -> np.ndarray:
    """Test parameters of the Section 4 comparison, float64 [n1 + n2][3]:
    n1 draws from the pure-convection domain [5, 8] x {0} x {0}, then n2 from
    the convection-diffusion-reaction domain [1, 3] x [0, 2] x [0, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d1 = np.stack([rng.uniform(5.0, 8.0, n1), np.zeros(n1), np.zeros(n1)], axis=1)
    d2 = np.stack([rng.uniform(1.0, 3.0, n2), rng.uniform(0.0, 2.0, n2),
                   rng.uniform(0.0, 2.0, n2)], axis=1)
    return np.concatenate([d1, d2])


def hyper_init(H: list, seed: int = 7) -> np.ndarray:
    """Parameters of a hypernetwork with widths H (packed per layer as W_k
    [H_k][H_{k-1}] row-major, then c_k): W ~ N(0, 1/H_{k-1}); hidden biases
    U(-0.5, 0.5); output biases U(0.5, 1.5), the range of the nets' s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(1, len(H)):
        out.append(rng.standard_normal(H[k] * H[k - 1]) / math.sqrt(H[k - 1]))
        lo, hi = (0.5, 1.5) if k == len(H) - 1 else (-0.5, 0.5)
        out.append(rng.uniform(lo, hi, H[k]))
    return np.concatenate(out).astype(np.float32)


def serving_stream(seed: int = 4, n_req: int = 2000, rate: float = 500.0):
    """Poisson stream of new-mu requests: arrival times (s), mu, point counts
    log-uniform in [1024, 65536], reduced widths drawn from {16, 32, 48}, and a
    per-request point seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, n_req)
    arrivals = np.cumsum(gaps)
    mu = make_mu(rng, n_req)
    n = np.round(np.exp(rng.uniform(math.log(1024), math.log(65536), n_req))).astype(np.int64)
    r_hat = rng.choice(np.array([16, 32, 48]), n_req)
    pt_seed = rng.integers(0, 2**31 - 1, n_req)
    return {"arrival": arrivals, "mu": mu, "n": n, "r_hat": r_hat, "pt_seed": pt_seed}


def request_points(pt_seed: int, n: int) -> Points:
    rng = np.random.Generator(np.random.PCG64(int(pt_seed)))
    return make_points(rng, n, max(1, n // 8), max(1, n // 8))


def convection_net(rng: np.random.Generator, M: list, r: list, beta: float) -> Net:
    """A net whose first layer sees only xi = x - beta t: r_1 = 1 and V^1
    proportional to (1, -beta).  Every output is then h(x - beta t) for some h."""
    net = make_net(rng, M, r)
    assert r[0] == 1
    # a power-of-two scale keeps the ratio -beta exact after FP32 rounding
    scale = 2.0 ** -math.ceil(math.log2(math.hypot(1.0, beta)))
    net.V[0] = (np.array([[1.0], [-beta]]) * scale).astype(np.float32)
    return net
