"""FP64 CPU oracle for the reference solution of the convection-diffusion-
reaction problem of Section 4, eq. (4.1), and for the L1 relative error of a
network's prediction against it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports or calls this
module; only ``tests/`` and ``bench.py``'s ``cpu_baseline`` leg may.  It shares
no code with the HIP solver.

Problem (Section 4, eq. 4.1), on x in (0, 2 pi) periodic, t in (0, t_end]:

    u_t + mu_1 u_x - mu_2 u_xx - mu_3 u (1 - u) = 0,   u(x, 0) = sin x.

The paper gives no solver; this one is Strang splitting (a published second-
order method) of the linear part L u = -mu_1 u_x + mu_2 u_xx and the reaction
R u = mu_3 u (1 - u):

    u_{n+1} = R(dt/2) L(dt) R(dt/2) u_n,

each sub-flow taken exactly:
  * L(tau) in Fourier space on the uniform grid x_j = 2 pi j / n_x: mode k is
    multiplied by exp(-(i mu_1 k + mu_2 k^2) tau), k in numpy's FFT order
    (k = -n_x/2 at the Nyquist index); the real part of the inverse transform
    is kept;
  * R(tau) is the logistic flow, u -> u e^{rho tau} / (1 + u (e^{rho tau} - 1)),
    which blows up within the sub-step when the denominator is <= 0.

Blow-up rule: if during step n (1-based) a denominator is <= 0, or a value is
not finite or exceeds U_MAX in magnitude, the instance stops with status n and
every output time at or after step n is NaN.  With u(x, 0) = sin x the exact
solution does blow up for part of the parameter domain (mu_3 large against
mu_2: along a characteristic with mu_2 = 0 the value -1 reaches -inf at
t = ln 2 / mu_3).

Outputs: u[k][j] at t_k = k t_end / (n_out - 1), k = 0..n_out-1, which needs
(n_out - 1) to divide n_t; dt = t_end / n_t.
"""
from __future__ import annotations

import math

import numpy as np

U_MAX = 1.0e6


def wavenumbers(n_x):
    """Integer wavenumbers of the FFT bins, in numpy's order."""
    return np.fft.fftfreq(n_x, d=1.0 / n_x)


def reaction_flow(u, rho, tau):
    """Exact logistic sub-flow of u' = rho u (1 - u) over time tau.
    Returns (u_new, ok) with ok False where the flow leaves R within tau."""
    e = math.exp(rho * tau)
    d = 1.0 + u * math.expm1(rho * tau)
    ok = d > 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        out = u * e / d
    return out, ok


def linear_flow(u, beta, nu, tau):
    """Exact flow of u_t = -beta u_x + nu u_xx over time tau (spectral)."""
    k = wavenumbers(u.shape[-1])
    fac = np.exp(-(1j * beta * k + nu * k * k) * tau)
    return np.fft.ifft(np.fft.fft(u) * fac).real


def cdr_solve(mu, n_x, n_t, n_out, t_end=1.0):
    """Strang-splitting solution of eq. (4.1) for one mu = (beta, nu, rho).
    Returns (u [n_out][n_x] float64, status)."""
    if n_out < 2 or n_t % (n_out - 1):
        raise ValueError("n_out - 1 must divide n_t")
    beta, nu, rho = (float(v) for v in mu)
    dt = t_end / n_t
    every = n_t // (n_out - 1)
    x = 2.0 * math.pi * np.arange(n_x) / n_x
    u = np.sin(x)
    out = np.full((n_out, n_x), np.nan)
    out[0] = u
    for n in range(1, n_t + 1):
        u, ok1 = reaction_flow(u, rho, 0.5 * dt)
        u = linear_flow(u, beta, nu, dt)
        u, ok2 = reaction_flow(u, rho, 0.5 * dt)
        bad = (not ok1.all()) or (not ok2.all()) or not np.all(np.isfinite(u)) \
            or np.max(np.abs(u)) > U_MAX
        if bad:
            return out, n
        if n % every == 0:
            out[n // every] = u
    return out, 0


def cdr_solve_batch(mus, n_x, n_t, n_out, t_end=1.0):
    """cdr_solve over mus [B][3]; returns (u [B][n_out][n_x], status [B])."""
    us, st = [], []
    for mu in np.asarray(mus, dtype=np.float64).reshape(-1, 3):
        u, s = cdr_solve(mu, n_x, n_t, n_out, t_end)
        us.append(u)
        st.append(s)
    return np.stack(us), np.array(st, dtype=np.int32)


def grid_points(n_x, n_out, t_end=1.0):
    """(x, t) pairs of the output grid, [n_out * n_x][2], t-major like u."""
    x = 2.0 * math.pi * np.arange(n_x) / n_x
    t = t_end * np.arange(n_out) / (n_out - 1)
    tt, xx = np.meshgrid(t, x, indexing="ij")
    return np.stack([xx.ravel(), tt.ravel()], axis=1)


def l1_relative_error(pred, ref):
    """sum |pred - ref| / sum |ref| (the error measure of the Section 4
    test-accuracy comparison), in float64."""
    pred = np.asarray(pred, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.sum(np.abs(pred - ref)) / np.sum(np.abs(ref)))
