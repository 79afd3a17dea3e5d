"""Pins of the CDR reference-solution oracle (oracle/cdr_reference.py) against
what the mathematics of eq. (4.1) fixes: closed forms where the splitting is
exact, the analytic blow-up time, the second order of Strang splitting and
the PDE residual of the computed solution."""
import math

import numpy as np
import pytest

from oracle import cdr_reference as cdr


@pytest.mark.parametrize("beta,nu", [(5.0, 0.0), (8.0, 0.0), (2.0, 1.5), (1.0, 0.3)])
def test_no_reaction_is_the_damped_travelling_wave(beta, nu):
    # rho = 0: u = exp(-nu t) sin(x - beta t); the linear sub-flow is exact
    n_x, n_t, n_out = 64, 50, 11
    u, st = cdr.cdr_solve((beta, nu, 0.0), n_x, n_t, n_out)
    assert st == 0
    x = 2 * math.pi * np.arange(n_x) / n_x
    for k in range(n_out):
        t = k / (n_out - 1)
        ref = math.exp(-nu * t) * np.sin(x - beta * t)
        np.testing.assert_allclose(u[k], ref, rtol=0, atol=1e-13)


def test_pure_reaction_is_the_logistic_flow():
    # beta = nu = 0: pointwise logistic ODE, u0 e^{rho t} / (1 - u0 + u0 e^{rho t})
    rho = 0.5
    n_x, n_t, n_out = 32, 40, 5
    u, st = cdr.cdr_solve((0.0, 0.0, rho), n_x, n_t, n_out)
    assert st == 0
    u0 = np.sin(2 * math.pi * np.arange(n_x) / n_x)
    for k in range(n_out):
        t = k / (n_out - 1)
        e = math.exp(rho * t)
        np.testing.assert_allclose(u[k], u0 * e / (1 - u0 + u0 * e), rtol=0, atol=1e-13)


@pytest.mark.parametrize("rho", [2.0, 1.5])
def test_blow_up_at_the_analytic_time(rho):
    # beta = nu = 0: the grid point x = 3 pi / 2 starts at -1 and reaches -inf
    # at t* = ln 2 / rho; the step that crosses t* is the first flagged one
    n_x, n_t, n_out = 64, 1000, 11
    u, st = cdr.cdr_solve((0.0, 0.0, rho), n_x, n_t, n_out)
    t_star = math.log(2.0) / rho
    assert st == math.ceil(t_star * n_t)
    last = (st - 1) // (n_t // (n_out - 1))     # last output written before it
    assert np.all(np.isfinite(u[:last + 1]))
    assert np.all(np.isnan(u[last + 1:]))


def test_strang_splitting_is_second_order():
    # successive differences shrink by 4 when dt halves (Lie splitting: by 2)
    mu, n_x = (2.0, 1.0, 0.8), 64
    sols = [cdr.cdr_solve(mu, n_x, n_t, 2)[0][-1] for n_t in (50, 100, 200, 400)]
    d = [np.max(np.abs(a - b)) for a, b in zip(sols, sols[1:])]
    for a, b in zip(d, d[1:]):
        assert 3.6 < a / b < 4.4, d


def test_solution_satisfies_the_pde():
    # spectral u_x, u_xx and a central difference in t of a fine solution
    mu = (1.5, 0.4, 0.8)
    n_x, n_t, n_out = 64, 4000, 1001
    u, st = cdr.cdr_solve(mu, n_x, n_t, n_out)
    assert st == 0
    k = cdr.wavenumbers(n_x)
    h = 1.0 / (n_out - 1)
    worst = 0.0
    for j in (100, 500, 900):
        uh = np.fft.fft(u[j])
        ux = np.fft.ifft(1j * k * uh).real
        uxx = np.fft.ifft(-(k * k) * uh).real
        ut = (u[j + 1] - u[j - 1]) / (2 * h)
        res = ut + mu[0] * ux - mu[1] * uxx - mu[2] * u[j] * (1 - u[j])
        worst = max(worst, np.max(np.abs(res)) / np.max(np.abs(ut)))
    assert worst < 1e-4, worst
    # a dropped reaction term fails the same check
    res_bad = (u[501] - u[499]) / (2 * h) + mu[0] * np.fft.ifft(1j * k * np.fft.fft(u[500])).real \
        - mu[1] * np.fft.ifft(-(k * k) * np.fft.fft(u[500])).real
    assert np.max(np.abs(res_bad)) > 1e-2


def test_grid_points_and_l1_error():
    g = cdr.grid_points(8, 3)
    assert g.shape == (24, 2)
    assert np.allclose(g[:8, 1], 0.0) and np.allclose(g[16:, 1], 1.0)
    assert np.allclose(g[:8, 0], 2 * math.pi * np.arange(8) / 8)
    ref = np.array([1.0, -2.0, 3.0, -4.0])
    assert cdr.l1_relative_error(ref * 1.1, ref) == pytest.approx(0.1)
    assert cdr.l1_relative_error(ref + np.array([1.0, 0, 0, 0]), ref) == pytest.approx(0.1)
