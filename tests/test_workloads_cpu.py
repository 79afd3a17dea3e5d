"""The seeded generators added for the reference-solver, meta-learning and
factored-bias workloads: ranges, shapes and determinism."""
import numpy as np

import workloads as wl


def test_cdr_test_cases_cover_the_two_domains():
    m = wl.cdr_test_cases()
    assert m.shape == (20, 3) and m.dtype == np.float64
    d1, d2 = m[:10], m[10:]
    assert np.all((d1[:, 0] >= 5) & (d1[:, 0] <= 8)) and np.all(d1[:, 1:] == 0)
    assert np.all((d2[:, 0] >= 1) & (d2[:, 0] <= 3))
    assert np.all((d2[:, 1:] >= 0) & (d2[:, 1:] <= 2))
    assert np.array_equal(m, wl.cdr_test_cases())
    assert not np.array_equal(m, wl.cdr_test_cases(6))
    assert wl.cdr_test_cases(8, 32, 32).shape == (64, 3)


def test_hyper_init_layout():
    H = [3, 33, 33, 33]
    th = wl.hyper_init(H)
    assert th.dtype == np.float32
    assert th.size == sum(H[k] * H[k - 1] + H[k] for k in range(1, len(H)))
    c_out = th[-H[-1]:]
    assert np.all((c_out >= 0.5) & (c_out <= 1.5))
    assert np.array_equal(th, wl.hyper_init(H))


def test_grid_points_are_t_major():
    g = wl.grid_points(8, 3)
    assert g.shape == (24, 2) and g.dtype == np.float32
    assert np.allclose(g[:8, 1], 0) and np.allclose(g[8:16, 1], 0.5) and np.allclose(g[16:, 1], 1)
    assert np.allclose(g[:8, 0], 2 * np.pi * np.arange(8) / 8)
