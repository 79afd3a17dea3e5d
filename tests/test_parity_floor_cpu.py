"""The FP32 rounding floor of the parity metric (tests/_util.assert_close):
the oracle's own chain run in float32 on the same inputs.  These CPU tests
show that the floor (i) is the float32 evaluation of the same formulas,
(ii) stays far below the 1e-4 bar on every well-conditioned block, so it
never loosens one, and (iii) binds only on blocks that are rounding residues
of a cancellation, where no FP32 evaluation can meet a relative bar."""
import numpy as np
import pytest

import workloads as wl
from oracle import lrnr_oracle as orc

from _util import (FLOOR_FACTOR, LOSS_BLOCKS, _rel_errs, assert_close, b_blocks, fp32,
                   s_blocks)


def _custom(seed, M, rank, n_r, n_0, n_b, mu=(3.0, 0.7, 1.3)):
    rng = np.random.Generator(np.random.PCG64(seed))
    net = wl.make_net(rng, list(M), wl.ranks(list(M), rank))
    return wl.Workload(net, wl.make_points(rng, n_r, n_0, n_b), np.array([mu], np.float32))


def _blocks(v, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(v[o:o + n])
        o += n
    return out


def test_working_precision_switches_the_arithmetic_and_restores_it():
    w = wl.small_lrnr(0, 256)
    with orc.working_precision(np.float32):
        jets = orc.lrnr_forward_jets(w.net, w.net.s, w.pts.xt_r)
        assert jets.dtype == np.float32
    jets64 = orc.lrnr_forward_jets(w.net, w.net.s, w.pts.xt_r)
    assert jets64.dtype == np.float64
    # the float32 run is the same chain: it agrees to float32 rounding
    e = np.abs(jets - jets64).max() / np.abs(jets64).max()
    assert 1e-9 < e < 1e-5, e


def test_floor_stays_far_below_the_bar_on_well_conditioned_blocks():
    """Small net, full CDR residual: every loss term and every layer block of
    grad_s and grad_b has FLOOR_FACTOR x floor below 1e-4, so the floor can
    never admit a larger error there than the plain bar does."""
    w = _custom(21, (2, 64, 64, 64, 64, 1), 8, 2048, 256, 256)
    r64 = orc.lrnr_loss(w.net, w.net.s, w.mu[0].astype(np.float64), w.pts, {}, with_grad=True)
    r32 = fp32(lambda: orc.lrnr_loss(w.net, w.net.s, w.mu[0], w.pts, {}, with_grad=True))()
    for got, ref, sizes in ((r32[0], r64[0], LOSS_BLOCKS), (r32[1], r64[1], s_blocks(w.net)),
                            (r32[2], r64[2], b_blocks(w.net))):
        for g, r in zip(_blocks(np.asarray(got, np.float64), sizes), _blocks(ref, sizes)):
            e2, einf = _rel_errs(g, r)
            assert 0 < FLOOR_FACTOR * max(e2, einf) < 1e-4, (e2, einf)


def test_floor_binds_on_a_cancellation_residue():
    """Boundary points only: b^L cancels in u(0, t) - u(2 pi, t), so dL/db^L
    is exactly zero and both evaluations return a rounding residue; the
    float32 residue is many orders above the float64 one, so a relative bar
    on that block is unreachable and the floor (not the bar) decides."""
    w = _custom(21, (2, 64, 64, 64, 1), 8, 0, 0, 40)
    r64 = orc.lrnr_loss(w.net, w.net.s, w.mu[0].astype(np.float64), w.pts, {}, with_grad=True)
    r32 = fp32(lambda: orc.lrnr_loss(w.net, w.net.s, w.mu[0], w.pts, {}, with_grad=True))()
    gb64, gb32 = _blocks(r64[2], b_blocks(w.net))[-1], _blocks(r32[2], b_blocks(w.net))[-1]
    scale = np.abs(r64[2]).max()
    assert abs(gb64[0]) < 1e-12 * scale
    assert abs(gb32[0]) < 1e-5 * scale
    assert _rel_errs(gb32, gb64)[0] > 1.0


def test_assert_close_uses_the_floor_only_where_the_bar_fails():
    ref = np.array([1.0, 2.0, 1e-9, -1e-9])
    blocks = [2, 2]
    ref32 = ref + np.array([1e-7, -1e-7, 3e-10, 1e-10])      # block 2: a residue
    ok = ref + np.array([2e-7, 0.0, 2e-9, 0.0])              # within 10 x floor
    assert_close(ok, ref, 1e-4, "floor ok", blocks=blocks, floor=lambda: ref32)
    with pytest.raises(AssertionError):                       # no floor: the bar fails
        assert_close(ok, ref, 1e-4, "no floor", blocks=blocks)
    bad = ref + np.array([0.0, 0.0, 5e-8, 0.0])              # 100 x beyond the floor
    with pytest.raises(AssertionError):
        assert_close(bad, ref, 1e-4, "beyond floor", blocks=blocks, floor=lambda: ref32)
    far = ref + np.array([1e-3, 0.0, 0.0, 0.0])              # the whole-vector bar still holds
    with pytest.raises(AssertionError):
        assert_close(far, ref, 1e-4, "whole vector", blocks=blocks, floor=lambda: ref + 1e-2)
