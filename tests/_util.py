"""Shared helpers of the test suite."""
import re
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrnr.h")


def header_functions():
    """Names of the functions declared in include/lrnr.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(lrnr_\w+|fastlrnr_\w+)\s*\(",
                     text, flags=re.M)
    return sorted(set(names))


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _rel_errs(got, ref):
    """Relative errors of got against ref in the 2-norm and in the max-norm."""
    re2 = rel_err(got, ref)
    mref = np.abs(ref).max() if ref.size else 0.0
    reinf = (np.abs(got - ref).max() / mref) if mref > 0 else (np.abs(got).max() if got.size else 0.0)
    return re2, reinf


# the loss record [total, interior, initial, boundary]: each term on its own
LOSS_BLOCKS = [1, 1, 1, 1]


def s_blocks(net):
    """Layer blocks of a flat s or grad_s: r_1, ..., r_L."""
    return [int(x) for x in net.r]


def b_blocks(net):
    """Layer blocks of a flat b or grad_b: M_1, ..., M_L."""
    return [int(x) for x in net.M[1:]]


def u_blocks(net):
    """Layer blocks of a packed U or grad_U: M_l r_l."""
    return [int(net.M[l + 1]) * int(net.r[l]) for l in range(len(net.r))]


def v_blocks(net):
    """Layer blocks of a packed V or grad_V: M_{l-1} r_l."""
    return [int(net.M[l]) * int(net.r[l]) for l in range(len(net.r))]


# A block whose FP32 value is the residue of a cancellation (a boundary-only
# loss term of two nearly equal values of u, a gradient entry whose per-point
# terms cancel, an entry that is exactly zero in exact arithmetic) cannot meet
# a relative bar against its own norm in any FP32 evaluation.  Such a block is
# held instead to FLOOR_FACTOR times the error of the oracle's own chain run
# in float32 on the same inputs (the rounding floor of the formulas, measured,
# not assumed).  The factor allows for a different FP32 evaluation: the kernels
# take sin/cos from the hardware units (absolute error up to 4.3e-7 against
# the correctly rounded 6e-8 of numpy) and sum in another order; measured
# kernel-to-floor ratios on the cases where the floor binds are up to ~5.
FLOOR_FACTOR = 10.0


def assert_close(got, ref, tol, what="", blocks=None, block_tol=None, floor=None):
    """Parity metric: relative error in the 2-norm and in the max-norm,
    ||got - ref|| <= tol ||ref|| for both, over the whole vector and, when
    ``blocks`` (sizes of consecutive blocks, e.g. the layers of grad_s) is
    given, over every block against that block's own norms (``block_tol``,
    default tol), so that a layer whose entries are small next to the others
    is held to the same relative bar.  A per-entry relative test is not used:
    entries that are the residue of a cancellation (a jet crossing zero at a
    point, a gradient entry whose per-point terms nearly cancel) carry an FP32
    error set by the size of the cancelling terms, which the max-norm of the
    block bounds.

    ``floor``: a callable returning the same quantity from the oracle run in
    float32 (``oracle.lrnr_oracle.working_precision``).  It is evaluated only
    when a block misses its bar; that block then passes if its errors stay
    within FLOOR_FACTOR times the float32 oracle's errors on the block."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    re2, reinf = _rel_errs(got, ref)
    msg = f"{what}: rel err 2-norm {re2:.3e}, max-norm {reinf:.3e} (tol {tol:g})"
    bad = re2 > tol or reinf > tol
    if blocks is not None:
        assert sum(blocks) == got.size, (what, blocks, got.size)
        btol = tol if block_tol is None else block_tol
        gmax = np.abs(ref).max() if ref.size else 0.0
        ref32 = None
        parts, o = [], 0
        for k, n in enumerate(blocks):
            g, r = got[o:o + n], ref[o:o + n]
            o += n
            if n == 0:
                continue
            if np.abs(r).max() == 0.0:
                # an identically zero block: absolute bar at the global scale
                e = np.abs(g).max() / gmax if gmax > 0 else np.abs(g).max()
                parts.append(f"{k + 1}:{e:.1e}(zero)")
                bad = bad or e > btol
                continue
            b2, binf = _rel_errs(g, r)
            part = f"{k + 1}:{b2:.1e}/{binf:.1e}"
            if (b2 > btol or binf > btol) and floor is not None:
                if ref32 is None:
                    ref32 = np.asarray(floor(), np.float64).reshape(-1)
                    assert ref32.shape == ref.shape, (what, ref32.shape, ref.shape)
                f2, finf = _rel_errs(ref32[o - n:o], r)
                lim2, liminf = max(btol, FLOOR_FACTOR * f2), max(btol, FLOOR_FACTOR * finf)
                part += f"(fp32 floor {f2:.1e}/{finf:.1e})"
                bad = bad or b2 > lim2 or binf > liminf
            else:
                bad = bad or b2 > btol or binf > btol
            parts.append(part)
        msg += f"; per block (2-norm/max-norm, tol {btol:g}) " + " ".join(parts)
    log(f"  {msg}")
    assert not bad, msg
    return re2


def fp32(fn):
    """A memoised zero-argument callable: the oracle call ``fn`` (no
    arguments) run with the oracle's arithmetic in float32, for the
    ``floor`` of assert_close."""
    box = []

    def run():
        if not box:
            from oracle import lrnr_oracle as orc
            with orc.working_precision(np.float32):
                box.append(fn())
        return box[0]
    return run


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()
