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


def assert_close(got, ref, tol, what=""):
    """Parity metric: relative error in the 2-norm and in the max-norm,
    ||got - ref|| <= tol ||ref|| for both.  A per-entry relative test is not
    used: entries that are the residue of a cancellation (a jet crossing zero
    at a point, a gradient entry whose per-point terms nearly cancel) carry an
    FP32 error set by the size of the cancelling terms, which the max-norm
    bounds."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    re2 = rel_err(got, ref)
    mref = np.abs(ref).max() if ref.size else 0.0
    reinf = (np.abs(got - ref).max() / mref) if mref > 0 else (np.abs(got).max() if got.size else 0.0)
    msg = f"{what}: rel err 2-norm {re2:.3e}, max-norm {reinf:.3e} (tol {tol:g})"
    assert re2 <= tol and reinf <= tol, msg
    log(f"  {msg}")
    return re2


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()
