"""Host-side checks of the C-ABI library: it loads, exports every function
that include/lrnr.h declares, and rejects bad arguments before any device
work (no compute call is made here)."""
import ctypes as C

import pytest

from paper_2410_04001_amd import _clib as cl

from _util import header_functions


@pytest.fixture(scope="module")
def lib():
    return cl.lib()


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ("lrnr_forward_jets", "lrnr_residual_loss", "lrnr_grad_s",
              "fastlrnr_build", "fastlrnr_grad_s"):
        assert n in names
    assert set(names) == set(cl.SIGNATURES), set(names) ^ set(cl.SIGNATURES)


def test_library_exports_every_declared_symbol(lib):
    for n in header_functions():
        assert hasattr(lib, n), n


def test_missing_library_fails_loudly():
    """Without the built library the binding raises (there is no fallback);
    checked in a child interpreter so this process keeps its loaded library."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2410_04001_amd import _clib as cl\n"
            "cl.LIB_PATH = '/nonexistent/liblrnr.so'\n"
            "try:\n"
            "    cl.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "is missing" in r.stdout, r.stdout


def _net(L=5, M=(2, 64, 64, 64, 64, 1), r=(0, 2, 8, 8, 8, 1), ptr=16):
    n = cl.LrnrNet()
    n.L = L
    for i, m in enumerate(M):
        n.M[i] = m
    for i, x in enumerate(r):
        n.r[i] = x
    n.U = n.V = n.b = ptr
    return n


def _pts(n_r=100, n_0=10, n_b=10, ptr=16):
    return cl.LrnrPoints(ptr, n_r, ptr, n_0, ptr, n_b)


def test_workspace_size_and_validation(lib):
    good = _net()
    pts = _pts()
    assert lib.lrnr_workspace_size(C.byref(good), C.byref(pts), 1) > 0
    assert lib.lrnr_workspace_size(C.byref(good), C.byref(pts), 4) > \
        lib.lrnr_workspace_size(C.byref(good), C.byref(pts), 1)
    bad = [
        _net(M=(3, 64, 64, 64, 64, 1)),           # input width must be 2
        _net(M=(2, 64, 64, 64, 64, 2)),           # output width must be 1
        _net(r=(0, 3, 8, 8, 8, 1)),               # r_1 > M_0
        _net(r=(0, 2, 8, 8, 8, 2)),               # r_L > M_L
        _net(r=(0, 2, 0, 8, 8, 1)),               # zero rank
        _net(L=1),
        _net(L=9),
        _net(M=(2, 300, 64, 64, 64, 1)),          # width above the compiled limit
        _net(r=(0, 2, 40, 8, 8, 1), M=(2, 64, 64, 64, 64, 1)),  # rank above 32
        _net(ptr=0),                              # NULL factors
    ]
    for b in bad:
        assert lib.lrnr_workspace_size(C.byref(b), C.byref(pts), 1) == 0
    assert lib.lrnr_workspace_size(C.byref(good), C.byref(_pts(n_r=-1)), 1) == 0
    assert lib.lrnr_workspace_size(C.byref(good), C.byref(_pts(ptr=0)), 1) == 0
    assert lib.lrnr_workspace_size(C.byref(good), C.byref(pts), 0) == 0
    # a hidden rank above the widths next to it is valid: the reduced net of a
    # FastLRNR has widths r_hat_l that may be below the ranks (eq. 2.7-2.8)
    narrow = _net(M=(2, 4, 4, 5, 4, 1), r=(0, 2, 8, 20, 8, 1))
    assert lib.lrnr_workspace_size(C.byref(narrow), C.byref(pts), 1) > 0
    assert lib.lrnr_workspace_size(C.byref(_net(M=(2, 1, 1, 1, 1, 1))), C.byref(pts), 1) > 0
    # empty point sets are valid and still need a (minimal) workspace
    assert lib.lrnr_workspace_size(C.byref(good), C.byref(_pts(0, 0, 0, ptr=0)), 1) >= 256


def test_entry_points_reject_bad_arguments_without_device_work(lib):
    net = _net()
    pts = _pts()
    cfg = cl.LrnrLossCfg(0, 1.0, 1.0, 1.0, 0.0, None)
    out = C.c_void_p(16)
    # NULL net / points / cfg
    assert lib.lrnr_grad_s(None, out, out, C.byref(pts), C.byref(cfg), out, None, None,
                           out, 1 << 30, None) == cl.EINVAL
    assert lib.lrnr_grad_s(C.byref(net), out, out, None, C.byref(cfg), out, None, None,
                           out, 1 << 30, None) == cl.EINVAL
    assert lib.lrnr_residual_loss(C.byref(net), out, out, C.byref(pts), None, out, out,
                                  1 << 30, None) == cl.EINVAL
    # bad loss form, lambda without s_ref
    bad_cfg = cl.LrnrLossCfg(2, 1.0, 1.0, 1.0, 0.0, None)
    assert lib.lrnr_residual_loss(C.byref(net), out, out, C.byref(pts), C.byref(bad_cfg), out,
                                  out, 1 << 30, None) == cl.EINVAL
    loc_cfg = cl.LrnrLossCfg(0, 1.0, 1.0, 1.0, 0.5, None)
    assert lib.lrnr_grad_s(C.byref(net), out, out, C.byref(pts), C.byref(loc_cfg), out, None,
                           None, out, 1 << 30, None) == cl.EINVAL
    # workspace too small / misaligned
    assert lib.lrnr_grad_s(C.byref(net), out, out, C.byref(pts), C.byref(cfg), out, None, None,
                           out, 16, None) == cl.ENOMEM
    assert lib.lrnr_grad_s(C.byref(net), out, out, C.byref(pts), C.byref(cfg), out, None, None,
                           C.c_void_p(24), 1 << 30, None) == cl.EINVAL
    # unsupported sizes
    wide = _net(M=(2, 300, 64, 64, 64, 1))
    assert lib.lrnr_forward_jets(C.byref(wide), out, out, 10, out, None) == cl.EUNSUPPORTED
    # negative counts, Adam arguments
    assert lib.lrnr_forward_jets(C.byref(net), out, out, -1, out, None) == cl.EINVAL
    assert lib.lrnr_adam_step(out, out, out, out, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == cl.EINVAL
    # FastLRNR build arguments
    h = C.c_void_p()
    rh = (C.c_int32 * 4)(32, 32, 32, 32)
    assert lib.fastlrnr_build(C.byref(net), out, 0, out, 10, rh, C.byref(h), None) == cl.EINVAL
    rh_bad = (C.c_int32 * 4)(65, 32, 32, 32)
    assert lib.fastlrnr_build(C.byref(net), out, 1, out, 100, rh_bad, C.byref(h),
                              None) == cl.EINVAL
    rh_many = (C.c_int32 * 4)(32, 32, 32, 32)
    assert lib.fastlrnr_build(C.byref(net), out, 1, out, 10, rh_many, C.byref(h),
                              None) == cl.EINVAL   # r_hat above the snapshot count
    assert lib.fastlrnr_grad_s(None, out, out, C.byref(pts), C.byref(cfg), out, out, out,
                               1 << 30, None) == cl.EINVAL
    assert lib.fastlrnr_destroy(None) == cl.EINVAL
    # the workspace-free gradient refuses sizes beyond its fixed scratch
    # before any device work
    n = 1 << 20
    big = _pts(n, n // 8, n // 8)
    assert lib.lrnr_workspace_size(C.byref(net), C.byref(big), 1) > 64 << 20
    assert lib.lrnr_grad_s_noalloc(C.byref(net), out, out, C.byref(big), C.byref(cfg), out, out,
                                   out, None) == cl.EUNSUPPORTED


def test_status_strings(lib):
    assert lib.lrnr_status_string(0) == b"ok"
    net = _net(M=(2, 300, 64, 64, 64, 1))
    lib.lrnr_forward_jets(C.byref(net), C.c_void_p(16), C.c_void_p(16), 10, C.c_void_p(16), None)
    s = lib.lrnr_status_string(cl.EUNSUPPORTED).decode()
    assert "unsupported" in s and "M[1]=300" in s


# ---------------------------------------------------------------- layouts ---

STRUCTS = {
    "lrnr_net": cl.LrnrNet, "lrnr_points": cl.LrnrPoints, "lrnr_loss_cfg": cl.LrnrLossCfg,
    "lrnr_task": cl.LrnrTask, "lrnr_srv_model": cl.LrnrSrvModel, "lrnr_srv_cfg": cl.LrnrSrvCfg,
    "lrnr_srv_request": cl.LrnrSrvRequest, "lrnr_srv_done": cl.LrnrSrvDone,
    "lrnr_srv_stats": cl.LrnrSrvStats,
}


def test_ctypes_struct_layouts_match_the_header(tmp_path):
    """sizeof and every field offset of the public structs, as the C compiler
    lays them out, equal the ctypes views the binding uses."""
    import shutil
    import subprocess
    from _util import ROOT
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "lrnr.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", f"{ROOT}/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for cname, cls in STRUCTS.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


# ---------------------------------------------------------- task tables ---

def test_tasks_workspace_and_validation(lib):
    nets = (cl.LrnrNet * 2)(_net(), _net(L=3, M=(2, 48, 40, 1), r=(0, 2, 8, 1)))
    t = (cl.LrnrTask * 2)()
    for i in range(2):
        t[i].net = i
        t[i].s = t[i].mu = t[i].grad_s = t[i].loss = 16
        t[i].pts = _pts(1000 * (i + 1), 100, 100)
    n1 = lib.lrnr_tasks_workspace_size(cl.MODE_GRAD, nets, 2, t, 1)
    n2 = lib.lrnr_tasks_workspace_size(cl.MODE_GRAD, nets, 2, t, 2)
    assert 0 < n1 < n2
    assert lib.lrnr_tasks_workspace_size(cl.MODE_LOSS, nets, 2, t, 2) < n2
    assert lib.lrnr_tasks_workspace_size(7, nets, 2, t, 2) == 0          # bad mode
    t[1].net = 2
    assert lib.lrnr_tasks_workspace_size(cl.MODE_GRAD, nets, 2, t, 2) == 0  # bad net index
    t[1].net = 1
    t[1].s = None
    assert lib.lrnr_tasks_workspace_size(cl.MODE_GRAD, nets, 2, t, 2) == 0  # NULL s
    t[1].s = 16
    ws = C.c_void_p(256)
    st = lib.lrnr_tasks_run(cl.MODE_GRAD, nets, 2, t, 2, C.byref(cl.LrnrLossCfg(0, 1, 1, 1, 0, None)),
                            ws, n2 - 1, None)
    assert st == cl.ENOMEM


# -------------------------------------------------------------- serving ---

def _srv_cfg(models, **kw):
    c = cl.LrnrSrvCfg()
    c.n_models = len(models)
    c.models = C.cast(models, C.POINTER(cl.LrnrSrvModel))
    c.K, c.steps_per_launch, c.max_slots, c.max_inflight = 100, 1, 64, 2
    c.arena_bytes, c.max_tiles, c.use_graph = 1 << 30, 1 << 16, 1
    c.loss = cl.LrnrLossCfg(0, 1.0, 1.0, 1.0, 0.0, None)
    c.lr, c.beta1, c.beta2, c.eps = 1e-3, 0.9, 0.999, 1e-8
    c.grid_nx, c.grid_nt = 256, 100
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_serving_footprint_and_config_validation(lib):
    models = (cl.LrnrSrvModel * 2)()
    models[0].net = _net(M=(2, 32, 32, 32, 32, 1))
    models[1].net = _net(M=(2, 48, 48, 48, 48, 1))
    models[0].s_init = models[1].s_init = 16
    cfg = _srv_cfg(models)
    fp = lambda m, n: lib.lrnr_srv_footprint(C.byref(cfg), m, n, n // 8, n // 8)
    a, b = fp(0, 1024), fp(0, 65536)
    assert 0 < a < b
    # points, state, records and the grid output all count
    assert b - a >= (65536 - 1024) * 8
    assert fp(0, 1024) >= 256 * 100 * 4
    assert fp(1, 4096) > fp(0, 4096)            # wider net: longer records
    assert fp(2, 1024) == 0                     # no such model
    for bad in ({"K": 0}, {"steps_per_launch": 0}, {"max_slots": 0}, {"max_slots": 5000},
                {"grid_nt": 1}, {"arena_bytes": 16}, {"lr": 0.0}, {"beta2": 1.0}):
        c = _srv_cfg(models, **bad)
        assert lib.lrnr_srv_footprint(C.byref(c), 0, 1024, 128, 128) == 0, bad
    models[1].s_init = None
    assert lib.lrnr_srv_footprint(C.byref(cfg), 0, 1024, 128, 128) == 0


def test_host_tensors_are_refused_at_the_boundary():
    # every array of the C ABI is device memory; a host tensor is refused
    # before any call is made
    torch = pytest.importorskip("torch")
    from paper_2410_04001_amd import api
    with pytest.raises(ValueError):
        api._p(torch.zeros(4))
    assert api._p(None) is None
