"""Torch-facing wrappers of the C ABI (argument marshalling only).

Tensors must be float32 CUDA (ROCm) tensors; calls run on torch's current
stream.  Every computation happens inside liblrnr.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _clib as cl


def _p(t):
    """Device address of a tensor for the C ABI, whose arrays are all device
    memory: a host tensor here would reach a kernel as a bad address, so it is
    refused."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("a device (cuda) tensor is required, got one on " + str(t.device))
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, device):
    t = torch.as_tensor(x, dtype=torch.float32, device=device)
    return t.contiguous()


class DeviceNet:
    """An LRNR in device memory: widths M[0..L], ranks r[1..L] and the packed
    factors of include/lrnr.h."""

    def __init__(self, M, r, U, V, b, device="cuda", _keep=None):
        self.M = [int(m) for m in M]
        self.r = [int(x) for x in r]          # r_1..r_L
        self.L = len(self.r)
        self.U = _dev(U, device) if not isinstance(U, int) else U
        self.V = _dev(V, device) if not isinstance(V, int) else V
        self.b = _dev(b, device) if not isinstance(b, int) else b
        self._keep = _keep
        self._c = cl.LrnrNet()
        self._c.L = self.L
        for l, m in enumerate(self.M):
            self._c.M[l] = m
        for l, x in enumerate(self.r, start=1):
            self._c.r[l] = x
        self._c.U = self.U if isinstance(self.U, int) else self.U.data_ptr()
        self._c.V = self.V if isinstance(self.V, int) else self.V.data_ptr()
        self._c.b = self.b if isinstance(self.b, int) else self.b.data_ptr()

    @classmethod
    def from_net(cls, net, device="cuda"):
        """From any object with M, r and packed() -> (U, V, b, s) host arrays."""
        U, V, b, _ = net.packed()
        return cls(net.M, net.r, U, V, b, device)

    @property
    def r_total(self):
        return sum(self.r)

    @property
    def b_total(self):
        return sum(self.M[1:])

    def c(self):
        return C.byref(self._c)


class DevicePoints:
    def __init__(self, xt_r, x_0, t_b, device="cuda"):
        self.xt_r = _dev(np.asarray(xt_r, np.float32).reshape(-1, 2), device)
        self.x_0 = _dev(np.asarray(x_0, np.float32).reshape(-1), device)
        self.t_b = _dev(np.asarray(t_b, np.float32).reshape(-1), device)
        self._c = cl.LrnrPoints(
            self.xt_r.data_ptr() if self.xt_r.numel() else None, self.xt_r.shape[0],
            self.x_0.data_ptr() if self.x_0.numel() else None, self.x_0.shape[0],
            self.t_b.data_ptr() if self.t_b.numel() else None, self.t_b.shape[0])

    @classmethod
    def from_points(cls, pts, device="cuda"):
        return cls(pts.xt_r, pts.x_0, pts.t_b, device)

    @property
    def counts(self):
        return self.xt_r.shape[0], self.x_0.shape[0], self.t_b.shape[0]

    def c(self):
        return C.byref(self._c)


class LossCfg:
    def __init__(self, form=0, w_r=1.0, w_0=1.0, w_b=1.0, lambda_loc=0.0, s_ref=None):
        self.s_ref = s_ref
        self._c = cl.LrnrLossCfg(int(form), float(w_r), float(w_0), float(w_b),
                                 float(lambda_loc),
                                 None if s_ref is None else s_ref.data_ptr())

    def c(self):
        return C.byref(self._c)


class Workspace:
    """A device byte buffer, grown on demand and reused across calls."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        return self.buf

    def ptr_size(self, nbytes):
        b = self.get(nbytes)
        addr = b.data_ptr()
        pad = (-addr) % 256
        return C.c_void_p(addr + pad), b.numel() - pad


_default_ws = {}


def _ws(device):
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def workspace_size(net, pts, batch=1):
    n = cl.lib().lrnr_workspace_size(net.c(), pts.c(), int(batch))
    if n == 0:
        raise cl.LrnrError(cl.EINVAL, "lrnr_workspace_size")
    return n


def forward_jets(net, s, xt):
    n = xt.shape[0]
    out = torch.empty((4, n), dtype=torch.float32, device=xt.device)
    cl.check(cl.lib().lrnr_forward_jets(net.c(), _p(s), _p(xt), n, _p(out), _stream()),
             "lrnr_forward_jets")
    return out


def forward_value(net, s, xt):
    n = xt.shape[0]
    out = torch.empty((n,), dtype=torch.float32, device=xt.device)
    cl.check(cl.lib().lrnr_forward_value(net.c(), _p(s), _p(xt), n, _p(out), _stream()),
             "lrnr_forward_value")
    return out


def reduced_states(net, s, xt):
    """y^{l+1} = V^{(l+1)T} z^l of every hidden layer at the points xt
    (lrnr_reduced_states): a list of [r_{l+1}][n] tensors, l = 1..L-1."""
    n = xt.shape[0]
    rows = net.r[1:]
    y = torch.empty((sum(rows), n), dtype=torch.float32, device=xt.device)
    cl.check(cl.lib().lrnr_reduced_states(net.c(), _p(s), _p(xt), n, _p(y), _stream()),
             "lrnr_reduced_states")
    return list(torch.split(y, rows, dim=0))


def residual_loss(net, s, mu, pts, cfg, ws=None):
    ws = ws or _ws(s.device)
    wp, wn = ws.ptr_size(workspace_size(net, pts))
    loss = torch.empty(4, dtype=torch.float32, device=s.device)
    cl.check(cl.lib().lrnr_residual_loss(net.c(), _p(s), _p(mu), pts.c(), cfg.c(), _p(loss),
                                         wp, wn, _stream()), "lrnr_residual_loss")
    return loss


def grad_s(net, s, mu, pts, cfg, with_b=True, ws=None):
    ws = ws or _ws(s.device)
    wp, wn = ws.ptr_size(workspace_size(net, pts))
    gs = torch.empty(net.r_total, dtype=torch.float32, device=s.device)
    gb = torch.empty(net.b_total, dtype=torch.float32, device=s.device) if with_b else None
    loss = torch.empty(4, dtype=torch.float32, device=s.device)
    cl.check(cl.lib().lrnr_grad_s(net.c(), _p(s), _p(mu), pts.c(), cfg.c(), _p(gs), _p(gb),
                                  _p(loss), wp, wn, _stream()), "lrnr_grad_s")
    return gs, gb, loss


def grad_s_batched(net, s, mu, pts, cfg, ws=None):
    B = s.shape[0]
    ws = ws or _ws(s.device)
    wp, wn = ws.ptr_size(workspace_size(net, pts, B))
    gs = torch.empty((B, net.r_total), dtype=torch.float32, device=s.device)
    loss = torch.empty((B, 4), dtype=torch.float32, device=s.device)
    cl.check(cl.lib().lrnr_grad_s_batched(net.c(), B, _p(s), _p(mu), pts.c(), cfg.c(), _p(gs),
                                          _p(loss), wp, wn, _stream()), "lrnr_grad_s_batched")
    return gs, loss


MODE_JETS, MODE_VALUE, MODE_LOSS, MODE_GRAD, MODE_VJP = (
    cl.MODE_JETS, cl.MODE_VALUE, cl.MODE_LOSS, cl.MODE_GRAD, cl.MODE_VJP)


class TaskTable:
    """Host description of a task table for lrnr_tasks_run.

    Each task references device memory by address; the table keeps the tensors
    it was given alive.  Build it once and run it many times while those
    tensors keep their storage (in-place updates of s are seen by every run).
    """

    def __init__(self, nets):
        self.nets = list(nets)
        self._nets_c = (cl.LrnrNet * len(self.nets))(*[n._c for n in self.nets])
        self._tasks = []
        self._keep = []
        self._arr = None

    def add(self, net=0, s=None, mu=None, xt_r=None, x_0=None, t_b=None, s_ref=None,
            cot=None, out=None, grad_s=None, grad_b=None, loss=None):
        """Each argument is a contiguous float32 device tensor or None; a row
        view of a larger tensor (s[i], xt[i]) addresses that row."""
        def ref(x):
            if x is None:
                return None
            if x.dtype != torch.float32 or not x.is_contiguous():
                raise ValueError("task arrays must be contiguous float32 tensors")
            self._keep.append(x)
            return x.data_ptr()

        def cnt(x, per):
            return 0 if x is None else x.numel() // per

        t = cl.LrnrTask()
        t.net = int(net)
        t.s = ref(s)
        t.mu = ref(mu)
        t.pts = cl.LrnrPoints(ref(xt_r), cnt(xt_r, 2), ref(x_0), cnt(x_0, 1),
                              ref(t_b), cnt(t_b, 1))
        t.s_ref = ref(s_ref)
        t.cot = ref(cot)
        t.out = ref(out)
        t.grad_s = ref(grad_s)
        t.grad_b = ref(grad_b)
        t.loss = ref(loss)
        self._tasks.append(t)
        self._arr = None
        return len(self._tasks) - 1

    def __len__(self):
        return len(self._tasks)

    def _c(self):
        if self._arr is None:
            self._arr = (cl.LrnrTask * len(self._tasks))(*self._tasks)
        return self._arr

    def workspace_size(self, mode):
        n = cl.lib().lrnr_tasks_workspace_size(int(mode), self._nets_c, len(self.nets),
                                               self._c(), len(self._tasks))
        if n == 0:
            raise cl.LrnrError(cl.EINVAL, "lrnr_tasks_workspace_size")
        return n

    def run(self, mode, cfg=None, ws=None, device="cuda"):
        ws = ws or _ws(device)
        wp, wn = ws.ptr_size(self.workspace_size(mode))
        cl.check(cl.lib().lrnr_tasks_run(int(mode), self._nets_c, len(self.nets), self._c(),
                                         len(self._tasks), None if cfg is None else cfg.c(),
                                         wp, wn, _stream()), "lrnr_tasks_run")


class HipEvent:
    """A timing hipEvent_t made through the HIP runtime (torch's Event will
    not report the time of an event recorded outside torch)."""

    _hip = None

    def __init__(self):
        if HipEvent._hip is None:
            h = C.CDLL("libamdhip64.so")
            h.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
            h.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
            h.hipEventDestroy.argtypes = [C.c_void_p]
            h.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
            HipEvent._hip = h
        self.ev = C.c_void_p()
        if HipEvent._hip.hipEventCreate(C.byref(self.ev)) != 0:
            raise RuntimeError("hipEventCreate failed")

    def record(self):
        HipEvent._hip.hipEventRecord(self.ev, _stream())

    def elapsed_ms(self, end):
        out = C.c_float()
        rc = HipEvent._hip.hipEventElapsedTime(C.byref(out), self.ev, end.ev)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return out.value

    def __del__(self):
        try:
            if self.ev.value:
                HipEvent._hip.hipEventDestroy(self.ev)
        except Exception:
            pass


def download(ptr, n):
    """Copy n floats from a raw device pointer (e.g. the operators a FastLRNR
    handle owns) into a host numpy array."""
    if HipEvent._hip is None:
        HipEvent()
    h = HipEvent._hip
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    torch.cuda.synchronize()
    out = np.empty(n, np.float32)
    rc = h.hipMemcpy(out.ctypes.data, C.c_void_p(ptr), 4 * n, 2)  # device to host
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


def time_next_fused(start, stop):
    """Bracket the next fused-kernel launch of this thread with two HipEvent
    objects (recorded on the call's stream by the library)."""
    cl.check(cl.lib().lrnr_time_next_fused(start.ev, stop.ev), "lrnr_time_next_fused")


def adam_step(s, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    cl.check(cl.lib().lrnr_adam_step(_p(s), _p(m), _p(v), _p(g), s.numel(), int(step),
                                     float(lr), float(beta1), float(beta2), float(eps),
                                     _stream()), "lrnr_adam_step")


class BiasBasis:
    """Factored biases b^l = B^l s_b^l (lrnr_bias_basis): widths M[0..L] of
    the net, columns q[1..L] and the packed basis B (device float32)."""

    def __init__(self, M, q, B, device="cuda", _keep=None):
        self.M = [int(m) for m in M]
        self.q = [int(x) for x in q]
        self.L = len(self.q)
        self.B = _dev(B, device) if not isinstance(B, int) else B
        self._keep = _keep
        self._c = cl.LrnrBiasBasis()
        self._c.L = self.L
        for l, m in enumerate(self.M):
            self._c.M[l] = m
        for l, x in enumerate(self.q, start=1):
            self._c.q[l] = x
        self._c.B = self.B if isinstance(self.B, int) else self.B.data_ptr()

    @property
    def q_total(self):
        return sum(self.q)

    @property
    def b_total(self):
        return sum(self.M[1:])

    def c(self):
        return C.byref(self._c)


def bias_compose(bb, s_b, out=None):
    """b = B s_b per layer (lrnr_bias_compose)."""
    if out is None:
        out = torch.empty(bb.b_total, dtype=torch.float32, device=s_b.device)
    cl.check(cl.lib().lrnr_bias_compose(bb.c(), _p(s_b), _p(out), _stream()),
             "lrnr_bias_compose")
    return out


def bias_grad(bb, grad_b):
    """grad_sb^l = B^lT grad_b^l (lrnr_bias_grad)."""
    g = torch.empty(bb.q_total, dtype=torch.float32, device=grad_b.device)
    cl.check(cl.lib().lrnr_bias_grad(bb.c(), _p(grad_b), _p(g), _stream()), "lrnr_bias_grad")
    return g


def with_bias(net, b):
    """The same net (U, V shared) with its biases taken from the tensor b."""
    U = net.U if isinstance(net.U, int) else net.U.data_ptr()
    V = net.V if isinstance(net.V, int) else net.V.data_ptr()
    return DeviceNet(net.M, net.r, U, V, b.data_ptr(), _keep=(net, b))


def grad_s_factored(net, bb, s, s_b, mu, pts, cfg, ws=None):
    """Loss and gradients to s and s_b of the net with factored biases:
    lrnr_bias_compose, lrnr_grad_s (with grad_b), lrnr_bias_grad."""
    b = bias_compose(bb, s_b)
    gs, gb, loss = grad_s(with_bias(net, b), s, mu, pts, cfg, with_b=True, ws=ws)
    return gs, bias_grad(bb, gb), loss


class Hyper:
    """The hypernetwork f_hyper (lrnr_hyper): widths H[0..K] (H[0] = 3,
    H[K] = r_total) and the packed parameters theta (device float32)."""

    def __init__(self, H, theta):
        self.H = [int(h) for h in H]
        self.K = len(self.H) - 1
        self.theta = theta
        self._c = cl.LrnrHyper()
        self._c.K = self.K
        for k, h in enumerate(self.H):
            self._c.H[k] = h
        self._c.theta = theta.data_ptr()

    @staticmethod
    def n_params(H):
        return sum(H[k] * H[k - 1] + H[k] for k in range(1, len(H)))

    def c(self):
        return C.byref(self._c)


def hyper_forward(f, mu, out=None):
    """s [B][r_total] = f_hyper(mu) for mu [B][3] (lrnr_hyper_forward)."""
    s = out if out is not None else torch.empty((mu.shape[0], f.H[-1]), dtype=torch.float32,
                                                device=mu.device)
    cl.check(cl.lib().lrnr_hyper_forward(f.c(), mu.shape[0], _p(mu), _p(s), _stream()),
             "lrnr_hyper_forward")
    return s


def hyper_backward(f, net, mu, s_bar, gamma, lambda_sparse, ws=None):
    """(grad_theta, R_sparse) of the meta objective (lrnr_hyper_backward)."""
    ws = ws or _ws(mu.device)
    wp, wn = ws.ptr_size(cl.lib().lrnr_hyper_workspace_size(f.c(), mu.shape[0]))
    g = torch.empty_like(f.theta)
    r = torch.empty(1, dtype=torch.float32, device=mu.device)
    cl.check(cl.lib().lrnr_hyper_backward(f.c(), net.c(), mu.shape[0], _p(mu), _p(s_bar),
                                          float(gamma), float(lambda_sparse), _p(g), _p(r),
                                          wp, wn, _stream()), "lrnr_hyper_backward")
    return g, r


def truncate(net, f, mu, ws=None):
    """Truncation after meta-learning (lrnr_truncate): drops the coefficients
    that f_hyper sets to zero at every mu [B][3], with their columns of U and
    V and their hypernetwork outputs.  Returns (DeviceNet with the new ranks,
    Hyper of the truncated map, keep mask as a host bool array)."""
    ws = ws or _ws(mu.device)
    wp, wn = ws.ptr_size(cl.lib().lrnr_truncate_workspace_size(f.c(), mu.shape[0]))
    U = torch.empty_like(net.U)
    V = torch.empty_like(net.V)
    theta = torch.empty_like(f.theta)
    r_out = (C.c_int32 * (net.L + 1))()
    keep = (C.c_int32 * net.r_total)()
    cl.check(cl.lib().lrnr_truncate(net.c(), f.c(), mu.shape[0], _p(mu), r_out, keep, _p(U),
                                    _p(V), _p(theta), wp, wn, _stream()), "lrnr_truncate")
    r = [int(x) for x in r_out[1:]]
    nU = sum(net.M[l] * r[l - 1] for l in range(1, net.L + 1))
    nV = sum(net.M[l - 1] * r[l - 1] for l in range(1, net.L + 1))
    H = f.H[:-1] + [sum(r)]
    tnet = DeviceNet(net.M, r, U[:nU], V[:nV], net.b)
    return tnet, Hyper(H, theta[:Hyper.n_params(H)]), np.array(keep[:], dtype=bool)


def meta_grad(f, net, mu, pts, cfg, gamma, lambda_sparse, ws=None):
    """One gradient of the meta objective with fixed bases: s = f_hyper(mu),
    the batched loss gradient at s, then the hypernetwork backward.  Returns
    (grad_theta, per-sample losses [B][4], R_sparse) as device tensors."""
    s = hyper_forward(f, mu)
    gs, loss = grad_s_batched(net, s, mu, pts, cfg, ws=ws)
    g, r = hyper_backward(f, net, mu, gs, gamma, lambda_sparse, ws=ws)
    return g, loss, r


def rows_mean(x):
    """(1/B) sum_b x[b] for x [B][n] (lrnr_rows_mean)."""
    out = torch.empty(x.shape[1], dtype=torch.float32, device=x.device)
    cl.check(cl.lib().lrnr_rows_mean(_p(x), x.shape[0], x.shape[1], _p(out), _stream()),
             "lrnr_rows_mean")
    return out


def orth_reg(net, with_grad=True):
    """R_orth of eq. 3.3 on the net's bases (lrnr_orth_reg): (value [1],
    grad_U, grad_V) device tensors (the gradients None without with_grad)."""
    v = torch.empty(1, dtype=torch.float32, device="cuda")
    gU = torch.empty(sum(net.M[l] * net.r[l - 1] for l in range(1, net.L + 1)),
                     dtype=torch.float32, device="cuda") if with_grad else None
    gV = torch.empty(sum(net.M[l - 1] * net.r[l - 1] for l in range(1, net.L + 1)),
                     dtype=torch.float32, device="cuda") if with_grad else None
    cl.check(cl.lib().lrnr_orth_reg(net.c(), _p(v), _p(gU), _p(gV), _stream()), "lrnr_orth_reg")
    return v, gU, gV


def _basis_out(net, device):
    gU = torch.empty(sum(net.M[l] * net.r[l - 1] for l in range(1, net.L + 1)),
                     dtype=torch.float32, device=device)
    gV = torch.empty(sum(net.M[l - 1] * net.r[l - 1] for l in range(1, net.L + 1)),
                     dtype=torch.float32, device=device)
    return gU, gV


def basis_grad(net, s, mu, pts, cfg, ws=None):
    """(grad_U, grad_V) of the loss, packed as net.U and net.V (lrnr_basis_grad)."""
    ws = ws or _ws(s.device)
    wp, wn = ws.ptr_size(cl.lib().lrnr_basis_grad_workspace_size(net.c(), pts.c()))
    gU, gV = _basis_out(net, s.device)
    cl.check(cl.lib().lrnr_basis_grad(net.c(), _p(s), _p(mu), pts.c(), cfg.c(), _p(gU), _p(gV),
                                      wp, wn, _stream()), "lrnr_basis_grad")
    return gU, gV


def basis_grad_batched(net, s, mu, pts, cfg, ws=None):
    """The mean over the B rows of s [B][r_total] and mu [B][3] of
    (grad_U, grad_V) (lrnr_basis_grad_batched)."""
    B = s.shape[0]
    ws = ws or _ws(s.device)
    wp, wn = ws.ptr_size(cl.lib().lrnr_basis_grad_batched_workspace_size(net.c(), pts.c(), B))
    gU, gV = _basis_out(net, s.device)
    cl.check(cl.lib().lrnr_basis_grad_batched(net.c(), B, _p(s), _p(mu), pts.c(), cfg.c(),
                                              _p(gU), _p(gV), wp, wn, _stream()),
             "lrnr_basis_grad_batched")
    return gU, gV


class MetaStep:
    """Gradient of the meta objective in Theta and in the biases b (eq. 3.4
    with U, V fixed) for samples mu [B][3] sharing the points pts: s =
    f_hyper(mu) into a task table of B GRAD tasks (per-sample grad_s and
    grad_b), the hypernetwork backward, and the mean of the bias gradients.
    The table is built once; the net's b may be updated in place between
    calls."""

    def __init__(self, f, net, mu, pts):
        B, R = mu.shape[0], f.H[-1]
        dev = mu.device
        self.f, self.net, self.mu = f, net, mu
        self.s = torch.empty((B, R), dtype=torch.float32, device=dev)
        self.gs = torch.empty((B, R), dtype=torch.float32, device=dev)
        self.gb = torch.empty((B, net.b_total), dtype=torch.float32, device=dev)
        self.loss = torch.empty((B, 4), dtype=torch.float32, device=dev)
        self.table = TaskTable([net])
        for b in range(B):
            self.table.add(0, s=self.s[b], mu=mu[b], xt_r=pts.xt_r, x_0=pts.x_0, t_b=pts.t_b,
                           grad_s=self.gs[b], grad_b=self.gb[b], loss=self.loss[b])

    def __call__(self, cfg, gamma, lambda_sparse, ws=None):
        """Returns (grad_theta, grad_b, per-sample losses [B][4], R_sparse)."""
        hyper_forward(self.f, self.mu, out=self.s)
        self.table.run(MODE_GRAD, cfg, ws=ws, device=self.mu.device)
        g, r = hyper_backward(self.f, self.net, self.mu, self.gs, gamma, lambda_sparse, ws=ws)
        return g, rows_mean(self.gb), self.loss, r


def cdr_reference(mu, n_x, n_t, n_out, t_end=1.0):
    """Reference solution of eq. 4.1 for mu [B][3] (float64 device tensor) by
    lrnr_cdr_reference: returns (u [B][n_out][n_x] float64, status [B] int32),
    both on the device."""
    mu = mu.contiguous()
    if mu.dtype != torch.float64 or mu.dim() != 2 or mu.shape[1] != 3:
        raise ValueError("mu must be a float64 [B][3] tensor")
    B = mu.shape[0]
    u = torch.empty(B, n_out, n_x, dtype=torch.float64, device=mu.device)
    st = torch.empty(B, dtype=torch.int32, device=mu.device)
    cl.check(cl.lib().lrnr_cdr_reference(_p(mu), B, int(n_x), int(n_t), int(n_out),
                                          float(t_end), _p(u), _p(st), _stream()),
             "lrnr_cdr_reference")
    return u, st


def l1_error_sums(pred, ref, out=None):
    """(sum |pred - ref|, sum |ref|) as a float64 [2] device tensor
    (lrnr_l1_error); pred float32, ref float64, same number of elements."""
    pred, ref = pred.contiguous(), ref.contiguous()
    if pred.dtype != torch.float32 or ref.dtype != torch.float64 or pred.numel() != ref.numel():
        raise ValueError("pred float32 and ref float64 of the same size")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=ref.device)
    cl.check(cl.lib().lrnr_l1_error(_p(pred), _p(ref), pred.numel(), _p(out), _stream()),
             "lrnr_l1_error")
    return out


class FastLRNR:
    """A FastLRNR built on the device by fastlrnr_build (eq. 2.7); its reduced
    net runs through the same entry points as the LRNR."""

    def __init__(self, net, s_snap, xt_snap, r_hat, selection="deim"):
        """selection: "deim" (greedy DEIM) or "qdeim" (pivoted-QR selection)."""
        L = net.L
        if np.isscalar(r_hat):
            r_hat = [int(r_hat)] * (L - 1)
        self.r_hat = [int(x) for x in r_hat]
        rh = (C.c_int32 * (L - 1))(*self.r_hat)
        h = C.c_void_p()
        s_snap = s_snap.reshape(-1, net.r_total).contiguous()
        sel = {"deim": cl.SEL_DEIM, "qdeim": cl.SEL_QDEIM}[selection]
        cl.check(cl.lib().fastlrnr_build_sel(net.c(), _p(s_snap), s_snap.shape[0], _p(xt_snap),
                                             xt_snap.shape[0], rh, sel, C.byref(h), _stream()),
                 "fastlrnr_build_sel")
        self._h = h
        cnet = cl.LrnrNet()
        cl.check(cl.lib().fastlrnr_get_net(h, C.byref(cnet)), "fastlrnr_get_net")
        self.net = DeviceNet(list(cnet.M)[:L + 1], list(cnet.r)[1:L + 1], int(cnet.U),
                             int(cnet.V), int(cnet.b), device=s_snap.device, _keep=self)

    def operators(self):
        """Host copies of the reduced factors (U_hat^l, V_hat^{l+1}, b_hat^l per
        hidden layer) unpacked from the handle's net."""
        n = self.net
        nU = sum(n.M[l] * n.r[l - 1] for l in range(1, n.L + 1))
        nV = sum(n.M[l - 1] * n.r[l - 1] for l in range(1, n.L + 1))
        nb = sum(n.M[1:])
        U, V, b = download(n.U, nU), download(n.V, nV), download(n.b, nb)
        Uh, Vh, bh = [], [], []
        ou, ov, ob = 0, 2 * n.r[0], 0
        for l in range(1, n.L):
            w, rl, ro = n.M[l], n.r[l - 1], n.r[l]
            Uh.append(U[ou:ou + w * rl].reshape(w, rl))
            bh.append(b[ob:ob + w])
            Vh.append(V[ov:ov + w * ro].reshape(w, ro))
            ou += w * rl
            ob += w
            ov += w * ro
        return {"U_hat": Uh, "V_hat": Vh, "b_hat": bh}

    def indices(self):
        tot = sum(self.r_hat)
        buf = (C.c_int32 * tot)()
        cl.check(cl.lib().fastlrnr_get_indices(self._h, buf), "fastlrnr_get_indices")
        out, o = [], 0
        for r in self.r_hat:
            out.append(np.array(buf[o:o + r], dtype=np.int64))
            o += r
        return out

    def grad_s(self, s, mu, pts, cfg, ws=None):
        ws = ws or _ws(s.device)
        wp, wn = ws.ptr_size(workspace_size(self.net, pts))
        gs = torch.empty(self.net.r_total, dtype=torch.float32, device=s.device)
        loss = torch.empty(4, dtype=torch.float32, device=s.device)
        cl.check(cl.lib().fastlrnr_grad_s(self._h, _p(s), _p(mu), pts.c(), cfg.c(), _p(gs),
                                          _p(loss), wp, wn, _stream()), "fastlrnr_grad_s")
        return gs, loss

    def bias_basis(self, full):
        """The reduced basis (fastlrnr_bias_basis): rows of the full basis at
        the indices P, as a BiasBasis over the reduced widths."""
        n = self.net
        # a basis of another depth is rejected by the library (LRNR_EINVAL)
        nB = sum(n.M[l] * full.q[l - 1] for l in range(1, min(n.L, full.L) + 1))
        Bh = torch.empty(max(nB, 1), dtype=torch.float32, device=full.B.device)
        red = cl.LrnrBiasBasis()
        cl.check(cl.lib().fastlrnr_bias_basis(self._h, full.c(), _p(Bh), C.byref(red), _stream()),
                 "fastlrnr_bias_basis")
        return BiasBasis(n.M, full.q, Bh)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            cl.lib().fastlrnr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
