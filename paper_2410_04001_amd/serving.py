"""Serving form: new-parameter requests through the native continuous-batching
engine of liblrnr.so (include/lrnr.h, lrnr_srv_*).

A request carries PDE parameters mu, its collocation points and the model
(FastLRNR reduced width) to use; the engine tunes s with K Adam steps of the
physics-informed loss (eq. 3.5-3.7, residual eq. 4.1) and returns the tuned
net on an nx x nt grid.  Admission, batching, graph replay and result delivery
all happen inside the library; this module marshals arguments, holds request
payloads in pinned host memory and replays Poisson arrival streams in real
time to measure latency and throughput.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import _clib as cl
from . import api


def clock():
    """Seconds on the engine's monotonic clock."""
    return cl.lib().lrnr_srv_clock()


class Request:
    """Host payload of one request: pinned inputs and host outputs."""

    def __init__(self, rid, model, mu, pts, grid_points, r_total):
        self.id = int(rid)
        self.model = int(model)
        self.mu = np.asarray(mu, np.float32)
        def pinned(a):
            a = np.ascontiguousarray(a, np.float32)
            t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
            t.copy_(torch.from_numpy(a))
            return t

        self.xt = pinned(np.asarray(pts.xt_r).reshape(-1, 2))
        self.x0 = pinned(np.asarray(pts.x_0).reshape(-1))
        self.tb = pinned(np.asarray(pts.t_b).reshape(-1))
        self.u = np.full(int(grid_points), np.nan, np.float32)
        self.s = np.full(int(r_total), np.nan, np.float32)
        self.loss = np.full(4, np.nan, np.float32)
        self.arrival = None
        self.record = None

    @property
    def n(self):
        return self.xt.shape[0]

    def c(self, arrival):
        r = cl.LrnrSrvRequest()
        r.id = self.id
        r.model = self.model
        for k in range(3):
            r.mu[k] = float(self.mu[k])
        r.arrival = float(arrival)

        def ptr(t):
            return t.data_ptr() if t.numel() else None

        r.xt_r, r.n_r = ptr(self.xt), self.xt.shape[0]
        r.x_0, r.n_0 = ptr(self.x0), self.x0.shape[0]
        r.t_b, r.n_b = ptr(self.tb), self.tb.shape[0]
        r.u_out = self.u.ctypes.data
        r.s_out = self.s.ctypes.data
        r.loss_out = self.loss.ctypes.data
        return r


class Server:
    """One engine on the current device.

    models: list of (DeviceNet, s_init device tensor [r_total]); every request
    names one by index.  The nets' device memory must outlive the server.
    """

    def __init__(self, models, K=100, steps_per_launch=2, max_slots=64, max_inflight=2,
                 arena_bytes=1 << 30, max_tiles=1 << 16, use_graph=True, loss=None,
                 lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grid=(256, 100)):
        self._keep = list(models)
        arr = (cl.LrnrSrvModel * len(models))()
        for i, (net, s0) in enumerate(models):
            arr[i].net = net._c
            arr[i].s_init = s0.data_ptr()
        self._models = arr
        loss = loss or api.LossCfg()
        self._loss = loss
        cfg = cl.LrnrSrvCfg()
        cfg.n_models = len(models)
        cfg.models = C.cast(arr, C.POINTER(cl.LrnrSrvModel))
        cfg.K, cfg.steps_per_launch = int(K), int(steps_per_launch)
        cfg.max_slots, cfg.max_inflight = int(max_slots), int(max_inflight)
        cfg.arena_bytes, cfg.max_tiles = int(arena_bytes), int(max_tiles)
        cfg.use_graph = int(bool(use_graph))
        cfg.loss = loss._c
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, beta1, beta2, eps
        cfg.grid_nx, cfg.grid_nt = int(grid[0]), int(grid[1])
        self.cfg = cfg
        self.grid = (int(grid[0]), int(grid[1]))
        self.r_totals = [net.r_total for net, _ in models]
        h = C.c_void_p()
        cl.check(cl.lib().lrnr_srv_create(C.byref(cfg), C.byref(h)), "lrnr_srv_create")
        self._h = h
        self._pending = {}

    @property
    def grid_points(self):
        return self.grid[0] * self.grid[1]

    def footprint(self, model, n_r, n_0, n_b):
        return cl.lib().lrnr_srv_footprint(C.byref(self.cfg), int(model), int(n_r), int(n_0),
                                           int(n_b))

    def request(self, rid, model, mu, pts):
        return Request(rid, model, mu, pts, self.grid_points, self.r_totals[model])

    def submit(self, req, arrival=None):
        req.arrival = clock() if arrival is None else float(arrival)
        rc = req.c(req.arrival)
        cl.check(cl.lib().lrnr_srv_submit(self._h, C.byref(rc)), "lrnr_srv_submit")
        self._pending[req.id] = req

    def poll(self):
        w, a = C.c_int32(), C.c_int32()
        cl.check(cl.lib().lrnr_srv_poll(self._h, C.byref(w), C.byref(a)), "lrnr_srv_poll")
        return w.value, a.value

    def cancel(self, rid):
        """Cancels a waiting or tuning request (lrnr_srv_cancel); its record
        then completes with status SRV_CANCELLED and no outputs."""
        cl.check(cl.lib().lrnr_srv_cancel(self._h, int(rid)), "lrnr_srv_cancel")

    def take_done(self, cap=256):
        out = (cl.LrnrSrvDone * cap)()
        n = C.c_int32()
        cl.check(cl.lib().lrnr_srv_take_done(self._h, out, cap, C.byref(n)), "lrnr_srv_take_done")
        done = []
        for k in range(n.value):
            d = out[k]
            req = self._pending.pop(d.id)
            req.record = {"id": d.id, "arrival": d.arrival, "admitted": d.admitted,
                          "done": d.done, "model": d.model, "tiles": d.tiles,
                          "status": d.status, "steps": d.steps}
            done.append(req)
        return done

    def stats(self):
        s = cl.LrnrSrvStats()
        cl.check(cl.lib().lrnr_srv_get_stats(self._h, C.byref(s)), "lrnr_srv_get_stats")
        return {name: getattr(s, name) for name, _ in cl.LrnrSrvStats._fields_}

    def run_until_done(self, timeout=60.0):
        """Polls until every submitted request has completed."""
        t_end = time.monotonic() + timeout
        done = []
        while self._pending:
            self.poll()
            done += self.take_done()
            if time.monotonic() > t_end:
                raise TimeoutError(f"{len(self._pending)} requests still pending")
        return done

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            cl.lib().lrnr_srv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server, requests, arrivals, timeout=300.0):
    """Submits requests[i] at start + arrivals[i] (seconds, ascending) on the
    engine clock, polling in between, until all have completed.

    Returns (completed requests, wall seconds from the first arrival to the
    last completion)."""
    n = len(requests)
    start = clock() + 0.005
    i = 0
    done = []
    t_end = start + float(arrivals[-1]) + timeout
    while len(done) < n:
        now = clock()
        while i < n and start + arrivals[i] <= now:
            server.submit(requests[i], start + float(arrivals[i]))
            i += 1
        w, a = server.poll()
        done += server.take_done()
        if w == 0 and a == 0 and i < n:
            # idle until the next arrival
            gap = start + float(arrivals[i]) - clock()
            if gap > 2e-4:
                time.sleep(gap - 1e-4)
        if now > t_end:
            raise TimeoutError(f"{n - len(done)} requests unfinished")
    last = max(r.record["done"] for r in done)
    return done, last - (start + float(arrivals[0]))


def latency_summary(done, wall):
    lat = np.array([r.record["done"] - r.record["arrival"] for r in done])
    queue = np.array([r.record["admitted"] - r.record["arrival"] for r in done])
    pts = sum(int(r.n) for r in done)
    return {
        "requests": len(done),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "queue_p99_ms": float(np.percentile(queue, 99) * 1e3),
        "req_per_s": len(done) / wall,
        "colloc_pts_per_s": pts / wall,
        "wall_s": wall,
    }
