"""Differentiation form: torch.autograd.Function wrappers of the fused kernels.

Both functions take the coefficients s of B instances ([B, r_total]) as the
differentiable input; the bases U, V and biases b of the net are frozen, as in
the fine-tuning problem of the paper's Section 3 (eq. 3.5-3.7).

CDRLoss   per-instance loss of eq. 3.5 / 3.6 (+ eq. 3.7) with the residual of
          eq. 4.1, each instance with its own PDE parameters and points.
          Forward runs the loss-only kernel; backward recomputes the forward
          jets and runs the fused reverse sweep (nothing per point is kept
          between the two), then scales by the incoming gradient.
LRNRJets  forward jets (u, u_x, u_t, u_xx) at each instance's points.  Backward
          is the vector-Jacobian product kernel: the reverse sweep seeded with
          the incoming cotangent of the jets, again recomputing the forward.

All B instances of a call run in one task-table launch (include/lrnr.h,
lrnr_tasks_run).  The torch code here only marshals arguments.
"""
from __future__ import annotations

import torch

from . import api


def _f32(t):
    if t.dtype != torch.float32:
        raise TypeError("float32 tensors expected")
    return t.contiguous()


class CDRBatch:
    """B loss instances on one net: mu [B, 3], interior points xt_r [B, N, 2],
    initial abscissae x_0 [B, N0], boundary times t_b [B, Nb] (device float32).
    Owns the output buffers and the task table of its launches."""

    def __init__(self, net, mu, xt_r, x_0, t_b, cfg, ws=None):
        self.net = net
        self.mu = _f32(mu)
        self.xt_r = _f32(xt_r)
        self.x_0 = _f32(x_0)
        self.t_b = _f32(t_b)
        self.cfg = cfg
        self.B = self.mu.shape[0]
        dev = self.mu.device
        self.ws = ws or api.Workspace(dev)
        self._loss = torch.empty((self.B, 4), dtype=torch.float32, device=dev)
        self._grad = torch.empty((self.B, net.r_total), dtype=torch.float32, device=dev)
        self._table = None
        self._table_s = None

    def _tasks(self, s):
        # rebuilt only when s moves to another storage (in-place updates are seen)
        if self._table is None or self._table_s != s.data_ptr():
            tab = api.TaskTable([self.net])
            for i in range(self.B):
                tab.add(0, s=s[i], mu=self.mu[i], xt_r=self.xt_r[i], x_0=self.x_0[i],
                        t_b=self.t_b[i], grad_s=self._grad[i], loss=self._loss[i])
            self._table, self._table_s = tab, s.data_ptr()
        return self._table

    def _check(self, s):
        if s.shape != (self.B, self.net.r_total):
            raise ValueError(f"s has shape {tuple(s.shape)}, expected "
                             f"{(self.B, self.net.r_total)}")

    def loss(self, s):
        """[B, 4]: total, interior, initial and boundary terms (loss-only kernel)."""
        s = _f32(s)
        self._check(s)
        self._tasks(s).run(api.MODE_LOSS, self.cfg, self.ws, s.device)
        return self._loss.clone()

    def loss_and_grad(self, s):
        """([B, 4] loss, [B, r_total] dL_i/ds_i) from the fused forward + reverse kernel."""
        s = _f32(s)
        self._check(s)
        self._tasks(s).run(api.MODE_GRAD, self.cfg, self.ws, s.device)
        return self._loss.clone(), self._grad.clone()


class CDRLoss(torch.autograd.Function):
    """loss_i(s_i) for every instance of a CDRBatch: s [B, r_total] -> [B]."""

    @staticmethod
    def forward(ctx, s, batch, recompute):
        s_ = s.detach()
        if recompute:
            loss = batch.loss(s_)
            ctx.grad = None
        else:
            # one fused pass computes both; only [B, r_total] is kept
            loss, ctx.grad = batch.loss_and_grad(s_)
        ctx.batch = batch
        ctx.save_for_backward(s_)
        return loss[:, 0]

    @staticmethod
    def backward(ctx, gout):
        (s_,) = ctx.saved_tensors
        g = ctx.grad if ctx.grad is not None else ctx.batch.loss_and_grad(s_)[1]
        return gout.to(g.dtype)[:, None] * g, None, None


def cdr_loss(s, batch, recompute=None):
    """Per-instance CDR loss [B] of the coefficients s [B, r_total].

    recompute: True runs the loss-only pass in the forward and the fused
    loss + gradient pass in the backward; False runs the fused pass in the
    forward and keeps the gradient ([B, r_total]) for the backward, one
    launch per step instead of two.  None (default) takes False when a
    backward can follow (grad mode on and s requires grad), else True."""
    if recompute is None:
        recompute = not (torch.is_grad_enabled() and s.requires_grad)
    return CDRLoss.apply(s, batch, recompute)


class JetsBatch:
    """Forward jets of B instances on one net at points xt [B, N, 2]."""

    def __init__(self, net, xt, ws=None):
        self.net = net
        self.xt = _f32(xt)
        self.B, self.N = self.xt.shape[0], self.xt.shape[1]
        dev = self.xt.device
        self.ws = ws or api.Workspace(dev)
        self._jets = torch.empty((self.B, 4, self.N), dtype=torch.float32, device=dev)
        self._cot = torch.empty((self.B, 4, self.N), dtype=torch.float32, device=dev)
        self._grad = torch.empty((self.B, net.r_total), dtype=torch.float32, device=dev)
        self._table = None
        self._table_s = None

    def _tasks(self, s):
        if self._table is None or self._table_s != s.data_ptr():
            tab = api.TaskTable([self.net])
            for i in range(self.B):
                tab.add(0, s=s[i], xt_r=self.xt[i], out=self._jets[i], cot=self._cot[i],
                        grad_s=self._grad[i])
            self._table, self._table_s = tab, s.data_ptr()
        return self._table

    def jets(self, s):
        s = _f32(s)
        self._tasks(s).run(api.MODE_JETS, None, self.ws, s.device)
        return self._jets.clone()

    def vjp(self, s, cot):
        """sum over points and components of cot * d(jets)/ds, per instance."""
        s = _f32(s)
        self._cot.copy_(cot)
        self._tasks(s).run(api.MODE_VJP, None, self.ws, s.device)
        return self._grad.clone()


class LRNRJets(torch.autograd.Function):
    """Jets [B, 4, N] (u, u_x, u_t, u_xx) of the coefficients s [B, r_total]."""

    @staticmethod
    def forward(ctx, s, batch):
        s_ = s.detach()
        ctx.batch = batch
        ctx.save_for_backward(s_)
        return batch.jets(s_)

    @staticmethod
    def backward(ctx, gjets):
        (s_,) = ctx.saved_tensors
        return ctx.batch.vjp(s_, gjets.to(torch.float32)), None


def lrnr_jets(s, batch):
    return LRNRJets.apply(s, batch)
