// C ABI entry points of lrnr.h: argument validation, workspace carving and
// launches of the fused kernel and the reduction.  No allocation happens on
// these paths; the caller passes the workspace.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "lrnr_internal.h"

using namespace lrnr;

namespace {
thread_local std::string g_detail;
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
}  // namespace

// Workspace of lrnr_grad_s_noalloc: one fixed device array per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address; it takes each device's address once (hipGetSymbolAddress, with
// that device current) and passes that pointer to the kernels.
constexpr size_t kScratchBytes = LRNR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

namespace lrnr {

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_detail = buf;
  return code;
}

int32_t hip_fail(hipError_t e, const char* where) {
  return fail(LRNR_EHIP, "%s: %s", where, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Validates the net and fills the kernel-side description.
int32_t make_knet(const lrnr_net* net, KNet* k, int* RP, int* Wmax_p) {
  if (!net) return fail(LRNR_EINVAL, "net is NULL");
  const int L = net->L;
  if (L < 2 || L > LRNR_MAX_LAYERS)
    return fail(L > LRNR_MAX_LAYERS ? LRNR_EUNSUPPORTED : LRNR_EINVAL, "L=%d outside [2,%d]", L,
                LRNR_MAX_LAYERS);
  if (net->M[0] != 2) return fail(LRNR_EINVAL, "M[0]=%d, expected 2 (x, t)", net->M[0]);
  if (net->M[L] != 1) return fail(LRNR_EINVAL, "M[L]=%d, expected 1 (scalar u)", net->M[L]);
  if (!net->U || !net->V || !net->b) return fail(LRNR_EINVAL, "U, V or b is NULL");
  *k = KNet{};
  k->L = L;
  int oU = 0, oV = 0, oB = 0, oS = 0, rmax = 1, wmax = 16;
  for (int l = 0; l <= L; ++l) k->M[l] = net->M[l];
  for (int l = 1; l <= L; ++l) {
    const int Ml = net->M[l], Mp = net->M[l - 1], rl = net->r[l];
    if (l < L && (Ml < 1 || Ml > LRNR_MAX_WIDTH))
      return fail(Ml > LRNR_MAX_WIDTH ? LRNR_EUNSUPPORTED : LRNR_EINVAL,
                  "M[%d]=%d outside [1,%d]", l, Ml, LRNR_MAX_WIDTH);
    // The input layer's rank is bounded by (x, t) and the output layer's by
    // the scalar u; a hidden rank may exceed the widths next to it (the
    // reduced net of a FastLRNR has widths r_hat_l that may be below r_l,
    // eq. 2.7-2.8: U_hat^l is r_hat_l x r_l): rank and width are padded
    // independently in the kernels.
    if (rl < 1 || (l == 1 && rl > Mp) || (l == L && rl > Ml))
      return fail(LRNR_EINVAL, "r[%d]=%d outside [1, %s]", l, rl,
                  l == 1 ? "M[0]" : l == L ? "M[L]" : "LRNR_MAX_RANK");
    if (rl > LRNR_MAX_RANK)
      return fail(LRNR_EUNSUPPORTED, "r[%d]=%d above %d", l, rl, LRNR_MAX_RANK);
    k->r[l] = rl;
    k->offU[l] = oU;
    k->offV[l] = oV;
    k->offB[l] = oB;
    k->offS[l] = oS;
    oU += Ml * rl;
    oV += Mp * rl;
    oB += Ml;
    oS += rl;
    if (l >= 2 && l <= L - 1 && rl > rmax) rmax = rl;
    if (l <= L - 1) wmax = std::max(wmax, (Ml + 15) & ~15);
  }
  k->r_total = oS;
  k->b_total = oB;
  k->U = net->U;
  k->V = net->V;
  k->b = net->b;
  *RP = padded_rank(rmax);
  if (*RP < 0) return fail(LRNR_EUNSUPPORTED, "rank %d above compiled tiles", rmax);
  *Wmax_p = wmax;
  return LRNR_OK;
}

int32_t check_points(const lrnr_points* pts) {
  if (!pts) return fail(LRNR_EINVAL, "points is NULL");
  if (pts->n_r < 0 || pts->n_0 < 0 || pts->n_b < 0)
    return fail(LRNR_EINVAL, "negative point count");
  if ((pts->n_r && !pts->xt_r) || (pts->n_0 && !pts->x_0) || (pts->n_b && !pts->t_b))
    return fail(LRNR_EINVAL, "point array is NULL for a nonzero count");
  const int64_t lim = (int64_t)1 << 36;
  if (pts->n_r > lim || pts->n_0 > lim || pts->n_b > lim)
    return fail(LRNR_EUNSUPPORTED, "point count above 2^36");
  return LRNR_OK;
}

int32_t check_cfg(const lrnr_loss_cfg* cfg, bool sref_elsewhere) {
  if (!cfg) return fail(LRNR_EINVAL, "loss cfg is NULL");
  if (cfg->form != 0 && cfg->form != 1) return fail(LRNR_EINVAL, "form=%d, expected 0 or 1", cfg->form);
  if (!std::isfinite(cfg->w_r) || !std::isfinite(cfg->w_0) || !std::isfinite(cfg->w_b) ||
      !std::isfinite(cfg->lambda_loc))
    return fail(LRNR_EINVAL, "non-finite loss weight");
  if (cfg->lambda_loc != 0.f && !cfg->s_ref && !sref_elsewhere)
    return fail(LRNR_EINVAL, "lambda_loc != 0 needs s_ref");
  return LRNR_OK;
}

}  // namespace lrnr

namespace {

struct Plan {
  KGrid grid;
  size_t off_partials, off_red1, off_ckpt, off_flags, total;
  int nchunk;
};

Plan make_plan(const KNet& k, int RP, int Wmax_p, const lrnr_points* pts, int B, bool grad) {
  Plan p{};
  KGrid& g = p.grid;
  g.G_r = (int)((pts->n_r + kPtsPerWG - 1) / kPtsPerWG);
  g.G_0 = (int)((pts->n_0 + kPtsPerWG - 1) / kPtsPerWG);
  g.G_b = (int)((pts->n_b + kBcPairsPerWG - 1) / kBcPairsPerWG);
  g.G_inst = g.G_r + g.G_0 + g.G_b;
  g.B = B;
  g.P = record_floats(k);
  g.Wmax_p = Wmax_p;
  g.res_layers = resident_layers(RP, Wmax_p, k.L);
  g.s_stride = k.r_total;
  // (L-1) slots per 64-point tile: y^2..y^{L-1} in the forward sweep, then
  // ybar^2..ybar^{L-1} on their way down in the reverse sweep
  g.ckpt_per_wave = grad ? (int64_t)(k.L - 1) * 4 * (RP / 4) * 64 * 4 : 0;
  p.nchunk = (g.G_inst + kRedChunk - 1) / kRedChunk;
  size_t off = 0;
  p.off_partials = off;
  off = align256(off + (size_t)B * g.G_inst * g.P * sizeof(float));
  p.off_red1 = off;
  off = align256(off + (size_t)B * p.nchunk * g.P * sizeof(double));
  p.off_ckpt = off;
  off = align256(off + (size_t)B * g.G_inst * kWaves * g.ckpt_per_wave * sizeof(float));
  p.off_flags = off;
  off = align256(off + (grad ? (size_t)B * g.G_inst * sizeof(int) : 0));
  p.total = std::max(off, (size_t)256);  // 0 is reserved for "invalid arguments"
  return p;
}

KInst make_inst(const float* s, const float* mu, const lrnr_points* pts, const lrnr_loss_cfg* cfg) {
  KInst in{};
  in.s = s;
  in.mu = mu;
  in.xt_r = pts->xt_r;
  in.x_0 = pts->x_0;
  in.t_b = pts->t_b;
  in.n_r = pts->n_r;
  in.n_0 = pts->n_0;
  in.n_b = pts->n_b;
  if (cfg) {
    in.form = cfg->form;
    in.wr_n = pts->n_r ? (float)((double)cfg->w_r / (double)pts->n_r) : 0.f;
    in.w0_n = pts->n_0 ? (float)((double)cfg->w_0 / (double)pts->n_0) : 0.f;
    in.wb_n = pts->n_b ? (float)((double)cfg->w_b / (double)pts->n_b) : 0.f;
  }
  return in;
}

// Shared body of the loss / gradient entry points.
int32_t run_loss(const lrnr_net* net, int B, const float* s, const float* mu,
                 const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_s, float* grad_b,
                 float* loss, void* ws, size_t ws_bytes, void* stream, bool grad) {
  KNet k;
  int RP, Wmax_p;
  int32_t st = make_knet(net, &k, &RP, &Wmax_p);
  if (st) return st;
  if ((st = check_points(pts)) || (st = check_cfg(cfg))) return st;
  if (B < 1) return fail(LRNR_EINVAL, "batch %d < 1", B);
  if (!s || !mu) return fail(LRNR_EINVAL, "s or mu is NULL");
  if (grad && !grad_s) return fail(LRNR_EINVAL, "grad_s is NULL");
  if (!grad && !loss) return fail(LRNR_EINVAL, "loss is NULL");
  Plan p = make_plan(k, RP, Wmax_p, pts, B, grad);
  if ((int64_t)B * p.grid.G_inst > 0x7fffffff) return fail(LRNR_EUNSUPPORTED, "grid too large");
  if (!ws || ws_bytes < p.total)
    return fail(LRNR_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.total);
  if ((uintptr_t)ws & 255) return fail(LRNR_EINVAL, "workspace not 256-byte aligned");
  char* base = static_cast<char*>(ws);
  p.grid.partials = reinterpret_cast<float*>(base + p.off_partials);
  p.grid.ckpt = grad ? reinterpret_cast<float*>(base + p.off_ckpt) : nullptr;
  p.grid.flags = grad ? reinterpret_cast<int*>(base + p.off_flags) : nullptr;
  KInst in = make_inst(s, mu, pts, cfg);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (p.grid.G_inst > 0) {
    const bool timed = g_ev_start && g_ev_stop;
    if (timed) (void)hipEventRecord(g_ev_start, hs);
    hipError_t e = launch_fused(RP, grad ? MODE_GRAD : MODE_LOSS, k, in, p.grid, hs);
    if (timed) {
      (void)hipEventRecord(g_ev_stop, hs);
      g_ev_start = g_ev_stop = nullptr;
    }
    if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
  }
  KReduce kr{};
  kr.partials = p.grid.partials;
  kr.red1 = reinterpret_cast<double*>(base + p.off_red1);
  kr.G_inst = p.grid.G_inst;
  kr.B = B;
  kr.P = p.grid.P;
  kr.nchunk = p.nchunk;
  kr.E = grad ? 4 + k.r_total + k.b_total : 4;
  kr.r_total = k.r_total;
  kr.b_total = k.b_total;
  kr.n_r = pts->n_r;
  kr.n_0 = pts->n_0;
  kr.n_b = pts->n_b;
  kr.w_r = cfg->w_r;
  kr.w_0 = cfg->w_0;
  kr.w_b = cfg->w_b;
  kr.lambda_loc = cfg->lambda_loc;
  kr.s = s;
  kr.s_ref = cfg->s_ref;
  kr.s_stride = k.r_total;
  kr.grad_s = grad ? grad_s : nullptr;
  kr.grad_b = grad ? grad_b : nullptr;
  kr.loss = loss;
  hipError_t e = launch_reduce(kr, hs);
  if (e != hipSuccess) return hip_fail(e, "reduction launch");
  return LRNR_OK;
}

int32_t run_forward(const lrnr_net* net, const float* s, const float* xt, int64_t n, float* out,
                    void* stream, int mode) {
  KNet k;
  int RP, Wmax_p;
  int32_t st = make_knet(net, &k, &RP, &Wmax_p);
  if (st) return st;
  if (n < 0) return fail(LRNR_EINVAL, "negative point count");
  if (n == 0) return LRNR_OK;
  if (!s || !xt || !out) return fail(LRNR_EINVAL, "s, xt or output is NULL");
  lrnr_points pts{xt, n, nullptr, 0, nullptr, 0};
  if ((st = check_points(&pts))) return st;
  Plan p = make_plan(k, RP, Wmax_p, &pts, 1, false);
  KInst in = make_inst(s, nullptr, &pts, nullptr);
  in.out = out;
  hipError_t e = launch_fused(RP, mode, k, in, p.grid, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
  return LRNR_OK;
}

}  // namespace

void lrnr::set_status_detail(const char* text) { g_detail = text; }

extern "C" {

int32_t lrnr_forward_jets(const lrnr_net* net, const float* s, const float* xt, int64_t n,
                          float* jets, void* stream) {
  return run_forward(net, s, xt, n, jets, stream, MODE_JETS);
}

int32_t lrnr_forward_value(const lrnr_net* net, const float* s, const float* xt, int64_t n,
                           float* u, void* stream) {
  return run_forward(net, s, xt, n, u, stream, MODE_VALUE);
}

size_t lrnr_workspace_size(const lrnr_net* net, const lrnr_points* pts, int32_t batch) {
  KNet k;
  int RP, Wmax_p;
  if (make_knet(net, &k, &RP, &Wmax_p) || check_points(pts) || batch < 1) return 0;
  return make_plan(k, RP, Wmax_p, pts, batch, true).total;
}

int32_t lrnr_residual_loss(const lrnr_net* net, const float* s, const float* mu,
                           const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* loss, void* ws,
                           size_t ws_bytes, void* stream) {
  return run_loss(net, 1, s, mu, pts, cfg, nullptr, nullptr, loss, ws, ws_bytes, stream, false);
}

int32_t lrnr_grad_s(const lrnr_net* net, const float* s, const float* mu, const lrnr_points* pts,
                    const lrnr_loss_cfg* cfg, float* grad_s, float* grad_b, float* loss, void* ws,
                    size_t ws_bytes, void* stream) {
  return run_loss(net, 1, s, mu, pts, cfg, grad_s, grad_b, loss, ws, ws_bytes, stream, true);
}

int32_t lrnr_grad_s_batched(const lrnr_net* net, int32_t B, const float* s, const float* mu,
                            const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_s,
                            float* loss, void* ws, size_t ws_bytes, void* stream) {
  return run_loss(net, B, s, mu, pts, cfg, grad_s, nullptr, loss, ws, ws_bytes, stream, true);
}

int32_t lrnr_grad_s_noalloc(const lrnr_net* net, const float* s, const float* mu,
                            const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_s,
                            float* grad_b, float* loss, void* stream) {
  // sizes beyond the fixed scratch are refused before any device work (an
  // invalid net or point set gives 0 here and is reported by run_loss)
  const size_t need = lrnr_workspace_size(net, pts, 1);
  if (need > kScratchBytes)
    return fail(LRNR_EUNSUPPORTED, "needs %zu bytes of workspace, the fixed scratch holds %zu",
                need, kScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices)
    return fail(LRNR_EUNSUPPORTED, "device %d beyond the %d the scratch table covers", dev,
                kScratchDevices);
  void* ws = nullptr;
  {
    // set-up, once per device with that device current: the array's address
    // on this GPU (each GPU holds its own copy at its own address)
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
      if (!ptr) return fail(LRNR_EHIP, "scratch has no device address");
      g_scratch_ptr[dev] = ptr;
    }
    ws = g_scratch_ptr[dev];
  }
  return run_loss(net, 1, s, mu, pts, cfg, grad_s, grad_b, loss, ws, kScratchBytes, stream,
                  true);
}

int32_t lrnr_adam_step(float* s, float* m, float* v, const float* g, int64_t n, int32_t step,
                       float lr, float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || step < 1) return fail(LRNR_EINVAL, "n=%lld step=%d", (long long)n, step);
  if (n > 0 && (!s || !m || !v || !g)) return fail(LRNR_EINVAL, "NULL Adam array");
  hipError_t e = launch_adam(s, m, v, g, n, step, lr, beta1, beta2, eps,
                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return LRNR_OK;
}

int32_t lrnr_time_next_fused(void* start_event, void* stop_event) {
  if ((start_event == nullptr) != (stop_event == nullptr))
    return fail(LRNR_EINVAL, "both events or neither");
  g_ev_start = static_cast<hipEvent_t>(start_event);
  g_ev_stop = static_cast<hipEvent_t>(stop_event);
  return LRNR_OK;
}

const char* lrnr_status_string(int32_t status) {
  static thread_local std::string msg;
  const char* base = "unknown status";
  switch (status) {
    case LRNR_OK: base = "ok"; break;
    case LRNR_EINVAL: base = "invalid argument"; break;
    case LRNR_ENOMEM: base = "out of memory / workspace too small"; break;
    case LRNR_EHIP: base = "HIP runtime error"; break;
    case LRNR_ESINGULAR: base = "singular POD/DEIM system"; break;
    case LRNR_EUNSUPPORTED: base = "unsupported size"; break;
  }
  msg = base;
  if (status != LRNR_OK && !g_detail.empty()) msg += ": " + g_detail;
  return msg.c_str();
}

}  // extern "C"
