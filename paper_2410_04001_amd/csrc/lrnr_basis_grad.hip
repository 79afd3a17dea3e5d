// Gradient of the physics-informed loss with respect to the bases U^l and
// V^l (the meta-learning phase of Section 3.1 trains them, eq. 3.4), for one
// instance or the mean over B instances that share the net and the points:
//   dL/dU^l = sum_p sum_c abar^l_{p,c} (s^l * y^l_{p,c})^T,
//   dL/dV^l = sum_p sum_c z^{l-1}_{p,c} ybar^l_{p,c}^T.
// The terms are formed inside the fused sweeps (lrnr_basis_fused.h), one
// record per wave; the records are summed here in a fixed order in FP64
// (chunks of 32 records, then the chunks), so results are bitwise
// reproducible and independent of the launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lrnr_basis_fused.h"

namespace lrnr {
namespace {

constexpr int kBgSumThreads = 256;
constexpr int kBgChunk = 32;  // records per first-stage partial sum

struct BasisPlan {
  KGrid grid;
  int PB, U_total, V_total;
  int64_t records, nchunk;
  size_t off_wrec, off_red1, off_ckpt, total;
};

BasisPlan basis_plan(const KNet& k, int RP, int Wmax_p, const lrnr_points* pts, int B) {
  BasisPlan p{};
  KGrid& g = p.grid;
  g.G_r = (int)((pts->n_r + kPtsPerWG - 1) / kPtsPerWG);
  g.G_0 = (int)((pts->n_0 + kPtsPerWG - 1) / kPtsPerWG);
  g.G_b = (int)((pts->n_b + kBcPairsPerWG - 1) / kBcPairsPerWG);
  g.G_inst = g.G_r + g.G_0 + g.G_b;
  g.B = B;
  g.Wmax_p = Wmax_p;
  g.s_stride = k.r_total;
  g.ckpt_per_wave = (int64_t)(k.L - 1) * 4 * (RP / 4) * 64 * 4;
  int u = 0, v = 0;
  for (int l = 1; l <= k.L; ++l) {
    u += k.M[l] * k.r[l];
    v += k.M[l - 1] * k.r[l];
  }
  p.U_total = u;
  p.V_total = v;
  p.PB = (u + v + 3) & ~3;
  p.records = (int64_t)B * g.G_inst * kWaves;
  p.nchunk = (p.records + kBgChunk - 1) / kBgChunk;
  size_t off = 0;
  p.off_wrec = off;
  off = align256(off + (size_t)p.records * p.PB * sizeof(float));
  p.off_red1 = off;
  // the levels of the fixed-order tree ping-pong between two regions: the
  // first level's partials and room for the second's
  const int64_t n2 = (p.nchunk + kBgChunk - 1) / kBgChunk;
  off = align256(off + (size_t)(std::max<int64_t>(p.nchunk, 1) + n2) * p.PB * sizeof(double));
  p.off_ckpt = off;
  off = align256(off + (size_t)p.records * g.ckpt_per_wave * sizeof(float));
  p.total = std::max(off, (size_t)256);
  return p;
}

// Partial sums of chunk blockIdx.y of the wave records, entries ascending.
__global__ void __launch_bounds__(kBgSumThreads) basis_sum1_kernel(const float* wrec, int PB,
                                                                   int n_used, int64_t records,
                                                                   double* red1) {
  const int e = blockIdx.x * kBgSumThreads + threadIdx.x;
  if (e >= n_used) return;
  const int64_t r0 = (int64_t)blockIdx.y * kBgChunk;
  const int64_t r1 = r0 + kBgChunk < records ? r0 + kBgChunk : records;
  const float* p = wrec + r0 * PB + e;
  double acc = 0.0;
  int64_t r = r0;
  // loads eight records at a time, additions in record order
  for (; r + 8 <= r1; r += 8) {
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[(int64_t)i * PB];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc += (double)v[i];
    p += (int64_t)8 * PB;
  }
  for (; r < r1; ++r, p += PB) acc += (double)*p;
  red1[(int64_t)blockIdx.y * PB + e] = acc;
}

// Next level of the tree: partial sums of chunk blockIdx.y of kBgChunk
// consecutive FP64 partials (in order).
__global__ void __launch_bounds__(kBgSumThreads) basis_sumd_kernel(const double* in, int PB,
                                                                   int n_used, int64_t n_in,
                                                                   double* out) {
  const int e = blockIdx.x * kBgSumThreads + threadIdx.x;
  if (e >= n_used) return;
  const int64_t c0 = (int64_t)blockIdx.y * kBgChunk;
  const int64_t c1 = c0 + kBgChunk < n_in ? c0 + kBgChunk : n_in;
  double acc = 0.0;
  for (int64_t c = c0; c < c1; ++c) acc += in[c * PB + e];
  out[(int64_t)blockIdx.y * PB + e] = acc;
}

// The last level (at most kBgChunk partials) in order, the mean over the B
// instances, into grad_U (entries [0, U_total)) and grad_V (the rest).
__global__ void __launch_bounds__(kBgSumThreads) basis_sum2_kernel(const double* red, int PB,
                                                                   int U_total, int n_used,
                                                                   int64_t n_in, double invB,
                                                                   float* gU, float* gV) {
  const int e = blockIdx.x * kBgSumThreads + threadIdx.x;
  if (e >= n_used) return;
  double acc = 0.0;
  for (int64_t c = 0; c < n_in; ++c) acc += red[c * PB + e];
  const float v = (float)(acc * invB);
  if (e < U_total)
    gU[e] = v;
  else
    gV[e - U_total] = v;
}

__global__ void __launch_bounds__(kBgSumThreads) basis_zero_kernel(int U_total, int n_used,
                                                                   float* gU, float* gV) {
  const int e = blockIdx.x * kBgSumThreads + threadIdx.x;
  if (e >= n_used) return;
  if (e < U_total)
    gU[e] = 0.f;
  else
    gV[e - U_total] = 0.f;
}

template <int RP>
hipError_t launch_basis(const KBasis& kb, int blocks, hipStream_t stream) {
  const size_t lds = basis_lds_bytes(RP, kb.grid.Wmax_p);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)lrnr_basis_kernel<RP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(lrnr_basis_kernel<RP>, dim3(blocks), dim3(kThreads), lds, stream, kb);
  return hipGetLastError();
}

hipError_t launch_basis_rp(int RP, const KBasis& kb, int blocks, hipStream_t stream) {
  switch (RP) {
    case 4: return launch_basis<4>(kb, blocks, stream);
    case 8: return launch_basis<8>(kb, blocks, stream);
    case 16: return launch_basis<16>(kb, blocks, stream);
    case 20: return launch_basis<20>(kb, blocks, stream);
    case 24: return launch_basis<24>(kb, blocks, stream);
    case 32: return launch_basis<32>(kb, blocks, stream);
    default: return hipErrorInvalidValue;
  }
}

int32_t basis_grad(const lrnr_net* net, int B, const float* s, const float* mu,
                   const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_U,
                   float* grad_V, void* ws, size_t ws_bytes, void* stream) {
  KNet k;
  int RP, Wp;
  int32_t rc = make_knet(net, &k, &RP, &Wp);
  if (rc != LRNR_OK) return rc;
  if ((rc = check_points(pts)) != LRNR_OK) return rc;
  if ((rc = check_cfg(cfg)) != LRNR_OK) return rc;
  if (B < 1) return fail(LRNR_EINVAL, "B=%d (at least one instance)", B);
  if (!s || !mu || !grad_U || !grad_V) return fail(LRNR_EINVAL, "NULL s, mu or gradient");
  BasisPlan p = basis_plan(k, RP, Wp, pts, B);
  if ((int64_t)B * p.grid.G_inst > 0x7fffffff) return fail(LRNR_EUNSUPPORTED, "grid too large");
  if (!ws || ws_bytes < p.total)
    return fail(LRNR_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.total);
  if ((uintptr_t)ws & 255) return fail(LRNR_EINVAL, "workspace not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  KBasis kb{};
  kb.net = k;
  KInst& in = kb.inst;
  in.s = s;
  in.mu = mu;
  in.xt_r = pts->xt_r;
  in.x_0 = pts->x_0;
  in.t_b = pts->t_b;
  in.n_r = pts->n_r;
  in.n_0 = pts->n_0;
  in.n_b = pts->n_b;
  in.form = cfg->form;
  in.wr_n = pts->n_r ? (float)((double)cfg->w_r / (double)pts->n_r) : 0.f;
  in.w0_n = pts->n_0 ? (float)((double)cfg->w_0 / (double)pts->n_0) : 0.f;
  in.wb_n = pts->n_b ? (float)((double)cfg->w_b / (double)pts->n_b) : 0.f;
  kb.grid = p.grid;
  kb.grid.ckpt = reinterpret_cast<float*>(base + p.off_ckpt);
  kb.wrec = reinterpret_cast<float*>(base + p.off_wrec);
  kb.PB = p.PB;
  kb.U_total = p.U_total;
  const int n_used = p.U_total + p.V_total;
  const unsigned nb = (unsigned)((n_used + kBgSumThreads - 1) / kBgSumThreads);
  double* red1 = reinterpret_cast<double*>(base + p.off_red1);
  hipError_t e;
  if (p.grid.G_inst == 0) {
    // no points: the gradient is zero
    hipLaunchKernelGGL(basis_zero_kernel, dim3(nb), dim3(kBgSumThreads), 0, st, p.U_total,
                       n_used, grad_U, grad_V);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "basis gradient zero launch");
    return LRNR_OK;
  }
  if ((e = launch_basis_rp(RP, kb, B * p.grid.G_inst, st)) != hipSuccess)
    return hip_fail(e, "basis gradient kernel launch");
  hipLaunchKernelGGL(basis_sum1_kernel, dim3(nb, (unsigned)p.nchunk), dim3(kBgSumThreads), 0, st,
                     kb.wrec, p.PB, n_used, p.records, red1);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "basis gradient sum launch");
  // fixed-order tree over the partials: levels of kBgChunk until one remains
  double* cur = red1;
  double* other = red1 + (size_t)std::max<int64_t>(p.nchunk, 1) * p.PB;
  int64_t n_in = p.nchunk;
  while (n_in > kBgChunk) {
    const int64_t n_out = (n_in + kBgChunk - 1) / kBgChunk;
    hipLaunchKernelGGL(basis_sumd_kernel, dim3(nb, (unsigned)n_out), dim3(kBgSumThreads), 0, st,
                       cur, p.PB, n_used, n_in, other);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "basis gradient sum launch");
    std::swap(cur, other);
    n_in = n_out;
  }
  hipLaunchKernelGGL(basis_sum2_kernel, dim3(nb), dim3(kBgSumThreads), 0, st, cur, p.PB,
                     p.U_total, n_used, n_in, 1.0 / (double)B, grad_U, grad_V);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "basis gradient sum launch");
  return LRNR_OK;
}

size_t basis_ws_size(const lrnr_net* net, const lrnr_points* pts, int B) {
  KNet k;
  int RP, Wp;
  if (make_knet(net, &k, &RP, &Wp) != LRNR_OK || check_points(pts) != LRNR_OK || B < 1) return 0;
  return basis_plan(k, RP, Wp, pts, B).total;
}

}  // namespace
}  // namespace lrnr

using namespace lrnr;

extern "C" {

size_t lrnr_basis_grad_workspace_size(const lrnr_net* net, const lrnr_points* pts) {
  return basis_ws_size(net, pts, 1);
}

size_t lrnr_basis_grad_batched_workspace_size(const lrnr_net* net, const lrnr_points* pts,
                                              int32_t B) {
  return basis_ws_size(net, pts, B);
}

int32_t lrnr_basis_grad(const lrnr_net* net, const float* s, const float* mu,
                        const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_U,
                        float* grad_V, void* ws, size_t ws_bytes, void* stream) {
  return basis_grad(net, 1, s, mu, pts, cfg, grad_U, grad_V, ws, ws_bytes, stream);
}

int32_t lrnr_basis_grad_batched(const lrnr_net* net, int32_t B, const float* s, const float* mu,
                                const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_U,
                                float* grad_V, void* ws, size_t ws_bytes, void* stream) {
  return basis_grad(net, B, s, mu, pts, cfg, grad_U, grad_V, ws, ws_bytes, stream);
}

}  // extern "C"
