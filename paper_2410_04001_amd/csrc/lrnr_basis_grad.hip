// Gradient of the physics-informed loss with respect to the bases U^l and
// V^l (the meta-learning phase of Section 3.1 trains them, eq. 3.4):
//   dL/dU^l = sum_p sum_c abar^l_{p,c} (s^l * y^l_{p,c})^T,
//   dL/dV^l = sum_p sum_c z^{l-1}_{p,c} ybar^l_{p,c}^T,
// with c over the jets (value, d/dx, d/dt, d2/dx2), abar^l the adjoint of the
// pre-activation of layer l, y^l = V^lT z^{l-1} its reduced input and ybar^l
// the adjoint of y^l.  Not the hot path: one thread per evaluation point runs
// the forward and reverse jets and leaves w = s * y, a, abar and ybar in a
// caller workspace; every entry of the two gradients is then a sum over the
// points, taken as partial sums over fixed chunks of points and a sum of the
// chunks in order (FP64), so the result is bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lrnr_internal.h"

namespace lrnr {
namespace {

constexpr int kBgThreads = 64;    // per-point kernels: more workgroups, more CUs busy
constexpr int kBgSumThreads = 256;
constexpr int kBgChunks = 64;     // point chunks of the contraction
constexpr float kTwoPi = 6.28318530717958647692f;

struct KBg {
  KNet k;
  const float* s;
  const float* mu;                // [3] (beta, nu, rho), device
  const float* xt_r;
  const float* x_0;
  const float* t_b;
  int64_t n_r, n_0, n_b, E;       // E = n_r + n_0 + 2 n_b evaluation points
  int form;
  float wr_n, w0_n, wb_n;         // w_r / n_r, w_0 / n_0, w_b / n_b
  // workspace (floats), each [E][4][dim]
  float* W[LRNR_MAX_LAYERS + 1];      // s^l * y^l, dim r_l (l = 1..L)
  float* A[LRNR_MAX_LAYERS + 1];      // a^l, dim M_l (l = 1..L-1)
  float* Abar[LRNR_MAX_LAYERS + 1];   // abar^l, dim M_l (l = 1..L)
  float* Ybar[LRNR_MAX_LAYERS + 1];   // ybar^l, dim r_l (l = 1..L)
  float* Ujet;                        // [E][4]
  double* part;                       // [chunks][n_out] partial sums
  int chunks;
  int64_t n_out;
};

__device__ inline void point_xt(const KBg& g, int64_t e, float& x, float& t) {
  if (e < g.n_r) {
    x = g.xt_r[2 * e];
    t = g.xt_r[2 * e + 1];
  } else if (e < g.n_r + g.n_0) {
    x = g.x_0[e - g.n_r];
    t = 0.f;
  } else {
    const int64_t j = e - g.n_r - g.n_0;
    x = (j & 1) ? kTwoPi : 0.f;
    t = g.t_b[j >> 1];
  }
}

// forward jets; stores W, A and the output jets (RPT >= every rank of the net)
template <int RPT>
__global__ void __launch_bounds__(kBgThreads) bg_forward_kernel(KBg g) {
  const int64_t e = (int64_t)blockIdx.x * kBgThreads + threadIdx.x;
  if (e >= g.E) return;
  const KNet& k = g.k;
  float x, t;
  point_xt(g, e, x, t);
  float y[4][RPT];
  const int r1 = k.r[1];
  const float* V1 = k.V + k.offV[1];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const bool on = j < r1;
    y[0][j] = on ? V1[j] * x + V1[r1 + j] * t : 0.f;
    y[1][j] = on ? V1[j] : 0.f;
    y[2][j] = on ? V1[r1 + j] : 0.f;
    y[3][j] = 0.f;
  }
  for (int l = 1; l <= k.L; ++l) {
    const int M = k.M[l], rl = k.r[l];
    const float* U = k.U + k.offU[l];
    const float* b = k.b + k.offB[l];
    const float* sl = g.s + k.offS[l];
    float* W = g.W[l] + e * 4 * rl;
#pragma unroll
    for (int j = 0; j < RPT; ++j)
      if (j < rl) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          y[c][j] *= sl[j];
          W[c * rl + j] = y[c][j];
        }
      }
    if (l == k.L) {   // linear output, M_L = 1
      float u[4] = {b[0], 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j < rl)
#pragma unroll
          for (int c = 0; c < 4; ++c) u[c] = fmaf(U[j], y[c][j], u[c]);
#pragma unroll
      for (int c = 0; c < 4; ++c) g.Ujet[e * 4 + c] = u[c];
      break;
    }
    const int ro = k.r[l + 1];
    const float* V = k.V + k.offV[l + 1];
    float* A = g.A[l] + e * 4 * M;
    float yn[4][RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) yn[c][j] = 0.f;
    for (int i = 0; i < M; ++i) {
      float a[4] = {b[i], 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j < rl)
#pragma unroll
          for (int c = 0; c < 4; ++c) a[c] = fmaf(U[i * rl + j], y[c][j], a[c]);
#pragma unroll
      for (int c = 0; c < 4; ++c) A[c * M + i] = a[c];
      const float sv = sinf(a[0]), cv = cosf(a[0]);
      const float z[4] = {sv, cv * a[1], cv * a[2], cv * a[3] - sv * a[1] * a[1]};
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j < ro)
#pragma unroll
          for (int c = 0; c < 4; ++c) yn[c][j] = fmaf(V[i * ro + j], z[c], yn[c][j]);
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c][j] = yn[c][j];
  }
}

__device__ inline float dphi(float v, int form) {
  return form == 0 ? 2.f * v : (v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f));
}

// output adjoint from the loss, then the reverse jets; stores Abar and Ybar
template <int RPT>
__global__ void __launch_bounds__(kBgThreads) bg_reverse_kernel(KBg g) {
  const int64_t e = (int64_t)blockIdx.x * kBgThreads + threadIdx.x;
  if (e >= g.E) return;
  const KNet& k = g.k;
  const float* u = g.Ujet + e * 4;
  float ub[4] = {0.f, 0.f, 0.f, 0.f};
  if (e < g.n_r) {
    const float beta = g.mu[0], nu = g.mu[1], rho = g.mu[2];
    const float res = u[2] + beta * u[1] - nu * u[3] - rho * u[0] * (1.f - u[0]);
    const float gr = g.wr_n * dphi(res, g.form);
    ub[0] = -rho * (1.f - 2.f * u[0]) * gr;
    ub[1] = beta * gr;
    ub[2] = gr;
    ub[3] = -nu * gr;
  } else if (e < g.n_r + g.n_0) {
    const float x = g.x_0[e - g.n_r];
    ub[0] = g.w0_n * dphi(u[0] - sinf(x), g.form);
  } else {
    const int64_t j = e - g.n_r - g.n_0;
    const int64_t left = e - (j & 1);
    const float d = g.Ujet[left * 4] - g.Ujet[(left + 1) * 4];
    const float gb = g.wb_n * dphi(d, g.form);
    ub[0] = (j & 1) ? -gb : gb;
  }
  // output layer: abar^L = ubar, wbar = U^L ubar, ybar^L = s^L * wbar
  float yb[4][RPT];
  {
    const int L = k.L, rl = k.r[L];
    const float* U = k.U + k.offU[L];
    const float* sl = g.s + k.offS[L];
#pragma unroll
    for (int c = 0; c < 4; ++c) g.Abar[L][e * 4 + c] = ub[c];
    float* Yb = g.Ybar[L] + e * 4 * rl;
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        yb[c][j] = (j < rl) ? sl[j] * U[j] * ub[c] : 0.f;
        if (j < rl) Yb[c * rl + j] = yb[c][j];
      }
  }
  for (int l = k.L - 1; l >= 1; --l) {
    const int M = k.M[l], rl = k.r[l], ro = k.r[l + 1];
    const float* U = k.U + k.offU[l];
    const float* V = k.V + k.offV[l + 1];
    const float* sl = g.s + k.offS[l];
    const float* A = g.A[l] + e * 4 * M;
    float* Ab = g.Abar[l] + e * 4 * M;
    float wb[4][RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) wb[c][j] = 0.f;
    for (int i = 0; i < M; ++i) {
      float zb[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j < ro)
#pragma unroll
          for (int c = 0; c < 4; ++c) zb[c] = fmaf(V[i * ro + j], yb[c][j], zb[c]);
      const float a0 = A[i], a1 = A[M + i], a2 = A[2 * M + i], a3 = A[3 * M + i];
      const float sv = sinf(a0), cv = cosf(a0);
      // z = (sin a0, cos a0 a1, cos a0 a2, cos a0 a3 - sin a0 a1^2)
      float ab[4];
      ab[0] = zb[0] * cv - zb[1] * sv * a1 - zb[2] * sv * a2 - zb[3] * (sv * a3 + cv * a1 * a1);
      ab[1] = zb[1] * cv - zb[3] * 2.f * sv * a1;
      ab[2] = zb[2] * cv;
      ab[3] = zb[3] * cv;
#pragma unroll
      for (int c = 0; c < 4; ++c) Ab[c * M + i] = ab[c];
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j < rl)
#pragma unroll
          for (int c = 0; c < 4; ++c) wb[c][j] = fmaf(U[i * rl + j], ab[c], wb[c][j]);
    }
    float* Yb = g.Ybar[l] + e * 4 * rl;
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        yb[c][j] = (j < rl) ? sl[j] * wb[c][j] : 0.f;
        if (j < rl) Yb[c * rl + j] = yb[c][j];
      }
  }
}

// Gradient entry id -> layer, U or V, row and column (U^l then V^l, l = 1..L).
__device__ inline bool bg_decode(const KNet& k, int64_t id, int& l, bool& isU, int& i, int& j) {
  int64_t rem = id;
  for (l = 1; l <= k.L; ++l) {
    const int64_t nu = (int64_t)k.M[l] * k.r[l], nv = (int64_t)k.M[l - 1] * k.r[l];
    if (rem < nu) {
      isU = true;
      break;
    }
    rem -= nu;
    if (rem < nv) {
      isU = false;
      break;
    }
    rem -= nv;
  }
  if (l > k.L) return false;
  i = (int)(rem / k.r[l]);
  j = (int)(rem - (int64_t)i * k.r[l]);
  return true;
}

// Partial sums over chunk blockIdx.y of the points, one thread per gradient
// entry: U^l[i][j] += Abar[e][c][i] W[e][c][j], V^l[i][j] += Z^{l-1}[e][c][i]
// Ybar[e][c][j], points ascending within the chunk, FP64.
__global__ void __launch_bounds__(kBgSumThreads) bg_contract_kernel(KBg g) {
  const KNet& k = g.k;
  const int64_t id = (int64_t)blockIdx.x * kBgSumThreads + threadIdx.x;
  int l, i, j;
  bool isU;
  if (id >= g.n_out || !bg_decode(k, id, l, isU, i, j)) return;
  const int64_t e0 = g.E * blockIdx.y / g.chunks, e1 = g.E * (blockIdx.y + 1) / g.chunks;
  const int rl = k.r[l];
  double acc = 0.0;
  if (isU) {
    const int M = k.M[l];
    const float* Ab = g.Abar[l];
    const float* W = g.W[l];
    for (int64_t e = e0; e < e1; ++e)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc += (double)Ab[(e * 4 + c) * M + i] * (double)W[(e * 4 + c) * rl + j];
  } else {
    const float* Yb = g.Ybar[l];
    for (int64_t e = e0; e < e1; ++e) {
      float z[4];
      if (l == 1) {
        float x, t;
        point_xt(g, e, x, t);
        z[0] = i == 0 ? x : t;
        z[1] = i == 0 ? 1.f : 0.f;
        z[2] = i == 0 ? 0.f : 1.f;
        z[3] = 0.f;
      } else {
        const int Mp = k.M[l - 1];
        const float* A = g.A[l - 1] + e * 4 * Mp;
        const float a0 = A[i], a1 = A[Mp + i], a2 = A[2 * Mp + i], a3 = A[3 * Mp + i];
        const float sv = sinf(a0), cv = cosf(a0);
        z[0] = sv;
        z[1] = cv * a1;
        z[2] = cv * a2;
        z[3] = cv * a3 - sv * a1 * a1;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) acc += (double)z[c] * (double)Yb[(e * 4 + c) * rl + j];
    }
  }
  g.part[(int64_t)blockIdx.y * g.n_out + id] = acc;
}

// Sum of the chunks in order, into grad_U / grad_V.
__global__ void __launch_bounds__(kBgSumThreads) bg_sum_kernel(KBg g, float* gU, float* gV) {
  const KNet& k = g.k;
  const int64_t id = (int64_t)blockIdx.x * kBgSumThreads + threadIdx.x;
  int l, i, j;
  bool isU;
  if (id >= g.n_out || !bg_decode(k, id, l, isU, i, j)) return;
  double acc = 0.0;
  for (int c = 0; c < g.chunks; ++c) acc += g.part[(int64_t)c * g.n_out + id];
  const int rl = k.r[l];
  if (isU)
    gU[k.offU[l] + i * rl + j] = (float)acc;
  else
    gV[k.offV[l] + i * rl + j] = (float)acc;
}

// workspace floats of each array (and the total), for E points
int64_t bg_layout(const KNet& k, int64_t E, KBg* g, float* base) {
  int64_t o = 0;
  auto take = [&](int64_t n) {
    float* p = base ? base + o : nullptr;
    o += (n + 63) & ~int64_t(63);
    return p;
  };
  for (int l = 1; l <= k.L; ++l) {
    g->W[l] = take(E * 4 * k.r[l]);
    g->Ybar[l] = take(E * 4 * k.r[l]);
    g->Abar[l] = take(E * 4 * k.M[l]);
    g->A[l] = (l < k.L) ? take(E * 4 * k.M[l]) : nullptr;
  }
  g->Ujet = take(E * 4);
  int64_t n_out = 0;
  for (int l = 1; l <= k.L; ++l) n_out += (int64_t)(k.M[l] + k.M[l - 1]) * k.r[l];
  g->n_out = n_out;
  g->chunks = (int)(E / 256 < kBgChunks ? (E / 256 > 0 ? E / 256 : 1) : kBgChunks);
  g->part = reinterpret_cast<double*>(take(2 * (int64_t)g->chunks * n_out));
  return o;
}

}  // namespace
}  // namespace lrnr

using namespace lrnr;

extern "C" {

size_t lrnr_basis_grad_workspace_size(const lrnr_net* net, const lrnr_points* pts) {
  KNet k;
  int RP, Wp;
  if (make_knet(net, &k, &RP, &Wp) != LRNR_OK || check_points(pts) != LRNR_OK) return 0;
  KBg g{};
  const int64_t E = pts->n_r + pts->n_0 + 2 * pts->n_b;
  return align256((size_t)bg_layout(k, E, &g, nullptr) * sizeof(float));
}

int32_t lrnr_basis_grad(const lrnr_net* net, const float* s, const float* mu,
                        const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_U,
                        float* grad_V, void* ws, size_t ws_bytes, void* stream) {
  KBg g{};
  int RP, Wp;
  int32_t rc = make_knet(net, &g.k, &RP, &Wp);
  if (rc != LRNR_OK) return rc;
  if ((rc = check_points(pts)) != LRNR_OK) return rc;
  if ((rc = check_cfg(cfg)) != LRNR_OK) return rc;
  if (!s || !mu || !grad_U || !grad_V) return fail(LRNR_EINVAL, "NULL s, mu or gradient");
  const size_t need = lrnr_basis_grad_workspace_size(net, pts);
  if (!ws || ws_bytes < need) return fail(LRNR_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  g.s = s;
  g.mu = mu;
  g.xt_r = pts->xt_r;
  g.x_0 = pts->x_0;
  g.t_b = pts->t_b;
  g.n_r = pts->n_r;
  g.n_0 = pts->n_0;
  g.n_b = pts->n_b;
  g.E = pts->n_r + pts->n_0 + 2 * pts->n_b;
  g.form = cfg->form;
  g.wr_n = pts->n_r ? cfg->w_r / (float)pts->n_r : 0.f;
  g.w0_n = pts->n_0 ? cfg->w_0 / (float)pts->n_0 : 0.f;
  g.wb_n = pts->n_b ? cfg->w_b / (float)pts->n_b : 0.f;
  bg_layout(g.k, g.E, &g, static_cast<float*>(ws));
  if (g.E > 0) {
    const unsigned nb = (unsigned)((g.E + kBgThreads - 1) / kBgThreads);
    int rmax = 1;
    for (int l = 1; l <= g.k.L; ++l) rmax = g.k.r[l] > rmax ? g.k.r[l] : rmax;
    auto fwd = rmax <= 8 ? bg_forward_kernel<8>
             : rmax <= 16 ? bg_forward_kernel<16> : bg_forward_kernel<LRNR_MAX_RANK>;
    auto rev = rmax <= 8 ? bg_reverse_kernel<8>
             : rmax <= 16 ? bg_reverse_kernel<16> : bg_reverse_kernel<LRNR_MAX_RANK>;
    hipLaunchKernelGGL(fwd, dim3(nb), dim3(kBgThreads), 0, st, g);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "basis gradient forward launch");
    hipLaunchKernelGGL(rev, dim3(nb), dim3(kBgThreads), 0, st, g);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "basis gradient reverse launch");
  }
  const unsigned nc = (unsigned)((g.n_out + kBgSumThreads - 1) / kBgSumThreads);
  hipLaunchKernelGGL(bg_contract_kernel, dim3(nc, g.chunks), dim3(kBgSumThreads), 0, st, g);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "basis gradient contraction launch");
  hipLaunchKernelGGL(bg_sum_kernel, dim3(nc), dim3(kBgSumThreads), 0, st, g, grad_U, grad_V);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "basis gradient sum launch");
  return LRNR_OK;
}

}  // extern "C"
