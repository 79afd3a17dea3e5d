// Meta-learning of the coefficient map (Section 3.1): the hypernetwork
// s = f_hyper(mu; Theta) (eq. 3.1), a network of the form of eq. 2.1 with the
// activation sin and a ReLU on its output, and the Theta gradient of the meta
// objective of eq. 3.4 with the bases held fixed:
//   (1/B) sum_b [ L(s_b; mu_b) + lambda R_sparse(s_b) ],
// where dL/ds_b comes from the batched loss gradient and R_sparse (eq. 3.3)
// is sum_l || ReLU(Gamma^l s^l) ||_1 with Gamma^l banded (-1 on the diagonal,
// gamma above it).
//
// The network is small (widths <= 256): forward and per-sample backward run
// one workgroup per sample; the per-sample gradients land in rows of a caller
// workspace and are summed over the samples in a fixed order (FP64), which
// keeps the result deterministic without atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "lrnr_internal.h"

namespace lrnr {
namespace {

constexpr int kHyperThreads = 256;
constexpr int kHyperMaxW = 256;

struct KHyper {
  int K;
  int H[LRNR_MAX_LAYERS + 1];
  int64_t offW[LRNR_MAX_LAYERS + 1];
  int64_t offC[LRNR_MAX_LAYERS + 1];
  const float* theta;
  // coefficient layout of the LRNR (for R_sparse): layer of each entry
  int L;
  int offS[LRNR_MAX_LAYERS + 2];
};

__global__ void __launch_bounds__(kHyperThreads) hyper_forward_kernel(KHyper f, const float* mu,
                                                                      float* s) {
  __shared__ float h[2][kHyperMaxW];
  const int b = blockIdx.x, tid = threadIdx.x;
  if (tid < 3) h[0][tid] = mu[3 * b + tid];
  __syncthreads();
  int cur = 0;
  for (int k = 1; k <= f.K; ++k) {
    const int Hp = f.H[k - 1], Hk = f.H[k];
    const float* W = f.theta + f.offW[k];
    const float* c = f.theta + f.offC[k];
    for (int j = tid; j < Hk; j += kHyperThreads) {
      float a = c[j];
      for (int i = 0; i < Hp; ++i) a = fmaf(W[(int64_t)j * Hp + i], h[cur][i], a);
      h[cur ^ 1][j] = (k < f.K) ? sinf(a) : fmaxf(a, 0.f);
    }
    __syncthreads();
    cur ^= 1;
  }
  const int R = f.H[f.K];
  for (int j = tid; j < R; j += kHyperThreads) s[(int64_t)b * R + j] = h[cur][j];
}

// One workgroup per sample b: forward, then the gradient of
// <(s_bar_b + lambda dR_b/ds) / B, s_b> with respect to Theta into row b of the
// workspace, and R_sparse(s_b) into its last entry.
__global__ void __launch_bounds__(kHyperThreads) hyper_sample_grad_kernel(
    KHyper f, int B, const float* mu, const float* s_bar, float gamma, float lam, float* ws,
    int64_t n_theta) {
  __shared__ float hin[LRNR_MAX_LAYERS + 1][kHyperMaxW];   // input of layer k at [k]
  __shared__ float pre[LRNR_MAX_LAYERS + 1][kHyperMaxW];   // pre-activation of layer k
  __shared__ float g[2][kHyperMaxW];
  __shared__ float red[kHyperThreads];
  const int b = blockIdx.x, tid = threadIdx.x, K = f.K, R = f.H[K];
  const float invB = 1.0f / (float)B;
  float* grad = ws + (int64_t)b * (n_theta + 1);
  if (tid < 3) hin[1][tid] = mu[3 * b + tid];
  __syncthreads();
  for (int k = 1; k <= K; ++k) {
    const int Hp = f.H[k - 1], Hk = f.H[k];
    const float* W = f.theta + f.offW[k];
    const float* c = f.theta + f.offC[k];
    for (int j = tid; j < Hk; j += kHyperThreads) {
      float a = c[j];
      for (int i = 0; i < Hp; ++i) a = fmaf(W[(int64_t)j * Hp + i], hin[k][i], a);
      pre[k][j] = a;
      if (k < K) hin[k + 1][j] = sinf(a);
    }
    __syncthreads();
  }
  // output gradient: ReLU, plus the R_sparse term on s = ReLU(pre_K)
  float rsum = 0.f;
  for (int m = tid; m < R; m += kHyperThreads) {
    int l = 1;
    while (m >= f.offS[l + 1]) ++l;
    const int i = m - f.offS[l], rl = f.offS[l + 1] - f.offS[l];
    const float sm = fmaxf(pre[K][m], 0.f);
    float dr = 0.f;
    if (i + 1 < rl) {
      const float t = -sm + gamma * fmaxf(pre[K][m + 1], 0.f);
      if (t > 0.f) {
        dr -= 1.f;
        rsum += t;
      }
    }
    if (i > 0) {
      const float t = -fmaxf(pre[K][m - 1], 0.f) + gamma * sm;
      if (t > 0.f) dr += gamma;
    }
    const float gs = (s_bar[(int64_t)b * R + m] + lam * dr) * invB;
    g[K & 1][m] = (pre[K][m] > 0.f) ? gs : 0.f;
  }
  red[tid] = rsum;
  __syncthreads();
  for (int k = K; k >= 1; --k) {
    const int Hp = f.H[k - 1], Hk = f.H[k];
    const float* gk = g[k & 1];
    const int64_t nW = (int64_t)Hk * Hp;
    float* gW = grad + f.offW[k];
    for (int64_t e = tid; e < nW; e += kHyperThreads) {
      const int j = (int)(e / Hp), i = (int)(e - (int64_t)j * Hp);
      gW[e] = gk[j] * hin[k][i];
    }
    float* gc = grad + f.offC[k];
    for (int j = tid; j < Hk; j += kHyperThreads) gc[j] = gk[j];
    if (k > 1) {
      const float* W = f.theta + f.offW[k];
      for (int i = tid; i < Hp; i += kHyperThreads) {
        float acc = 0.f;
        for (int j = 0; j < Hk; ++j) acc = fmaf(W[(int64_t)j * Hp + i], gk[j], acc);
        g[(k - 1) & 1][i] = acc * cosf(pre[k - 1][i]);
      }
    }
    __syncthreads();
  }
  for (int w = kHyperThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) grad[n_theta] = red[0];
}

// grad_theta[e] = sum_b ws[b][e] (b ascending, FP64); r_sparse = mean_b ws[b][n_theta]
__global__ void __launch_bounds__(kHyperThreads) hyper_sum_kernel(const float* ws, int B,
                                                                  int64_t n_theta, float* grad,
                                                                  float* r_sparse) {
  const int64_t e = (int64_t)blockIdx.x * kHyperThreads + threadIdx.x;
  const int64_t stride = n_theta + 1;
  if (e > n_theta || (e == n_theta && !r_sparse)) return;
  // loads issued eight at a time, added in sample order
  double acc = 0.0;
  int b = 0;
  for (; b + 8 <= B; b += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ws[(int64_t)(b + u) * stride + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (double)v[u];
  }
  for (; b < B; ++b) acc += (double)ws[(int64_t)b * stride + e];
  if (e < n_theta)
    grad[e] = (float)acc;
  else
    r_sparse[0] = (float)(acc / B);
}

// out[e] = (1/B) sum_b x[b][e] (b ascending, FP64, loads eight rows at a time)
__global__ void __launch_bounds__(kHyperThreads) rows_mean_kernel(const float* x, int B,
                                                                  int64_t n, float* out) {
  const int64_t e = (int64_t)blockIdx.x * kHyperThreads + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  int b = 0;
  for (; b + 8 <= B; b += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[(int64_t)(b + u) * n + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (double)v[u];
  }
  for (; b < B; ++b) acc += (double)x[(int64_t)b * n + e];
  out[e] = (float)(acc / B);
}

// R_orth of eq. 3.3 over every factor A (U^l [M_l][r_l], V^l [M_{l-1}][r_l]):
// D = A^T A - I, value += ||D||_F^2, grad A = 4 A D.  One workgroup walks the
// factors in order (a few hundred thousand multiply-adds), FP64 sums.
constexpr int kOrthThreads = 1024;

__global__ void __launch_bounds__(kOrthThreads) orth_reg_kernel(KNet k, float* value,
                                                                float* gU, float* gV) {
  __shared__ double D[LRNR_MAX_RANK * LRNR_MAX_RANK];
  __shared__ double red[kOrthThreads];
  const int tid = threadIdx.x;
  double vsum = 0.0;
  for (int f = 0; f < 2 * k.L; ++f) {
    const int l = f / 2 + 1;
    const bool isU = (f & 1) == 0;
    const int M = isU ? k.M[l] : k.M[l - 1], r = k.r[l];
    const float* A = isU ? k.U + k.offU[l] : k.V + k.offV[l];
    float* G = isU ? (gU ? gU + k.offU[l] : nullptr) : (gV ? gV + k.offV[l] : nullptr);
    for (int e = tid; e < r * r; e += kOrthThreads) {
      const int i = e / r, j = e - i * r;
      double acc = 0.0;
      for (int m = 0; m < M; ++m) acc += (double)A[m * r + i] * (double)A[m * r + j];
      const double d = acc - (i == j ? 1.0 : 0.0);
      D[e] = d;
      vsum += d * d;
    }
    __syncthreads();
    if (G) {
      for (int e = tid; e < M * r; e += kOrthThreads) {
        const int m = e / r, c = e - m * r;
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += (double)A[m * r + j] * D[j * r + c];
        G[e] = (float)(4.0 * acc);
      }
    }
    __syncthreads();
  }
  red[tid] = vsum;
  __syncthreads();
  for (int w = kOrthThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0 && value) value[0] = (float)red[0];
}

// Truncation after meta-learning: alive[m] = 1 when f_hyper's output m is
// nonzero for some sample (the ReLU output is exactly zero otherwise).
__global__ void __launch_bounds__(kHyperThreads) output_alive_kernel(const float* s, int B, int R,
                                                                     int* alive) {
  const int m = blockIdx.x * kHyperThreads + threadIdx.x;
  if (m >= R) return;
  int any = 0;
  for (int b = 0; b < B; ++b) any |= s[(int64_t)b * R + m] != 0.f;
  alive[m] = any;
}

// Gathers of the truncated factors: src[j] is the old flat coefficient index
// of new coefficient j (layer by layer, ascending).  Thread e of the grid
// strides over the U, V and theta outputs.
struct KTrunc {
  KNet old_net, new_net;
  const int* src;          // [new r_total]
  float* U;
  float* V;
  const float* theta;
  float* theta_out;
  int64_t theta_head;      // entries before the last layer's W_K (copied as is)
  int HK1;                 // H[K-1]
  int R_new;
  int64_t nU, nV, nT;      // output sizes
};

__global__ void __launch_bounds__(kHyperThreads) truncate_gather_kernel(KTrunc t) {
  const int64_t stride = (int64_t)gridDim.x * kHyperThreads;
  const int64_t e0 = (int64_t)blockIdx.x * kHyperThreads + threadIdx.x;
  const KNet& o = t.old_net;
  const KNet& n = t.new_net;
  for (int64_t e = e0; e < t.nU + t.nV; e += stride) {
    const bool isU = e < t.nU;
    const int64_t q = isU ? e : e - t.nU;
    int l = 1;
    const int* off = isU ? n.offU : n.offV;
    while (l < n.L && q >= off[l + 1]) ++l;
    const int64_t w = q - off[l];
    const int rn = n.r[l], ro = o.r[l];
    const int row = (int)(w / rn), j = (int)(w - (int64_t)row * rn);
    const int k = t.src[n.offS[l] + j] - o.offS[l];   // old column in the layer
    if (isU)
      t.U[e] = o.U[o.offU[l] + (int64_t)row * ro + k];
    else
      t.V[q] = o.V[o.offV[l] + (int64_t)row * ro + k];
  }
  for (int64_t e = e0; e < t.nT; e += stride) {
    float v;
    if (e < t.theta_head) {
      v = t.theta[e];
    } else if (e < t.theta_head + (int64_t)t.R_new * t.HK1) {
      const int64_t q = e - t.theta_head;
      const int j = (int)(q / t.HK1), i = (int)(q - (int64_t)j * t.HK1);
      v = t.theta[t.theta_head + (int64_t)t.src[j] * t.HK1 + i];
    } else {
      const int j = (int)(e - t.theta_head - (int64_t)t.R_new * t.HK1);
      const int64_t old_c = t.theta_head + (int64_t)o.r_total * t.HK1;
      v = t.theta[old_c + t.src[j]];
    }
    t.theta_out[e] = v;
  }
}

int32_t make_khyper(const lrnr_hyper* f, KHyper* k) {
  if (!f) return fail(LRNR_EINVAL, "NULL hypernetwork");
  if (f->K < 1 || f->K > LRNR_MAX_LAYERS) return fail(LRNR_EINVAL, "hypernetwork K=%d", f->K);
  if (f->H[0] != 3) return fail(LRNR_EINVAL, "hypernetwork H[0]=%d, expected 3 (mu)", f->H[0]);
  if (!f->theta) return fail(LRNR_EINVAL, "NULL theta");
  *k = KHyper{};
  k->K = f->K;
  k->H[0] = 3;
  int64_t o = 0;
  for (int l = 1; l <= f->K; ++l) {
    const int h = f->H[l];
    if (h < 1 || h > kHyperMaxW) return fail(LRNR_EINVAL, "hypernetwork H[%d]=%d", l, h);
    k->H[l] = h;
    k->offW[l] = o;
    o += (int64_t)h * f->H[l - 1];
    k->offC[l] = o;
    o += h;
  }
  k->theta = f->theta;
  return LRNR_OK;
}

int64_t hyper_params(const KHyper& k) { return k.offC[k.K] + k.H[k.K]; }

}  // namespace
}  // namespace lrnr

using namespace lrnr;

extern "C" {

int32_t lrnr_hyper_forward(const lrnr_hyper* f, int32_t B, const float* mu, float* s,
                           void* stream) {
  KHyper k;
  int32_t rc = make_khyper(f, &k);
  if (rc != LRNR_OK) return rc;
  if (B < 0) return fail(LRNR_EINVAL, "B=%d", B);
  if (B == 0) return LRNR_OK;
  if (!mu || !s) return fail(LRNR_EINVAL, "NULL mu or s");
  hipLaunchKernelGGL(hyper_forward_kernel, dim3(B), dim3(kHyperThreads), 0,
                     static_cast<hipStream_t>(stream), k, mu, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "hypernetwork forward launch");
  return LRNR_OK;
}

size_t lrnr_hyper_workspace_size(const lrnr_hyper* f, int32_t B) {
  KHyper k;
  if (make_khyper(f, &k) != LRNR_OK || B < 1) return 0;
  return align256((size_t)B * (size_t)(hyper_params(k) + 1) * sizeof(float));
}

int32_t lrnr_hyper_backward(const lrnr_hyper* f, const lrnr_net* net, int32_t B, const float* mu,
                            const float* s_bar, float gamma, float lambda_sparse,
                            float* grad_theta, float* r_sparse, void* ws, size_t ws_bytes,
                            void* stream) {
  KHyper k;
  int32_t rc = make_khyper(f, &k);
  if (rc != LRNR_OK) return rc;
  KNet kn;
  int RP, Wp;
  rc = make_knet(net, &kn, &RP, &Wp);
  if (rc != LRNR_OK) return rc;
  if (k.H[k.K] != kn.r_total)
    return fail(LRNR_EINVAL, "hypernetwork output %d, net r_total %d", k.H[k.K], kn.r_total);
  if (B < 1) return fail(LRNR_EINVAL, "B=%d (at least one sample)", B);
  if (!mu || !s_bar || !grad_theta) return fail(LRNR_EINVAL, "NULL mu, s_bar or grad_theta");
  const size_t need = lrnr_hyper_workspace_size(f, B);
  if (!ws || ws_bytes < need)
    return fail(LRNR_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  k.L = kn.L;
  for (int l = 1; l <= kn.L; ++l) k.offS[l] = kn.offS[l];
  k.offS[kn.L + 1] = kn.r_total;
  const int64_t n_theta = hyper_params(k);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* w = static_cast<float*>(ws);
  hipLaunchKernelGGL(hyper_sample_grad_kernel, dim3(B), dim3(kHyperThreads), 0, st, k, B, mu,
                     s_bar, gamma, lambda_sparse, w, n_theta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "hypernetwork backward launch");
  const int64_t nb = (n_theta + 1 + kHyperThreads - 1) / kHyperThreads;
  hipLaunchKernelGGL(hyper_sum_kernel, dim3((unsigned)nb), dim3(kHyperThreads), 0, st, w, B,
                     n_theta, grad_theta, r_sparse);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "hypernetwork sum launch");
  return LRNR_OK;
}

int32_t lrnr_rows_mean(const float* x, int32_t B, int64_t n, float* out, void* stream) {
  if (B < 1 || n < 0) return fail(LRNR_EINVAL, "B=%d n=%lld", B, (long long)n);
  if (n == 0) return LRNR_OK;
  if (!x || !out) return fail(LRNR_EINVAL, "NULL x or out");
  const int64_t nb = (n + kHyperThreads - 1) / kHyperThreads;
  hipLaunchKernelGGL(rows_mean_kernel, dim3((unsigned)nb), dim3(kHyperThreads), 0,
                     static_cast<hipStream_t>(stream), x, B, n, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "rows mean launch");
  return LRNR_OK;
}

int32_t lrnr_orth_reg(const lrnr_net* net, float* value, float* grad_U, float* grad_V,
                      void* stream) {
  KNet k;
  int RP, Wp;
  int32_t rc = make_knet(net, &k, &RP, &Wp);
  if (rc != LRNR_OK) return rc;
  if (!value && !grad_U && !grad_V) return LRNR_OK;
  hipLaunchKernelGGL(orth_reg_kernel, dim3(1), dim3(kOrthThreads), 0,
                     static_cast<hipStream_t>(stream), k, value, grad_U, grad_V);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "orthogonality term launch");
  return LRNR_OK;
}

size_t lrnr_truncate_workspace_size(const lrnr_hyper* f, int32_t B) {
  KHyper k;
  if (make_khyper(f, &k) != LRNR_OK || B < 1) return 0;
  const int R = k.H[k.K];
  return align256((size_t)B * R * sizeof(float)) + align256((size_t)R * sizeof(int)) +
         align256((size_t)R * sizeof(int));
}

int32_t lrnr_truncate(const lrnr_net* net, const lrnr_hyper* f, int32_t B, const float* mu,
                      int32_t* r_out, int32_t* keep, float* U_out, float* V_out,
                      float* theta_out, void* ws, size_t ws_bytes, void* stream) {
  KHyper k;
  int32_t rc = make_khyper(f, &k);
  if (rc != LRNR_OK) return rc;
  KNet kn;
  int RP, Wp;
  rc = make_knet(net, &kn, &RP, &Wp);
  if (rc != LRNR_OK) return rc;
  const int R = kn.r_total;
  if (k.H[k.K] != R)
    return fail(LRNR_EINVAL, "hypernetwork output %d, net r_total %d", k.H[k.K], R);
  if (B < 1) return fail(LRNR_EINVAL, "B=%d (at least one sample)", B);
  if (!mu || !r_out || !U_out || !V_out || !theta_out)
    return fail(LRNR_EINVAL, "NULL mu, r_out, U_out, V_out or theta_out");
  const size_t need = lrnr_truncate_workspace_size(f, B);
  if (!ws || ws_bytes < need)
    return fail(LRNR_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  if ((uintptr_t)ws & 255) return fail(LRNR_EINVAL, "workspace not 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* s = reinterpret_cast<float*>(base);
  int* alive_d = reinterpret_cast<int*>(base + align256((size_t)B * R * sizeof(float)));
  int* src_d = reinterpret_cast<int*>(base + align256((size_t)B * R * sizeof(float)) +
                                      align256((size_t)R * sizeof(int)));
  hipLaunchKernelGGL(hyper_forward_kernel, dim3(B), dim3(kHyperThreads), 0, st, k, mu, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "hypernetwork forward launch");
  hipLaunchKernelGGL(output_alive_kernel, dim3((R + kHyperThreads - 1) / kHyperThreads),
                     dim3(kHyperThreads), 0, st, s, B, R, alive_d);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "alive launch");
  std::vector<int> alive(R);
  if ((e = hipMemcpyAsync(alive.data(), alive_d, R * sizeof(int), hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hip_fail(e, "alive copy");
  // kept set: the alive coefficients; a layer with none keeps its first
  std::vector<int> src;
  KNet nn = kn;
  int oU = 0, oV = 0, oS = 0;
  for (int l = 1; l <= kn.L; ++l) {
    int cnt = 0;
    for (int j = 0; j < kn.r[l]; ++j)
      if (alive[kn.offS[l] + j]) {
        src.push_back(kn.offS[l] + j);
        ++cnt;
      }
    if (cnt == 0) {
      src.push_back(kn.offS[l]);
      cnt = 1;
    }
    nn.r[l] = cnt;
    nn.offU[l] = oU;
    nn.offV[l] = oV;
    nn.offS[l] = oS;
    oU += kn.M[l] * cnt;
    oV += kn.M[l - 1] * cnt;
    oS += cnt;
  }
  nn.r_total = oS;
  nn.U = U_out;
  nn.V = V_out;
  r_out[0] = 0;
  for (int l = 1; l <= kn.L; ++l) r_out[l] = nn.r[l];
  if (keep) {
    for (int m = 0; m < R; ++m) keep[m] = 0;
    for (int j : src) keep[j] = 1;
  }
  if ((e = upload_async(src_d, src.data(), src.size() * sizeof(int), st)) != hipSuccess)
    return hip_fail(e, "index upload");
  KTrunc t{};
  t.old_net = kn;
  t.new_net = nn;
  t.src = src_d;
  t.U = U_out;
  t.V = V_out;
  t.theta = f->theta;
  t.theta_out = theta_out;
  t.theta_head = k.offW[k.K];
  t.HK1 = k.H[k.K - 1];
  t.R_new = oS;
  t.nU = oU;
  t.nV = oV;
  t.nT = t.theta_head + (int64_t)oS * (t.HK1 + 1);
  const int64_t work = std::max<int64_t>(t.nU + t.nV, t.nT);
  const int blocks = (int)std::min<int64_t>((work + kHyperThreads - 1) / kHyperThreads, 4096);
  hipLaunchKernelGGL(truncate_gather_kernel, dim3(blocks), dim3(kHyperThreads), 0, st, t);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "truncation gather launch");
  return LRNR_OK;
}

}  // extern "C"
