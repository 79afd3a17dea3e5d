// Reduced states of the forward pass: y^{l+1} = V^{(l+1)T} z^l for every
// hidden layer (values only).  For a FastLRNR net (an LRNR whose hidden
// widths are r_hat_l, Section 2.2) these are the reduced states z_hat^l of
// eq. 2.8, and for the LRNR they are what z_hat^l approximates, so the same
// call measures the FastLRNR's state error against r_hat.  A diagnostic, not
// the hot path: one thread per point, FP32, weights through the caches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lrnr_internal.h"

namespace lrnr {
namespace {

constexpr int kStateThreads = 256;

__global__ void __launch_bounds__(kStateThreads) reduced_states_kernel(KNet k, const float* s,
                                                                       const float* xt, int64_t n,
                                                                       float* out) {
  const int64_t p = (int64_t)blockIdx.x * kStateThreads + threadIdx.x;
  if (p >= n) return;
  const float x = xt[2 * p], t = xt[2 * p + 1];
  float y[LRNR_MAX_RANK], yn[LRNR_MAX_RANK];
  const int r1 = k.r[1];
  const float* V1 = k.V + k.offV[1];
#pragma unroll
  for (int j = 0; j < LRNR_MAX_RANK; ++j) y[j] = (j < r1) ? V1[j] * x + V1[r1 + j] * t : 0.f;
  int64_t row = 0;   // first output row of the current layer
  for (int l = 1; l <= k.L - 1; ++l) {
    const int M = k.M[l], rl = k.r[l], ro = k.r[l + 1];
    const float* U = k.U + k.offU[l];
    const float* V = k.V + k.offV[l + 1];
    const float* b = k.b + k.offB[l];
    const float* sl = s + k.offS[l];
#pragma unroll
    for (int j = 0; j < LRNR_MAX_RANK; ++j) {
      if (j < rl) y[j] *= sl[j];
      yn[j] = 0.f;
    }
    for (int i = 0; i < M; ++i) {
      float a = b[i];
#pragma unroll
      for (int j = 0; j < LRNR_MAX_RANK; ++j)
        if (j < rl) a = fmaf(U[i * rl + j], y[j], a);
      const float z = sinf(a);
#pragma unroll
      for (int j = 0; j < LRNR_MAX_RANK; ++j)
        if (j < ro) yn[j] = fmaf(V[i * ro + j], z, yn[j]);
    }
#pragma unroll
    for (int j = 0; j < LRNR_MAX_RANK; ++j) {
      if (j < ro) out[(row + j) * n + p] = yn[j];
      y[j] = yn[j];
    }
    row += ro;
  }
}

}  // namespace
}  // namespace lrnr

using namespace lrnr;

extern "C" {

int32_t lrnr_reduced_states(const lrnr_net* net, const float* s, const float* xt, int64_t n,
                            float* y, void* stream) {
  KNet k;
  int RP, Wp;
  int32_t rc = make_knet(net, &k, &RP, &Wp);
  if (rc != LRNR_OK) return rc;
  if (n < 0) return fail(LRNR_EINVAL, "n=%lld", (long long)n);
  if (n == 0) return LRNR_OK;
  if (!s || !xt || !y) return fail(LRNR_EINVAL, "NULL s, xt or y");
  const int64_t blocks = (n + kStateThreads - 1) / kStateThreads;
  hipLaunchKernelGGL(reduced_states_kernel, dim3((unsigned)blocks), dim3(kStateThreads), 0,
                     static_cast<hipStream_t>(stream), k, s, xt, n, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "reduced states launch");
  return LRNR_OK;
}

}  // extern "C"
