// Cross-workgroup reduction of the fused kernel's per-workgroup records into
// the loss terms, dL/ds and dL/db, plus the fused Adam update.
//
// Both reduction stages add in a fixed order (FP64), so results are bitwise
// reproducible and do not depend on how many other instances share a launch.
#include "lrnr_internal.h"

namespace lrnr {

// Stage 1: red1[i][c][e] = sum of records [c*kRedChunk, (c+1)*kRedChunk) of
// instance i, element e.
__global__ void reduce_stage1(const float* __restrict__ partials, double* __restrict__ red1,
                              int G_inst, int P, int E, int nchunk) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, inst = blockIdx.z;
  if (e >= E) return;
  const int r0 = c * kRedChunk, r1 = min(G_inst, r0 + kRedChunk);
  const float* base = partials + ((int64_t)inst * G_inst) * P + e;
  double acc = 0.0;
  for (int r = r0; r < r1; ++r) acc += (double)base[(int64_t)r * P];
  red1[((int64_t)inst * nchunk + c) * P + e] = acc;
}

__device__ __forceinline__ double column_sum(const double* __restrict__ red1, int inst,
                                             int nchunk, int P, int e) {
  const double* base = red1 + (int64_t)inst * nchunk * P + e;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += base[(int64_t)c * P];
  return acc;
}

__device__ __forceinline__ float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// Stage 2: one thread per record element and instance.
__global__ void reduce_stage2(KReduce kr) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  const int P = kr.P;
  if (e >= kr.E) return;
  const float* s = kr.s + inst * kr.s_stride;
  const float* sref = kr.s_ref ? kr.s_ref + inst * kr.s_stride : nullptr;
  const bool loc = kr.lambda_loc != 0.f && sref != nullptr;
  if (e == 0 && kr.loss) {
    const double ti = kr.n_r ? (double)kr.w_r / kr.n_r * column_sum(kr.red1, inst, kr.nchunk, P, 0) : 0.0;
    const double t0 = kr.n_0 ? (double)kr.w_0 / kr.n_0 * column_sum(kr.red1, inst, kr.nchunk, P, 1) : 0.0;
    const double tb = kr.n_b ? (double)kr.w_b / kr.n_b * column_sum(kr.red1, inst, kr.nchunk, P, 2) : 0.0;
    double tl = 0.0;
    if (loc)
      for (int k = 0; k < kr.r_total; ++k) tl += fabs((double)s[k] - (double)sref[k]);
    float* out = kr.loss + 4 * inst;
    out[0] = (float)(ti + t0 + tb + (double)kr.lambda_loc * tl);
    out[1] = (float)ti;
    out[2] = (float)t0;
    out[3] = (float)tb;
  }
  if (e >= 4 && e < 4 + kr.r_total && kr.grad_s) {
    const int k = e - 4;
    double g = column_sum(kr.red1, inst, kr.nchunk, P, e);
    if (loc) g += (double)kr.lambda_loc * sgn(s[k] - sref[k]);
    kr.grad_s[(int64_t)inst * kr.r_total + k] = (float)g;
  }
  if (e >= 4 + kr.r_total && e < 4 + kr.r_total + kr.b_total && kr.grad_b && inst == 0) {
    kr.grad_b[e - 4 - kr.r_total] = (float)column_sum(kr.red1, inst, kr.nchunk, P, e);
  }
}

hipError_t launch_reduce(const KReduce& kr, hipStream_t stream) {
  const int bx = 256;
  const int gx = (kr.E + bx - 1) / bx;
  if (kr.nchunk > 0) {
    hipLaunchKernelGGL(reduce_stage1, dim3(gx, kr.nchunk, kr.B), dim3(bx), 0, stream,
                       kr.partials, kr.red1, kr.G_inst, kr.P, kr.E, kr.nchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(reduce_stage2, dim3(gx, kr.B), dim3(bx), 0, stream, kr);
  return hipGetLastError();
}

// Adam (Kingma & Ba), bias-corrected, step counted from 1.
__global__ void adam_kernel(float* __restrict__ s, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float beta1,
                            float beta2, float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  s[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t launch_adam(float* s, float* m, float* v, const float* g, int64_t n, int step,
                       float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const float bc1 = (float)(1.0 - pow((double)beta1, step));
  const float bc2 = (float)(1.0 - pow((double)beta2, step));
  const int bx = 256;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + bx - 1) / bx)), dim3(bx), 0, stream, s, m,
                     v, g, n, lr, beta1, beta2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace lrnr
