// Cross-workgroup reduction of the fused kernel's per-workgroup records into
// the loss terms, dL/ds and dL/db, plus the fused Adam update.
//
// Both reduction stages add in a fixed order (FP64), so results are bitwise
// reproducible and do not depend on how many other instances share a launch.
#include <algorithm>

#include "lrnr_internal.h"
#include "lrnr_task_status.h"

namespace lrnr {

// Sum of n values base[0], base[stride], ... in FP64, added strictly in index
// order; the loads are issued eight at a time, so the order (and the result)
// is that of the plain loop while the memory latency is paid n/8 times.
template <typename T>
__device__ __forceinline__ double ordered_sum(const T* __restrict__ base, int64_t stride, int n) {
  double acc = 0.0;
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = base[(int64_t)(i + j) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += (double)v[j];
  }
  for (; i < n; ++i) acc += (double)base[(int64_t)i * stride];
  return acc;
}

// Stage 1: red1[i][c][e] = sum of records [c*kRedChunk, (c+1)*kRedChunk) of
// instance i, element e.
__global__ void reduce_stage1(const float* __restrict__ partials, double* __restrict__ red1,
                              int G_inst, int P, int E, int nchunk) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, inst = blockIdx.z;
  if (e >= E) return;
  const int r0 = c * kRedChunk, r1 = min(G_inst, r0 + kRedChunk);
  const float* base = partials + ((int64_t)inst * G_inst + r0) * P + e;
  red1[((int64_t)inst * nchunk + c) * P + e] = ordered_sum(base, P, r1 - r0);
}

__device__ __forceinline__ double column_sum(const double* __restrict__ red1, int inst,
                                             int nchunk, int P, int e) {
  return ordered_sum(red1 + (int64_t)inst * nchunk * P + e, P, nchunk);
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

// Both stages in one launch when an instance has at most kRedFusedChunks
// chunks (2048 records; the working-size launch has 1408 in 44 chunks):
// thread (ex, c) of a block (ex fastest, so that a wave reads 16 consecutive
// elements of four chunk rows) forms the stage-1 sum of chunk c for element
// blockIdx.x * kRedFusedElems + ex, and thread (ex, 0) then adds the chunk
// sums in chunk order.  The additions and their order are those of
// reduce_stage1 + reduce_stage2, so the results are the same bits.
constexpr int kRedFusedElems = 16;
constexpr int kRedFusedChunks = 64;

__global__ __launch_bounds__(kRedFusedElems* kRedFusedChunks) void reduce_fused(KReduce kr) {
  __shared__ double part[kRedFusedChunks][kRedFusedElems];
  __shared__ double col[kRedFusedElems];
  const int ex = threadIdx.x % kRedFusedElems, c = threadIdx.x / kRedFusedElems;
  const int e = blockIdx.x * kRedFusedElems + ex, inst = blockIdx.y;
  const int P = kr.P;
  if (e < kr.E && c < kr.nchunk) {
    const int r0 = c * kRedChunk, r1 = min(kr.G_inst, r0 + kRedChunk);
    const float* base = kr.partials + ((int64_t)inst * kr.G_inst + r0) * P + e;
    part[c][ex] = ordered_sum(base, P, r1 - r0);
  }
  __syncthreads();
  if (c == 0) {
    double acc = 0.0;
    for (int k = 0; k < kr.nchunk; ++k) acc += part[k][ex];
    col[ex] = acc;
  }
  __syncthreads();
  if (c != 0 || e >= kr.E) return;
  const float* s = kr.s + inst * kr.s_stride;
  const float* sref = kr.s_ref ? kr.s_ref + inst * kr.s_stride : nullptr;
  const bool loc = kr.lambda_loc != 0.f && sref != nullptr;
  if (e == 0 && kr.loss) {
    // elements 0, 1, 2 of the record are in this block (kRedFusedElems >= 3)
    const double ti = kr.n_r ? (double)kr.w_r / kr.n_r * col[0] : 0.0;
    const double t0 = kr.n_0 ? (double)kr.w_0 / kr.n_0 * col[1] : 0.0;
    const double tb = kr.n_b ? (double)kr.w_b / kr.n_b * col[2] : 0.0;
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
    double g = col[ex];
    if (loc) g += (double)kr.lambda_loc * sgn(s[k] - sref[k]);
    kr.grad_s[(int64_t)inst * kr.r_total + k] = (float)g;
  }
  if (e >= 4 + kr.r_total && e < 4 + kr.r_total + kr.b_total && kr.grad_b && inst == 0)
    kr.grad_b[e - 4 - kr.r_total] = (float)col[ex];
}

hipError_t launch_reduce(const KReduce& kr, hipStream_t stream) {
  const int bx = 256;
  const int gx = (kr.E + bx - 1) / bx;
  if (kr.nchunk > 0 && kr.nchunk <= kRedFusedChunks) {
    // threads for the chunks in use, rounded up to whole waves
    const int gf = (kr.E + kRedFusedElems - 1) / kRedFusedElems;
    const int nt = (kRedFusedElems * kr.nchunk + 63) & ~63;
    hipLaunchKernelGGL(reduce_fused, dim3(gf, kr.B), dim3(nt), 0, stream, kr);
    return hipGetLastError();
  }
  if (kr.nchunk > 0) {
    hipLaunchKernelGGL(reduce_stage1, dim3(gx, kr.nchunk, kr.B), dim3(bx), 0, stream,
                       kr.partials, kr.red1, kr.G_inst, kr.P, kr.E, kr.nchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(reduce_stage2, dim3(gx, kr.B), dim3(bx), 0, stream, kr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Task tables: one workgroup per task (grid-stride).  Each record element is
// summed in the order of the two-stage reduction above (chunks of kRedChunk
// records, then the chunk sums in order), so a task's results depend only on
// its own records and match the single-instance path.  When the chunk sums
// of a task fit kTablePartials doubles, every (element, chunk) pair has its
// own thread and one thread per element then adds the chunk sums in order
// (the same additions, a few rounds of loads instead of one per chunk);
// otherwise one thread runs all chunks of an element.
// ---------------------------------------------------------------------------
constexpr int kTableReduceThreads = 256;
constexpr int kTablePartials = 2048;

__global__ __launch_bounds__(kTableReduceThreads) void table_reduce_kernel(KTableGrid tg,
                                                                           int reduce_b,
                                                                           KAdam adam) {
  __shared__ double sums[4];
  __shared__ float gsh[LRNR_MAX_LAYERS * LRNR_MAX_RANK];
  __shared__ double part[kTablePartials];
  const KTableHdr* hdr = reinterpret_cast<const KTableHdr*>(tg.table);
  const int* start = reinterpret_cast<const int*>(tg.table + sizeof(KTableHdr));
  const KTask* tasks = reinterpret_cast<const KTask*>(tg.table + tg.off_tasks);
  const int n_tasks = hdr->n_tasks;
  const int tid = threadIdx.x;
  for (int t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const KTask& T = tasks[t];
    const bool adam_on = T.m != nullptr;
    int step = 0;
    if (adam_on) {
      step = *T.step;
      if (T.steps_max > 0 && step >= T.steps_max) continue;  // finished: nothing ran
    }
    const int G = start[t + 1] - start[t];
    const int r_total = T.net.r_total, b_total = T.net.b_total;
    // loss-only records carry their first four elements only
    const bool want_b = reduce_b && T.grad_b != nullptr;
    const bool want_s = T.grad_s != nullptr || adam_on || want_b;
    const int E = 4 + (want_s ? r_total : 0) + (want_b ? b_total : 0);
    const int P = T.P;
    const float* rec = tg.partials + T.rec0;
    const float* s = T.inst.s;
    const float* sref = T.s_ref;
    const bool loc = T.lambda_loc != 0.f && sref != nullptr;
    const int nchunk = (G + kRedChunk - 1) / kRedChunk;
    const bool split = nchunk * E <= kTablePartials;
    if (split) {
      for (int q = tid; q < nchunk * E; q += kTableReduceThreads) {
        const int c = q / E, e = q - c * E;
        const int r0 = c * kRedChunk, r1 = min(G, r0 + kRedChunk);
        part[q] = ordered_sum(rec + (int64_t)r0 * P + e, P, r1 - r0);
      }
      __syncthreads();
    }
    int nonfinite = 0;
    for (int e = tid; e < E; e += kTableReduceThreads) {
      double acc = 0.0;
      for (int c = 0; c < nchunk; ++c) {
        if (split) {
          acc += part[c * E + e];
        } else {
          const int r0 = c * kRedChunk, r1 = min(G, r0 + kRedChunk);
          acc += ordered_sum(rec + (int64_t)r0 * P + e, P, r1 - r0);
        }
      }
      if (e < 4) {
        sums[e] = acc;
        nonfinite |= !isfinite(acc);
      } else if (e < 4 + r_total) {
        const int k = e - 4;
        if (loc) acc += (double)T.lambda_loc * sgn(s[k] - sref[k]);
        const float g = (float)acc;
        gsh[k] = g;
        nonfinite |= !isfinite(g);
        if (T.grad_s) T.grad_s[k] = g;
      } else {
        T.grad_b[e - 4 - r_total] = (float)acc;
      }
    }
    const bool failed = __syncthreads_or(nonfinite) != 0;
    if (tid == 0 && T.loss) {
      const int64_t n_r = T.inst.n_r, n_0 = T.inst.n_0, n_b = T.inst.n_b;
      const double ti = n_r ? (double)T.w_r / n_r * sums[0] : 0.0;
      const double t0 = n_0 ? (double)T.w_0 / n_0 * sums[1] : 0.0;
      const double tb = n_b ? (double)T.w_b / n_b * sums[2] : 0.0;
      double tl = 0.0;
      if (loc)
        for (int k = 0; k < r_total; ++k) tl += fabs((double)s[k] - (double)sref[k]);
      T.loss[0] = (float)(ti + t0 + tb + (double)T.lambda_loc * tl);
      T.loss[1] = (float)ti;
      T.loss[2] = (float)t0;
      T.loss[3] = (float)tb;
    }
    if (adam_on && failed) {
      // a non-finite loss or gradient: s, m and v stay as they are and the
      // task is finished (its counter now exceeds any step limit)
      __syncthreads();  // every thread has read *T.step
      if (tid == 0) *T.step = step | kTaskFailed;
    } else if (adam_on) {
      // Adam (Kingma & Ba), bias-corrected, step counted from 1
      const int stp = step + 1;
      const float bc1 = (float)(1.0 - pow((double)adam.beta1, (double)stp));
      const float bc2 = (float)(1.0 - pow((double)adam.beta2, (double)stp));
      for (int k = tid; k < r_total; k += kTableReduceThreads) {
        const float gi = gsh[k];
        const float mi = adam.beta1 * T.m[k] + (1.f - adam.beta1) * gi;
        const float vi = adam.beta2 * T.v[k] + (1.f - adam.beta2) * gi * gi;
        T.m[k] = mi;
        T.v[k] = vi;
        T.s_upd[k] -= adam.lr * (mi / bc1) / (sqrtf(vi / bc2) + adam.eps);
      }
      __syncthreads();  // every thread has read *T.step
      if (tid == 0) *T.step = stp;
    }
    __syncthreads();
  }
}

hipError_t launch_table_reduce(const KTableGrid& tg, int cap, int reduce_b, KAdam adam,
                               hipStream_t stream) {
  const int grid = std::max(1, std::min(cap, 1024));
  hipLaunchKernelGGL(table_reduce_kernel, dim3(grid), dim3(kTableReduceThreads), 0, stream, tg,
                     reduce_b, adam);
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
