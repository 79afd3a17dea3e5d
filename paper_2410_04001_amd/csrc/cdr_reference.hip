// Reference solution of the convection-diffusion-reaction problem of
// Section 4, eq. (4.1), and the L1 relative error of a prediction against it
// (the test-accuracy measure of the Section 4 comparison of FastLRNR and LRNR
// against wall time).
//
// Solver: Strang splitting u_{n+1} = R(dt/2) L(dt) R(dt/2) u_n with both
// sub-flows exact: L (convection-diffusion) diagonal in Fourier space on the
// uniform periodic grid, R the logistic flow of u' = mu_3 u (1 - u).  FP64
// throughout.
//
// Device layout: one workgroup per parameter instance, the grid of n_x values
// in LDS as complex doubles.  Grids of 4^m points take the radix-4 kernel
// further down (half the passes); the others this one.  The transform pair is
// a radix-2 decimation-in-
// frequency forward FFT (natural order in, bit-reversed out) followed by a
// decimation-in-time inverse FFT (bit-reversed in, natural out), so no
// permutation pass is needed: the Fourier propagator is stored in bit-
// reversed order.  Work that touches the same pair of grid points in
// consecutive passes stays in registers: the first reaction half-step runs
// inside the first forward stage, the propagator multiply between the last
// forward and the first inverse stage, and the second reaction half-step
// (and the output store) inside the last inverse stage.  A step costs
// 2 log2(n_x) - 2 workgroup barriers; thread t always owns butterflies
// b = t + T q, so the pairs (b, b + n_x/2) of the outer stages and (2b, 2b+1)
// of the inner ones are its own.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>

#include "lrnr_internal.h"

namespace lrnr {
namespace {

constexpr double kUMax = 1.0e6;   // |u| above this ends an instance (blow-up)
constexpr int kMaxNx = 1024;
constexpr int kL1Threads = 1024;

struct CdrArgs {
  const double* mu;   // [B][3]
  int n_x, log2n, n_t, every, n_out;
  double dt;
  double* u;          // [B][n_out][n_x]
  int32_t* status;    // [B]
};

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmul_conj(double2 a, double2 w) {   // a * conj(w)
  return make_double2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Logistic flow over one half-step: u e / (1 + u (e - 1)); bad when the flow
// leaves R within the half-step (denominator <= 0, NaN included).
__device__ inline double react(double u, double e, double em1, bool& bad) {
  const double d = 1.0 + u * em1;
  bad |= !(d > 0.0);
  return u * e / d;
}

// Q butterflies per thread per stage: Q = n_x / (2 T).
template <int Q>
__global__ void __launch_bounds__(256) cdr_strang_kernel(CdrArgs a) {
  extern __shared__ double2 lds[];
  const int N = a.n_x, H = N >> 1, T = blockDim.x, tid = threadIdx.x;
  double2* X = lds;            // [N] state / spectrum
  double2* tw = lds + N;       // [N/2] exp(-2 pi i m / N)
  double2* Pb = lds + N + H;   // [N] propagator / N at bit-reversed positions

  const int inst = blockIdx.x;
  const double beta = a.mu[3 * inst], nu = a.mu[3 * inst + 1], rho = a.mu[3 * inst + 2];
  const double e = exp(rho * 0.5 * a.dt), em1 = expm1(rho * 0.5 * a.dt);
  double* out = a.u + (int64_t)inst * a.n_out * N;

  for (int m = tid; m < H; m += T) {
    double sv, cv;
    sincos((2.0 * M_PI) * m / N, &sv, &cv);
    tw[m] = make_double2(cv, -sv);
  }
  for (int i = tid; i < N; i += T) {
    const int m = (int)(__brev((unsigned)i) >> (32 - a.log2n));   // spectral index at i
    const double k = (m < H) ? (double)m : (double)(m - N);
    double sv, cv;
    sincos(beta * k * a.dt, &sv, &cv);
    const double g = exp(-nu * k * k * a.dt) / N;
    Pb[i] = make_double2(g * cv, -g * sv);
  }

  double lo[Q], hi[Q];   // u at b and b + N/2 for this thread's butterflies
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = tid + T * q;
    lo[q] = sin((2.0 * M_PI) * b / N);
    hi[q] = sin((2.0 * M_PI) * (b + H) / N);
    out[b] = lo[q];
    out[b + H] = hi[q];
  }
  __syncthreads();

  for (int n = 1; n <= a.n_t; ++n) {
    bool bad = false;
    // first reaction half-step fused into the forward stage of span N
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = tid + T * q;
      const double u0 = react(lo[q], e, em1, bad), u1 = react(hi[q], e, em1, bad);
      X[b] = make_double2(u0 + u1, 0.0);
      const double dlt = u0 - u1;
      X[b + H] = make_double2(dlt * tw[b].x, dlt * tw[b].y);
    }
    __syncthreads();
    // forward stages of span N/2 .. 4
    for (int s = a.log2n - 1; s >= 2; --s) {
      const int len = 1 << s, h = len >> 1, tws = a.log2n - s;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int b = tid + T * q;
        const int p = b & (h - 1), i0 = ((b >> (s - 1)) << s) + p, i1 = i0 + h;
        const double2 x0 = X[i0], x1 = X[i1];
        X[i0] = cadd(x0, x1);
        X[i1] = cmul(csub(x0, x1), tw[p << tws]);
      }
      __syncthreads();
    }
    // span 2 forward, propagator, span 2 inverse (twiddle 1 on both)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i0 = 2 * (tid + T * q), i1 = i0 + 1;
      const double2 x0 = X[i0], x1 = X[i1];
      const double2 y0 = cmul(cadd(x0, x1), Pb[i0]), y1 = cmul(csub(x0, x1), Pb[i1]);
      X[i0] = cadd(y0, y1);
      X[i1] = csub(y0, y1);
    }
    __syncthreads();
    // inverse stages of span 4 .. N/2
    for (int s = 2; s < a.log2n; ++s) {
      const int len = 1 << s, h = len >> 1, tws = a.log2n - s;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int b = tid + T * q;
        const int p = b & (h - 1), i0 = ((b >> (s - 1)) << s) + p, i1 = i0 + h;
        const double2 x0 = X[i0], t = cmul_conj(X[i1], tw[p << tws]);
        X[i0] = cadd(x0, t);
        X[i1] = csub(x0, t);
      }
      __syncthreads();
    }
    // inverse stage of span N (real parts only) and the second half-step
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = tid + T * q;
      const double2 x0 = X[b], t = cmul_conj(X[b + H], tw[b]);
      lo[q] = react(x0.x + t.x, e, em1, bad);
      hi[q] = react(x0.x - t.x, e, em1, bad);
      bad |= !(fabs(lo[q]) <= kUMax) || !(fabs(hi[q]) <= kUMax);
    }
    // every thread has read X before any thread rewrites it next step
    if (__syncthreads_or(bad)) {
      if (tid == 0) a.status[inst] = n;
      for (int k = (n + a.every - 1) / a.every; k < a.n_out; ++k)
        for (int j = tid; j < N; j += T) out[(int64_t)k * N + j] = __longlong_as_double(0x7ff8000000000000LL);
      return;
    }
    if (n % a.every == 0) {
      double* o = out + (int64_t)(n / a.every) * N;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int b = tid + T * q;
        o[b] = lo[q];
        o[b + H] = hi[q];
      }
    }
  }
  if (tid == 0) a.status[inst] = 0;
}

__device__ inline double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }   // a * (-i)
__device__ inline double2 mul_pi(double2 a) { return make_double2(-a.y, a.x); }   // a * (+i)

// Radix-4 variant for n_x = 4^m (m >= 2): decimation in frequency with
// radix-4 butterflies leaves the spectrum in base-4 digit-reversed order, the
// propagator is stored in that order, and radix-4 decimation in time returns
// to natural order.  One butterfly (four grid points) per thread and stage,
// n_x/4 threads (one wave at n_x = 256): half the passes of the radix-2
// kernel, 2m - 1 barriers per step.  The same fusions: the first reaction
// half-step inside the outermost forward stage, the propagator between the
// span-4 stages, the second half-step and the output inside the outermost
// inverse stage (thread t owns points t + r n_x/4 there and 4t..4t+3 in the
// span-4 stages).
__global__ void __launch_bounds__(256) cdr_strang4_kernel(CdrArgs a) {
  extern __shared__ double2 lds[];
  const int N = a.n_x, Qn = N >> 2, m = a.log2n >> 1, tid = threadIdx.x;
  double2* X = lds;            // [N]
  double2* tw = lds + N;       // [N] exp(-2 pi i k / N)
  double2* Pd = lds + 2 * N;   // [N] propagator / N at digit-reversed positions

  const int inst = blockIdx.x;
  const double beta = a.mu[3 * inst], nu = a.mu[3 * inst + 1], rho = a.mu[3 * inst + 2];
  const double e = exp(rho * 0.5 * a.dt), em1 = expm1(rho * 0.5 * a.dt);
  double* out = a.u + (int64_t)inst * a.n_out * N;
  const int T = blockDim.x;

  for (int k = tid; k < N; k += T) {
    double sv, cv;
    sincos((2.0 * M_PI) * k / N, &sv, &cv);
    tw[k] = make_double2(cv, -sv);
    int r = 0, i = k;
    for (int d = 0; d < m; ++d) {
      r = (r << 2) | (i & 3);
      i >>= 2;
    }
    const double kk = (r < (N >> 1)) ? (double)r : (double)(r - N);   // wavenumber at k
    sincos(beta * kk * a.dt, &sv, &cv);
    const double g = exp(-nu * kk * kk * a.dt) / N;
    Pd[k] = make_double2(g * cv, -g * sv);
  }

  double u[4];   // u at tid + r N/4
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    u[r] = sin((2.0 * M_PI) * (tid + r * Qn) / N);
    out[tid + r * Qn] = u[r];
  }
  __syncthreads();

  for (int n = 1; n <= a.n_t; ++n) {
    bool bad = false;
    {   // reaction half-step, forward stage of span N (p = tid, twiddle step 1)
      double v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = react(u[r], e, em1, bad);
      const double t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3], t3 = v[1] - v[3];
      // (t1 + t3*(-i)), (t1 - t3*(-i)) with t1, t3 real
      X[tid] = make_double2(t0 + t2, 0.0);
      X[tid + Qn] = cmul(make_double2(t1, -t3), tw[tid]);
      X[tid + 2 * Qn] = make_double2((t0 - t2) * tw[2 * tid].x, (t0 - t2) * tw[2 * tid].y);
      X[tid + 3 * Qn] = cmul(make_double2(t1, t3), tw[3 * tid]);
    }
    __syncthreads();
    for (int s = m - 1; s >= 2; --s) {   // forward stages of span 4^s
      const int q = 1 << (2 * (s - 1)), sh = 2 * (m - s);
      const int p = tid & (q - 1), i0 = ((tid >> (2 * (s - 1))) << (2 * s)) + p;
      const double2 x0 = X[i0], x1 = X[i0 + q], x2 = X[i0 + 2 * q], x3 = X[i0 + 3 * q];
      const double2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3),
                    t3 = mul_mi(csub(x1, x3));
      X[i0] = cadd(t0, t2);
      X[i0 + q] = cmul(cadd(t1, t3), tw[p << sh]);
      X[i0 + 2 * q] = cmul(csub(t0, t2), tw[(2 * p) << sh]);
      X[i0 + 3 * q] = cmul(csub(t1, t3), tw[(3 * p) << sh]);
      __syncthreads();
    }
    {   // span 4 forward, propagator, span 4 inverse (all twiddles 1)
      const int i0 = 4 * tid;
      const double2 x0 = X[i0], x1 = X[i0 + 1], x2 = X[i0 + 2], x3 = X[i0 + 3];
      const double2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3),
                    t3 = mul_mi(csub(x1, x3));
      const double2 a0 = cmul(cadd(t0, t2), Pd[i0]), a1 = cmul(cadd(t1, t3), Pd[i0 + 1]),
                    a2 = cmul(csub(t0, t2), Pd[i0 + 2]), a3 = cmul(csub(t1, t3), Pd[i0 + 3]);
      const double2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3),
                    b3 = mul_pi(csub(a1, a3));
      X[i0] = cadd(b0, b2);
      X[i0 + 1] = cadd(b1, b3);
      X[i0 + 2] = csub(b0, b2);
      X[i0 + 3] = csub(b1, b3);
    }
    __syncthreads();
    for (int s = 2; s < m; ++s) {   // inverse stages of span 4^s
      const int q = 1 << (2 * (s - 1)), sh = 2 * (m - s);
      const int p = tid & (q - 1), i0 = ((tid >> (2 * (s - 1))) << (2 * s)) + p;
      const double2 a0 = X[i0], a1 = cmul_conj(X[i0 + q], tw[p << sh]),
                    a2 = cmul_conj(X[i0 + 2 * q], tw[(2 * p) << sh]),
                    a3 = cmul_conj(X[i0 + 3 * q], tw[(3 * p) << sh]);
      const double2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3),
                    b3 = mul_pi(csub(a1, a3));
      X[i0] = cadd(b0, b2);
      X[i0 + q] = cadd(b1, b3);
      X[i0 + 2 * q] = csub(b0, b2);
      X[i0 + 3 * q] = csub(b1, b3);
      __syncthreads();
    }
    {   // inverse stage of span N (real parts only), second half-step
      const double2 a0 = X[tid], a1 = cmul_conj(X[tid + Qn], tw[tid]),
                    a2 = cmul_conj(X[tid + 2 * Qn], tw[2 * tid]),
                    a3 = cmul_conj(X[tid + 3 * Qn], tw[3 * tid]);
      const double2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3),
                    b3 = mul_pi(csub(a1, a3));
      u[0] = react(b0.x + b2.x, e, em1, bad);
      u[1] = react(b1.x + b3.x, e, em1, bad);
      u[2] = react(b0.x - b2.x, e, em1, bad);
      u[3] = react(b1.x - b3.x, e, em1, bad);
#pragma unroll
      for (int r = 0; r < 4; ++r) bad |= !(fabs(u[r]) <= kUMax);
    }
    if (__syncthreads_or(bad)) {
      if (tid == 0) a.status[inst] = n;
      for (int k = (n + a.every - 1) / a.every; k < a.n_out; ++k)
        for (int j = tid; j < N; j += T) out[(int64_t)k * N + j] = __longlong_as_double(0x7ff8000000000000LL);
      return;
    }
    if (n % a.every == 0) {
      double* o = out + (int64_t)(n / a.every) * N;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[tid + r * Qn] = u[r];
    }
  }
  if (tid == 0) a.status[inst] = 0;
}

// sum |pred - ref| and sum |ref| in FP64, one workgroup, fixed order: thread t
// takes i = t, t + 1024, ... ascending, then a fixed tree over the threads.
__global__ void __launch_bounds__(kL1Threads) l1_error_kernel(const float* pred, const double* ref,
                                                            int64_t n, double* out) {
  __shared__ double sd[kL1Threads], sr[kL1Threads];
  const int t = threadIdx.x;
  double d = 0.0, r = 0.0;
  for (int64_t i = t; i < n; i += kL1Threads) {
    const double v = ref[i];
    d += fabs((double)pred[i] - v);
    r += fabs(v);
  }
  sd[t] = d;
  sr[t] = r;
  __syncthreads();
  for (int w = kL1Threads / 2; w > 0; w >>= 1) {
    if (t < w) {
      sd[t] += sd[t + w];
      sr[t] += sr[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = sd[0];
    out[1] = sr[0];
  }
}

}  // namespace
}  // namespace lrnr

using namespace lrnr;

extern "C" {

int32_t lrnr_cdr_reference(const double* mu, int32_t B, int32_t n_x, int32_t n_t, int32_t n_out,
                            double t_end, double* u, int32_t* status, void* stream) {
  if (B < 0) return fail(LRNR_EINVAL, "B=%d", B);
  if (n_x < 8 || n_x > kMaxNx || (n_x & (n_x - 1)))
    return fail(LRNR_EINVAL, "n_x=%d (power of two in [8, %d])", n_x, kMaxNx);
  if (n_t < 1 || n_out < 2 || n_t % (n_out - 1))
    return fail(LRNR_EINVAL, "n_t=%d n_out=%d (n_out - 1 must divide n_t)", n_t, n_out);
  if (!(t_end > 0.0) || !std::isfinite(t_end)) return fail(LRNR_EINVAL, "t_end=%g", t_end);
  if (B == 0) return LRNR_OK;
  if (!mu || !u || !status) return fail(LRNR_EINVAL, "NULL mu, u or status");
  CdrArgs a;
  a.mu = mu;
  a.n_x = n_x;
  a.log2n = 0;
  while ((1 << a.log2n) < n_x) ++a.log2n;
  a.n_t = n_t;
  a.every = n_t / (n_out - 1);
  a.n_out = n_out;
  a.dt = t_end / n_t;
  a.u = u;
  a.status = status;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((a.log2n & 1) == 0) {   // n_x = 4^m, m >= 2: radix-4 pair, n_x / 4 threads
    const size_t lds = (size_t)3 * n_x * sizeof(double2);
    hipLaunchKernelGGL(cdr_strang4_kernel, dim3(B), dim3(n_x / 4), lds, st, a);
  } else {
    const int T = n_x / 2 < 256 ? n_x / 2 : 256;
    const size_t lds = (size_t)(n_x + n_x / 2 + n_x) * sizeof(double2);
    if (n_x / 2 <= 256)
      hipLaunchKernelGGL(cdr_strang_kernel<1>, dim3(B), dim3(T), lds, st, a);
    else
      hipLaunchKernelGGL(cdr_strang_kernel<2>, dim3(B), dim3(T), lds, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "cdr solver launch");
  return LRNR_OK;
}

int32_t lrnr_l1_error(const float* pred, const double* ref, int64_t n, double* out, void* stream) {
  if (n < 0) return fail(LRNR_EINVAL, "n=%lld", (long long)n);
  if (!out || (n > 0 && (!pred || !ref))) return fail(LRNR_EINVAL, "NULL pred, ref or out");
  hipLaunchKernelGGL(l1_error_kernel, dim3(1), dim3(kL1Threads), 0, static_cast<hipStream_t>(stream),
                     pred, ref, n, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "l1 error launch");
  return LRNR_OK;
}

}  // extern "C"
