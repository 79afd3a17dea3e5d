// Fused LRNR / FastLRNR kernel for gfx950: forward jets, CDR residual loss and
// reverse sweep to s and b (arXiv 2410.04001: eq. 2.1-2.2 for the chain, eq. 2.8
// for the reduced chain, eq. 3.5-3.7 for the loss, eq. 4.1 for the residual).
//
// Work mapping.  One lane owns one collocation point for the whole chain, and
// keeps the point's jets (value, d/dx, d/dt, d2/dx2) in registers.  Every
// contraction is a v_mfma_f32_4x4x1_16b_f32 whose 16 blocks of 4 columns are
// the 64 lanes of the wave, so the MFMA result of lane p is always point p:
//
//  * U side, a_c[p][w0+i] += U[w0+i][k] * (s*y_c)[p][k]: A operand lane 4b+i
//    holds U[w0+i][k] (a row of U in LDS), B operand lane p its own (s*y)[k];
//    accumulator GPR i holds neuron w0+i.
//  * V side, y'_c[p][4g+i] += V[w][4g+i] * z_c[p][w]: A operand is a 4-rank
//    slice of row w of V, B operand is z of the lane's own point; accumulator
//    GPR i holds rank 4g+i.
//
// The reduced coordinates y^l = V^lT z^{l-1} (r_l floats per jet) are the only
// per-point state carried between layers; in the gradient mode they are
// checkpointed to global scratch in the forward sweep and the W-wide
// activations are recomputed in the reverse sweep.  The factors of one layer
// are staged into LDS (zero-padded to 4-aligned widths and the compiled rank
// tile RP), which lets the same code run the full LRNR (width M_l) and the
// FastLRNR (width r_hat_l).
#pragma once

#include "lrnr_internal.h"

namespace lrnr {

typedef float f4 __attribute__((ext_vector_type(4)));

#define LRNR_TWO_PI_F 6.28318530717958647692f

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 zero4() { return f4{0.f, 0.f, 0.f, 0.f}; }

// Sum each of the four components of v over the 64 lanes.  On return the lanes
// of 16-lane row q hold the total of component sum4_component(q*16).
__device__ __forceinline__ float wave_sum4(f4 v, int lane) {
  const bool hi32 = lane & 32;
  const float k01 = hi32 ? v[1] : v[0], p01 = hi32 ? v[0] : v[1];
  const float k23 = hi32 ? v[3] : v[2], p23 = hi32 ? v[2] : v[3];
  const float r01 = k01 + __shfl_xor(p01, 32);
  const float r23 = k23 + __shfl_xor(p23, 32);
  const bool hi16 = lane & 16;
  float r = (hi16 ? r23 : r01) + __shfl_xor(hi16 ? r01 : r23, 16);
  r += __shfl_xor(r, 8);
  r += __shfl_xor(r, 4);
  r += __shfl_xor(r, 2);
  r += __shfl_xor(r, 1);
  return r;
}

__device__ __forceinline__ int sum4_component(int lane) {
  return ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1);
}

// ---------------------------------------------------------------------------
// One hidden layer, forward: y (s-scaled in place) -> yo = V^T sin-jets(U y + b)
// ---------------------------------------------------------------------------
template <int NJ, int RGM, int RGI, int RGO>
__device__ __forceinline__ void layer_fwd(const float* __restrict__ Us,
                                          const float* __restrict__ Vs,
                                          const float* __restrict__ bs,
                                          const float* __restrict__ ss, int Wp, int li,
                                          f4 (&y)[NJ][RGM], f4 (&yo)[NJ][RGM]) {
  constexpr int KI = 4 * RGI, KO = 4 * RGO;
#pragma unroll
  for (int g = 0; g < RGI; ++g) {
    const f4 s4 = *reinterpret_cast<const f4*>(ss + 4 * g);
#pragma unroll
    for (int c = 0; c < NJ; ++c) y[c][g] *= s4;
  }
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGO; ++g) yo[c][g] = zero4();

  for (int w0 = 0; w0 < Wp; w0 += 4) {
    f4 a[NJ];
    a[0] = *reinterpret_cast<const f4*>(bs + w0);
#pragma unroll
    for (int c = 1; c < NJ; ++c) a[c] = zero4();
    const float* urow = Us + (w0 + li) * KI;
#pragma unroll
    for (int g = 0; g < RGI; ++g) {
      const f4 u4 = *reinterpret_cast<const f4*>(urow + 4 * g);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int c = 0; c < NJ; ++c) a[c] = mfma4(u4[kk], y[c][g][kk], a[c]);
    }
    f4 z[NJ];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float sn, cs;
      sincosf(a[0][j], &sn, &cs);
      z[0][j] = sn;
      if constexpr (NJ == 4) {
        const float ax = a[1][j];
        z[1][j] = cs * ax;
        z[2][j] = cs * a[2][j];
        z[3][j] = cs * a[3][j] - sn * ax * ax;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float* vrow = Vs + (w0 + j) * KO;
#pragma unroll
      for (int g = 0; g < RGO; ++g) {
        const float v = vrow[4 * g + li];
#pragma unroll
        for (int c = 0; c < NJ; ++c) yo[c][g] = mfma4(v, z[c][j], yo[c][g]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One hidden layer, reverse: recompute a = U (s*y) + b, pull yb = dL/dy^{l+1}
// back through V and the sin jets, write the layer's dL/db row, and return
// wb = U^T abar (so that dL/ds = sum_c wb * y and dL/dy^l = s * wb).
// ---------------------------------------------------------------------------
template <int NJ, int RGM, int RGI, int RGO>
__device__ __forceinline__ void layer_bwd(const float* __restrict__ Us,
                                          const float* __restrict__ Vs,
                                          const float* __restrict__ bs,
                                          const float* __restrict__ ss, int Wp, int li,
                                          int lane, f4 (&y)[NJ][RGM],
                                          const f4 (&yb)[NJ][RGM], f4 (&wb)[NJ][RGM],
                                          float* __restrict__ bbar_row) {
  constexpr int KI = 4 * RGI, KO = 4 * RGO;
#pragma unroll
  for (int g = 0; g < RGI; ++g) {
    const f4 s4 = *reinterpret_cast<const f4*>(ss + 4 * g);
#pragma unroll
    for (int c = 0; c < NJ; ++c) y[c][g] *= s4;
  }
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGI; ++g) wb[c][g] = zero4();
  const int comp = sum4_component(lane);

  for (int w0 = 0; w0 < Wp; w0 += 4) {
    f4 a[NJ];
    a[0] = *reinterpret_cast<const f4*>(bs + w0);
#pragma unroll
    for (int c = 1; c < NJ; ++c) a[c] = zero4();
    const float* urow = Us + (w0 + li) * KI;
#pragma unroll
    for (int g = 0; g < RGI; ++g) {
      const f4 u4 = *reinterpret_cast<const f4*>(urow + 4 * g);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int c = 0; c < NJ; ++c) a[c] = mfma4(u4[kk], y[c][g][kk], a[c]);
    }
    f4 zb[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) zb[c] = zero4();
    const float* vrow = Vs + (w0 + li) * KO;
#pragma unroll
    for (int g = 0; g < RGO; ++g) {
      const f4 v4 = *reinterpret_cast<const f4*>(vrow + 4 * g);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int c = 0; c < NJ; ++c) zb[c] = mfma4(v4[kk], yb[c][g][kk], zb[c]);
    }
    f4 ab[NJ];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float sn, cs;
      sincosf(a[0][j], &sn, &cs);
      if constexpr (NJ == 4) {
        const float ax = a[1][j], at = a[2][j], axx = a[3][j];
        const float zv = zb[0][j], zx = zb[1][j], zt = zb[2][j], zxx = zb[3][j];
        ab[3][j] = cs * zxx;
        ab[2][j] = cs * zt;
        ab[1][j] = cs * zx - 2.f * sn * ax * zxx;
        ab[0][j] = cs * zv - sn * (ax * zx + at * zt + axx * zxx) - cs * ax * ax * zxx;
      } else {
        ab[0][j] = cs * zb[0][j];
      }
    }
    const float bsum = wave_sum4(ab[0], lane);
    if ((lane & 15) == 0) bbar_row[w0 + comp] = bsum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float* ucol = Us + (w0 + j) * KI;
#pragma unroll
      for (int g = 0; g < RGI; ++g) {
        const float u = ucol[4 * g + li];
#pragma unroll
        for (int c = 0; c < NJ; ++c) wb[c][g] = mfma4(u, ab[c][j], wb[c][g]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Workgroup driver
// ---------------------------------------------------------------------------
struct Smem {
  float* Us;
  float* Vs;
  float* bs;
  float* ss;
  float* bbar;   // [kWaves][Wmax_p]
  float* sbar;   // [kWaves][RP]
  float* lw;     // [kWaves][4]
};

// Stage layer l's U^l [Wp][KI], V^{l+1} [Wp][KO], b^l [Wp] and s^l [KI] into
// LDS with zero padding.
__device__ void stage_layer(const KNet& net, const float* __restrict__ s, int l, int KI,
                            int KO, const Smem& sm) {
  const int W = net.M[l], Wp = (W + 3) & ~3, rl = net.r[l], ro = net.r[l + 1];
  const float* __restrict__ U = net.U + net.offU[l];
  const float* __restrict__ V = net.V + net.offV[l + 1];
  const float* __restrict__ b = net.b + net.offB[l];
  for (int i = threadIdx.x; i < Wp * KI; i += kThreads) {
    const int w = i / KI, k = i - w * KI;
    sm.Us[i] = (w < W && k < rl) ? U[w * rl + k] : 0.f;
  }
  for (int i = threadIdx.x; i < Wp * KO; i += kThreads) {
    const int w = i / KO, k = i - w * KO;
    sm.Vs[i] = (w < W && k < ro) ? V[w * ro + k] : 0.f;
  }
  for (int i = threadIdx.x; i < Wp; i += kThreads) sm.bs[i] = i < W ? b[i] : 0.f;
  for (int i = threadIdx.x; i < KI; i += kThreads)
    sm.ss[i] = i < rl ? s[net.offS[l] + i] : 0.f;
}

// Jets of y^1 = V^1T (x, t): value V^1T (x,t), d/dx row 0 of V^1, d/dt row 1,
// d2/dx2 zero (the input layer's trivial reduction).
template <int NJ, int RGM>
__device__ __forceinline__ void input_jets(const KNet& net, float x, float t,
                                           f4 (&y)[NJ][RGM]) {
  const int r1 = net.r[1];
  const float* V1 = net.V + net.offV[1];
  const float v00 = V1[0], v10 = V1[r1];
  const float v01 = r1 > 1 ? V1[1] : 0.f, v11 = r1 > 1 ? V1[r1 + 1] : 0.f;
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGM; ++g) y[c][g] = zero4();
  y[0][0] = f4{v00 * x + v10 * t, v01 * x + v11 * t, 0.f, 0.f};
  if constexpr (NJ == 4) {
    y[1][0] = f4{v00, v01, 0.f, 0.f};
    y[2][0] = f4{v10, v11, 0.f, 0.f};
  }
}

template <int NJ, int RGM>
__device__ __forceinline__ void fwd_dispatch(bool first, bool last, const Smem& sm, int Wp,
                                             int li, f4 (&y)[NJ][RGM],
                                             f4 (&yo)[NJ][RGM]) {
  if (first && last)
    layer_fwd<NJ, RGM, 1, 1>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, y, yo);
  else if (first)
    layer_fwd<NJ, RGM, 1, RGM>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, y, yo);
  else if (last)
    layer_fwd<NJ, RGM, RGM, 1>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, y, yo);
  else
    layer_fwd<NJ, RGM, RGM, RGM>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, y, yo);
}

template <int NJ, int RGM>
__device__ __forceinline__ void bwd_dispatch(bool first, bool last, const Smem& sm, int Wp,
                                             int li, int lane, f4 (&y)[NJ][RGM],
                                             const f4 (&yb)[NJ][RGM], f4 (&wb)[NJ][RGM],
                                             float* bbar_row) {
  if (first && last)
    layer_bwd<NJ, RGM, 1, 1>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, lane, y, yb, wb, bbar_row);
  else if (first)
    layer_bwd<NJ, RGM, 1, RGM>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, lane, y, yb, wb, bbar_row);
  else if (last)
    layer_bwd<NJ, RGM, RGM, 1>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, lane, y, yb, wb, bbar_row);
  else
    layer_bwd<NJ, RGM, RGM, RGM>(sm.Us, sm.Vs, sm.bs, sm.ss, Wp, li, lane, y, yb, wb,
                                 bbar_row);
}

template <int NJ, int RGM>
__device__ __forceinline__ void ckpt_store(float* __restrict__ base, int lane,
                                           const f4 (&y)[NJ][RGM]) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGM; ++g)
      *reinterpret_cast<f4*>(base + ((c * RGM + g) * 64 + lane) * 4) = y[c][g];
}

template <int NJ, int RGM>
__device__ __forceinline__ void ckpt_load(const float* __restrict__ base, int lane,
                                          f4 (&y)[NJ][RGM]) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGM; ++g)
      y[c][g] = *reinterpret_cast<const f4*>(base + ((c * RGM + g) * 64 + lane) * 4);
}

template <int RP, int MODE, int NJ>
__device__ void run_workgroup(const KNet& net, const KInst& inst, const KGrid& grid,
                              int kind, int wg, const float* __restrict__ s,
                              const float* __restrict__ mu, const Smem& sm) {
  constexpr int RGM = RP / 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 3;
  const int L = net.L;

  // ---- the lane's point -------------------------------------------------
  float x = 0.f, t = 0.f;
  bool valid = false;
  int64_t p = 0;
  if (kind == 0) {
    p = (int64_t)wg * kPtsPerWG + wave * 64 + lane;
    valid = p < inst.n_r;
    if (valid) {
      x = inst.xt_r[2 * p];
      t = inst.xt_r[2 * p + 1];
    }
  } else if (kind == 1) {
    p = (int64_t)wg * kPtsPerWG + wave * 64 + lane;
    valid = p < inst.n_0;
    if (valid) x = inst.x_0[p];
  } else {
    p = (int64_t)wg * kBcPairsPerWG + wave * 32 + (lane >> 1);
    valid = p < inst.n_b;
    x = (lane & 1) ? LRNR_TWO_PI_F : 0.f;
    if (valid) t = inst.t_b[p];
  }

  float* ckbase = nullptr;
  if constexpr (MODE == MODE_GRAD)
    ckbase = grid.ckpt + ((int64_t)blockIdx.x * kWaves + wave) * grid.ckpt_per_wave;
  constexpr int64_t kSlot = 4 * RGM * 64 * 4;  // floats per checkpointed layer

  // ---- forward sweep ------------------------------------------------------
  f4 y[NJ][RGM], yo[NJ][RGM];
  input_jets<NJ, RGM>(net, x, t, y);
  for (int l = 1; l <= L - 1; ++l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    __syncthreads();
    stage_layer(net, s, l, KI, KO, sm);
    __syncthreads();
    const int Wp = (net.M[l] + 3) & ~3;
    fwd_dispatch<NJ, RGM>(first, last, sm, Wp, li, y, yo);
    if constexpr (MODE == MODE_GRAD)
      if (!last) ckpt_store<NJ, RGM>(ckbase + (l - 1) * kSlot, lane, yo);
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
      for (int g = 0; g < RGM; ++g) y[c][g] = yo[c][g];
  }

  // ---- output layer: u = U^L (s^L * y^L) + b^L (r_L = M_L = 1) ------------
  const float UL = net.U[net.offU[L]];
  const float sL = s[net.offS[L]];
  const float bL = net.b[net.offB[L]];
  const float cL = UL * sL;
  float u[NJ];
#pragma unroll
  for (int c = 0; c < NJ; ++c) u[c] = cL * y[c][0][0];
  u[0] += bL;

  if constexpr (MODE == MODE_JETS) {
    if (valid) {
      const int64_t n = inst.n_r;
#pragma unroll
      for (int c = 0; c < NJ; ++c) inst.out[c * n + p] = u[c];
    }
    return;
  }
  if constexpr (MODE == MODE_VALUE) {
    if (valid) inst.out[p] = u[0];
    return;
  }

  // ---- residual (eq. 4.1) and loss adjoints (eq. 3.5 / 3.6) -------------
  const int form = inst.form;
  float lsum = 0.f;
  float ub[NJ];
#pragma unroll
  for (int c = 0; c < NJ; ++c) ub[c] = 0.f;
  if constexpr (NJ == 4) {
    const float beta = mu[0], nu = mu[1], rho = mu[2];
    const float res = u[2] + beta * u[1] - nu * u[3] - rho * u[0] * (1.f - u[0]);
    const float phi = form == 0 ? res * res : fabsf(res);
    const float dphi = form == 0 ? 2.f * res : (res > 0.f ? 1.f : (res < 0.f ? -1.f : 0.f));
    const float g = valid ? inst.wr_n * dphi : 0.f;
    lsum = valid ? phi : 0.f;
    ub[0] = -rho * (1.f - 2.f * u[0]) * g;
    ub[1] = beta * g;
    ub[2] = g;
    ub[3] = -nu * g;
  } else if (kind == 1) {
    const float e0 = u[0] - sinf(x);
    const float phi = form == 0 ? e0 * e0 : fabsf(e0);
    const float dphi = form == 0 ? 2.f * e0 : (e0 > 0.f ? 1.f : (e0 < 0.f ? -1.f : 0.f));
    lsum = valid ? phi : 0.f;
    ub[0] = valid ? inst.w0_n * dphi : 0.f;
  } else {
    const float other = __shfl_xor(u[0], 1);
    const bool right = lane & 1;
    const float eb = right ? other - u[0] : u[0] - other;
    const float phi = form == 0 ? eb * eb : fabsf(eb);
    const float dphi = form == 0 ? 2.f * eb : (eb > 0.f ? 1.f : (eb < 0.f ? -1.f : 0.f));
    lsum = (valid && !right) ? phi : 0.f;
    ub[0] = valid ? (right ? -inst.wb_n : inst.wb_n) * dphi : 0.f;
  }

  float* rec = grid.partials + (int64_t)blockIdx.x * grid.P;
  const int comp = sum4_component(lane);

  if constexpr (MODE == MODE_LOSS) {
    const float tot = wave_sum4(f4{lsum, 0.f, 0.f, 0.f}, lane);
    if ((lane & 15) == 0) sm.lw[wave * 4 + comp] = tot;
    __syncthreads();
    if (tid < 4) {
      const float v = ((sm.lw[0] + sm.lw[4]) + sm.lw[8]) + sm.lw[12];
      rec[tid] = tid == kind ? v : 0.f;
    }
    return;
  }

  // ---- output layer reverse ---------------------------------------------
  {
    float sLb = 0.f;
#pragma unroll
    for (int c = 0; c < NJ; ++c) sLb += ub[c] * y[c][0][0];
    const float tot = wave_sum4(f4{lsum, UL * sLb, ub[0], 0.f}, lane);
    if ((lane & 15) == 0) sm.lw[wave * 4 + comp] = tot;
  }
  f4 yb[NJ][RGM], wb[NJ][RGM];
#pragma unroll
  for (int c = 0; c < NJ; ++c) {
#pragma unroll
    for (int g = 0; g < RGM; ++g) yb[c][g] = zero4();
    yb[c][0][0] = cL * ub[c];
  }

  // ---- reverse sweep over the hidden layers --------------------------------
  for (int l = L - 1; l >= 1; --l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    const int Wp = (net.M[l] + 3) & ~3;
    __syncthreads();
    if (l == L - 1 && tid < 4) {
      // loss sums and the output layer's s and b gradients
      const float v = ((sm.lw[tid] + sm.lw[4 + tid]) + sm.lw[8 + tid]) + sm.lw[12 + tid];
      if (tid == 0) {
        rec[0] = kind == 0 ? v : 0.f;
        rec[1] = kind == 1 ? v : 0.f;
        rec[2] = kind == 2 ? v : 0.f;
        rec[3] = 0.f;
      } else if (tid == 1) {
        rec[4 + net.offS[L]] = v;
      } else if (tid == 2) {
        rec[4 + net.r_total + net.offB[L]] = v;
      }
    }
    stage_layer(net, s, l, KI, KO, sm);
    __syncthreads();
    if (first)
      input_jets<NJ, RGM>(net, x, t, y);
    else
      ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
    bwd_dispatch<NJ, RGM>(first, last, sm, Wp, li, lane, y, yb, wb, sm.bbar + wave * grid.Wmax_p);
    if (first)
      input_jets<NJ, RGM>(net, x, t, y);
    else
      ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
    const int RGI = first ? 1 : RGM;
#pragma unroll
    for (int g = 0; g < RGM; ++g) {
      if (g < RGI) {
        f4 acc = zero4();
#pragma unroll
        for (int c = 0; c < NJ; ++c) acc += wb[c][g] * y[c][g];
        const float tot = wave_sum4(acc, lane);
        if ((lane & 15) == 0) sm.sbar[wave * RP + 4 * g + comp] = tot;
      }
    }
    if (!first) {
#pragma unroll
      for (int g = 0; g < RGM; ++g) {
        const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + 4 * g);
#pragma unroll
        for (int c = 0; c < NJ; ++c) yb[c][g] = s4 * wb[c][g];
      }
    }
    __syncthreads();
    // the layer's s and b gradients, waves summed in a fixed order
    const int W = net.M[l], rl = net.r[l], Wm = grid.Wmax_p;
    for (int i = tid; i < W; i += kThreads)
      rec[4 + net.r_total + net.offB[l] + i] =
          ((sm.bbar[i] + sm.bbar[Wm + i]) + sm.bbar[2 * Wm + i]) + sm.bbar[3 * Wm + i];
    for (int i = tid; i < rl; i += kThreads)
      rec[4 + net.offS[l] + i] =
          ((sm.sbar[i] + sm.sbar[RP + i]) + sm.sbar[2 * RP + i]) + sm.sbar[3 * RP + i];
  }
}

template <int RP, int MODE>
__global__ __launch_bounds__(kThreads) void lrnr_fused_kernel(KNet net, KInst inst,
                                                              KGrid grid) {
  extern __shared__ float4 smem_raw[];
  float* base = reinterpret_cast<float*>(smem_raw);
  const int Wm = grid.Wmax_p;
  Smem sm;
  sm.Us = base;
  sm.Vs = sm.Us + Wm * RP;
  sm.bs = sm.Vs + Wm * RP;
  sm.ss = sm.bs + Wm;
  sm.bbar = sm.ss + RP;
  sm.sbar = sm.bbar + kWaves * Wm;
  sm.lw = sm.sbar + kWaves * RP;

  const int inst_id = blockIdx.x / grid.G_inst;
  int wg = blockIdx.x - inst_id * grid.G_inst;
  int kind = 0;
  if (wg >= grid.G_r + grid.G_0) {
    kind = 2;
    wg -= grid.G_r + grid.G_0;
  } else if (wg >= grid.G_r) {
    kind = 1;
    wg -= grid.G_r;
  }
  const float* s = inst.s + inst_id * grid.s_stride;
  const float* mu = inst.mu ? inst.mu + 3 * inst_id : nullptr;
  if constexpr (MODE == MODE_VALUE) {
    run_workgroup<RP, MODE, 1>(net, inst, grid, kind, wg, s, mu, sm);
  } else if constexpr (MODE == MODE_JETS) {
    run_workgroup<RP, MODE, 4>(net, inst, grid, kind, wg, s, mu, sm);
  } else {
    if (kind == 0)
      run_workgroup<RP, MODE, 4>(net, inst, grid, kind, wg, s, mu, sm);
    else
      run_workgroup<RP, MODE, 1>(net, inst, grid, kind, wg, s, mu, sm);
  }
}

template <int RP>
hipError_t launch_rp(int mode, const KNet& net, const KInst& inst, const KGrid& grid,
                            hipStream_t stream) {
  const dim3 blocks((unsigned)(grid.B * grid.G_inst)), threads(kThreads);
  const size_t lds = fused_lds_bytes(RP, grid.Wmax_p);
  if (lds > 65536) {
    const void* fns[4] = {(const void*)lrnr_fused_kernel<RP, MODE_JETS>,
                          (const void*)lrnr_fused_kernel<RP, MODE_VALUE>,
                          (const void*)lrnr_fused_kernel<RP, MODE_LOSS>,
                          (const void*)lrnr_fused_kernel<RP, MODE_GRAD>};
    hipError_t e = hipFuncSetAttribute(fns[mode & 3], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  switch (mode) {
    case MODE_JETS:
      hipLaunchKernelGGL((lrnr_fused_kernel<RP, MODE_JETS>), blocks, threads, lds, stream, net,
                         inst, grid);
      break;
    case MODE_VALUE:
      hipLaunchKernelGGL((lrnr_fused_kernel<RP, MODE_VALUE>), blocks, threads, lds, stream, net,
                         inst, grid);
      break;
    case MODE_LOSS:
      hipLaunchKernelGGL((lrnr_fused_kernel<RP, MODE_LOSS>), blocks, threads, lds, stream, net,
                         inst, grid);
      break;
    default:
      hipLaunchKernelGGL((lrnr_fused_kernel<RP, MODE_GRAD>), blocks, threads, lds, stream, net,
                         inst, grid);
      break;
  }
  return hipGetLastError();
}

}  // namespace lrnr
