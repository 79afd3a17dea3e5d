// Wave-specialised loss + gradient kernel (the LRNR / FastLRNR hot path of
// arXiv 2410.04001: eq. 2.1-2.2 / 2.8 chain with jets, eq. 4.1 residual,
// eq. 3.5-3.7 loss, reverse sweep to s and b).
//
// Every 64-point tile is owned by four waves, one per role, on one SIMD
// (waves w, w + 4, w + 8, w + 12 of the 16-wave workgroup):
//
//          forward                          reverse
//   M1     a = U (s y) + b     (MFMA)       a = U (s y) + b        (MFMA)
//   S0/S1  sin jets of half of the group    S0: adjoint of the sin jets and
//          each (VALU)                      the db row (VALU); S1: wbar +=
//                                           U^T abar (MFMA), then ds, ybar
//   M2     y' += V^T z (MFMA), then the     zbar = V ybar          (MFMA)
//          output layer and the residual
//
// Both sweeps are three-stage pipelines over 4-neuron groups (producers on
// group g, the middle stage on g - 1, the consumer on g - 2); values cross
// between roles through double-buffered LDS slots and one workgroup barrier
// ends every step.  No role holds more than one rank-sized jet array
// (4 x RP registers), so four waves fit per SIMD.  On this hardware FP32
// MFMA and VALU work of one SIMD do not overlap (measured), so the split does
// not hide the VALU work; it hides latency: while one wave waits on an LDS
// read, a barrier or a dependent MFMA, another wave of the SIMD issues.
// The role loops are separate code paths with equal barrier counts (the
// hardware barrier counts waves, not program locations).
//
// Between layers the reduced jets pass from wave to wave through the tile's
// exchange slots (M2 -> M1: y^{l+1} forward; S1 -> M2: ybar^l reverse).  The
// forward y^{l+1} also go to the tile's global checkpoint slab, from which
// M1 (U-side recompute) and S1 (ds term) read them in the reverse sweep.
// Layers are staged into LDS by the waves that are idle at the boundary.
#pragma once

#include <algorithm>
#include <map>
#include <mutex>

#include "lrnr_fused_impl.h"

namespace lrnr {

constexpr int kWsWaves = 16;
constexpr int kWsThreads = 64 * kWsWaves;
constexpr int kXFloats = 4 * 64 * 4;   // one exchange slot: 4 f4 per lane
constexpr int kMaxCols = 2;            // value points per lane of a value-only tile

typedef float f2 __attribute__((ext_vector_type(2)));

struct SmemWS {
  float* Us;
  float* Vs;
  float* bs;
  float* ss;    // [2][RP]: s^l of layer l in buffer l & 1
  float* xa;    // [4 tiles][2 slots][kXFloats]  a                     (M1 -> S)
  float* xz;    // [4 tiles][2 slots][kXFloats]  z (S -> M2) / zbar (M2 -> S0)
  float* xg;    // [4 tiles][2 slots][kXFloats]  abar                  (S0 -> S1)
  float* bbar;  // [kMaxCols][4][Wmax_p]
  float* sbar;  // [kMaxCols][4][RP]
  float* lw;    // [kMaxCols][16] loss sums, [16] range flags
};

inline size_t ws_lds_floats(int RP, int Wmax_p) {
  return (size_t)Wmax_p * RP * 2 + Wmax_p + 2 * RP + (size_t)3 * 4 * 2 * kXFloats +
         (size_t)kMaxCols * 4 * (Wmax_p + RP) + 16 * (kMaxCols + 1);
}

__device__ __forceinline__ SmemWS ws_smem(float* base, int Wm, int RP) {
  SmemWS sm;
  sm.Us = base;
  sm.Vs = sm.Us + Wm * RP;
  sm.bs = sm.Vs + Wm * RP;
  sm.ss = sm.bs + Wm;
  sm.xa = sm.ss + 2 * RP;
  sm.xz = sm.xa + 4 * 2 * kXFloats;
  sm.xg = sm.xz + 4 * 2 * kXFloats;
  sm.bbar = sm.xg + 4 * 2 * kXFloats;
  sm.sbar = sm.bbar + kMaxCols * 4 * Wm;
  sm.lw = sm.sbar + kMaxCols * 4 * RP;
  return sm;
}

template <int N>
__device__ __forceinline__ void xput(float* __restrict__ slot, int lane, const f4 (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) *reinterpret_cast<f4*>(slot + (i * 64 + lane) * 4) = v[i];
}

template <int N>
__device__ __forceinline__ void xget(const float* __restrict__ slot, int lane, f4 (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = *reinterpret_cast<const f4*>(slot + (i * 64 + lane) * 4);
}

// Half h (neurons 2h, 2h+1) of each f4 in a slot.
template <int N>
__device__ __forceinline__ void xput2(float* __restrict__ slot, int lane, int h,
                                      const f2 (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) *reinterpret_cast<f2*>(slot + (i * 64 + lane) * 4 + 2 * h) = v[i];
}

template <int N>
__device__ __forceinline__ void xget2(const float* __restrict__ slot, int lane, int h,
                                      f2 (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    v[i] = *reinterpret_cast<const f2*>(slot + (i * 64 + lane) * 4 + 2 * h);
}

// sin jets of two neurons (the policy of sincos4: hardware sin/cos when the
// whole wave is within kHwRange, else the Cody-Waite polynomial)
template <int NJ>
__device__ __forceinline__ void sigma_fwd2(const f2 (&a)[NJ], f2 (&z)[NJ], float& amax) {
  const float m = vmax(fabsf(a[0][0]), fabsf(a[0][1]));
  amax = vmax(amax, m);
  f2 sn, cs;
  if (__all(m <= kHwRange)) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float sj, cj;
      sincos_hw(a[0][j], sj, cj);
      sn[j] = sj;
      cs[j] = cj;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float sj, cj;
      sincos_fast(a[0][j], sj, cj);
      sn[j] = sj;
      cs[j] = cj;
    }
  }
  z[0] = sn;
  if constexpr (NJ == 4) {
    const f2 ax = a[1];
    z[1] = cs * ax;
    z[2] = cs * a[2];
    z[3] = cs * a[3] - sn * ax * ax;
  }
}

// sin of N pairs of pre-activations of value-only columns (independent
// points, no derivative jets), with one wave-uniform range test for all
template <int N>
__device__ __forceinline__ void sigma_fwd_vals(const f2 (&a)[N], f2 (&z)[N], float& amax) {
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) m = vmax(m, vmax(fabsf(a[i][0]), fabsf(a[i][1])));
  amax = vmax(amax, m);
  if (__all(m <= kHwRange)) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        float sj, cj;
        sincos_hw(a[i][j], sj, cj);
        z[i][j] = sj;
      }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        float sj, cj;
        sincos_fast(a[i][j], sj, cj);
        z[i][j] = sj;
      }
  }
}

// adjoint of sigma_fwd_vals: abar = cos(a) zbar
template <int N>
__device__ __forceinline__ void sigma_bwd_vals(const f4 (&a)[N], const f4 (&zb)[N], f4 (&ab)[N],
                                               float& amax) {
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i)
    m = vmax(m, vmax(vmax(fabsf(a[i][0]), fabsf(a[i][1])), vmax(fabsf(a[i][2]), fabsf(a[i][3]))));
  amax = vmax(amax, m);
  if (__all(m <= kHwRange)) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float sj, cj;
        sincos_hw(a[i][j], sj, cj);
        ab[i][j] = cj * zb[i][j];
      }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float sj, cj;
        sincos_fast(a[i][j], sj, cj);
        ab[i][j] = cj * zb[i][j];
      }
  }
}

// ---------------------------------------------------------------------------
// Contractions of one 4-neuron group with the factor entries read from LDS
// one rank group (or one neuron) ahead of the MFMAs that use them, which keeps
// the operand registers of a role small.
// ---------------------------------------------------------------------------

// out = R[w0..w0+3] y (+ bias): R row-major [W][4 RG], y in rank space
template <int NJ, int RGM, int RG, bool BIAS>
__device__ __forceinline__ void rows_times(const float* __restrict__ R,
                                           const float* __restrict__ bs, int w0, int li,
                                           const f4 (&y)[NJ][RGM], f4 (&out)[NJ]) {
  constexpr int K = 4 * RG;
  const float* row = R + (w0 + li) * K;
  if constexpr (BIAS)
    out[0] = *reinterpret_cast<const f4*>(bs + w0);
  else
    out[0] = zero4();
#pragma unroll
  for (int c = 1; c < NJ; ++c) out[c] = zero4();
  f4 nxt = *reinterpret_cast<const f4*>(row);
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const f4 cur = nxt;
    if (g + 1 < RG) nxt = *reinterpret_cast<const f4*>(row + 4 * (g + 1));
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int c = 0; c < NJ; ++c) out[c] = mfma4(cur[kk], y[c][g][kk], out[c]);
  }
}

// rows_times for NG consecutive groups w0, w0+4, ... at once: out[q * NJ + c]
// is jet c of group q.  The NG x NJ accumulator chains are interleaved, which
// keeps the one-jet (value-only) tiles from waiting on a single dependent
// MFMA chain; for NG = 1 this is rows_times.
template <int NJ, int RGM, int RG, bool BIAS, int NG, int KLAST = 4>
__device__ __forceinline__ void rows_times_ng(const float* __restrict__ R,
                                              const float* __restrict__ bs, int w0, int li,
                                              const f4 (&y)[NJ][RGM], f4 (&out)[NJ * NG]) {
  constexpr int K = 4 * RG;
  f4 nxt[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    f4 bias = zero4();
    if constexpr (BIAS) bias = *reinterpret_cast<const f4*>(bs + w0 + 4 * q);
    out[q * NJ] = bias;
    // four jets: the bias enters the value jet only; value columns: every one
#pragma unroll
    for (int c = 1; c < NJ; ++c) out[q * NJ + c] = NJ == 4 ? zero4() : bias;
    nxt[q] = *reinterpret_cast<const f4*>(R + (w0 + 4 * q + li) * K);
  }
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    f4 cur[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) cur[q] = nxt[q];
    if (g + 1 < RG) {
#pragma unroll
      for (int q = 0; q < NG; ++q)
        nxt[q] = *reinterpret_cast<const f4*>(R + (w0 + 4 * q + li) * K + 4 * (g + 1));
    }
    // the last rank group may be zero-padded beyond KLAST (the input layer:
    // r_1 <= 2 because (x, t) has two components)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (g < RG - 1 || kk < KLAST) {
#pragma unroll
        for (int q = 0; q < NG; ++q)
#pragma unroll
          for (int c = 0; c < NJ; ++c)
            out[q * NJ + c] = mfma4(cur[q][kk], y[c][g][kk], out[q * NJ + c]);
      }
    }
  }
}

// acc += R[w0..w0+3]^T v: R row-major [W][4 RG], v per neuron (f4 of 4 neurons)
template <int NJ, int RGM, int RG>
__device__ __forceinline__ void rows_t_times(const float* __restrict__ R, int w0, int li,
                                             const f4 (&v)[NJ], f4 (&acc)[NJ][RGM]) {
  constexpr int K = 4 * RG;
  float nxt[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) nxt[g] = R[w0 * K + 4 * g + li];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float cur[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) cur[g] = nxt[g];
    if (j + 1 < 4) {
#pragma unroll
      for (int g = 0; g < RG; ++g) nxt[g] = R[(w0 + j + 1) * K + 4 * g + li];
    }
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
      for (int c = 0; c < NJ; ++c) acc[c][g] = mfma4(cur[g], v[c][j], acc[c][g]);
  }
}

// ---------------------------------------------------------------------------
// Role loops of one hidden layer: `steps` steps, each ending in a workgroup
// barrier; step k works on neuron block k - (stage of the role) when that
// exists.  A block is NG 4-neuron groups: NG = 1 for the four-jet interior
// tiles, NG = 4 for the value-only IC/BC tiles, so every exchange slot holds
// NJ x NG = 4 f4 per lane and value-only tiles need a quarter of the steps.
// Slot entry q * NJ + c is jet c of group q.
// ---------------------------------------------------------------------------

// M1: a = U (s y) + b for block k (both sweeps)
template <int NJ, int RGM, int RGI, int NG, int KLAST = 4>
__device__ __forceinline__ void m1_loop(const SmemWS& sm, float* xa, int Gs, int steps, int li,
                                        int lane, const f4 (&ys)[NJ][RGM]) {
  for (int k = 0; k < steps; ++k) {
    if (k < Gs) {
      f4 a[NJ * NG];
      rows_times_ng<NJ, RGM, RGI, true, NG, KLAST>(sm.Us, sm.bs, 4 * k * NG, li, ys, a);
      xput<NJ * NG>(xa + (k & 1) * kXFloats, lane, a);
    }
    __syncthreads();
  }
}

// S0 / S1 forward: sin jets of neurons 2h, 2h+1 of every group of block k - 1
template <int NJ, int NG>
__device__ __forceinline__ void s_fwd_loop(const float* xa, float* xz, int Gs, int lane, int h,
                                           float& amax) {
  for (int k = 0; k < Gs + 2; ++k) {
    if (k >= 1 && k <= Gs) {
      f2 a[NJ * NG], z[NJ * NG];
      xget2<NJ * NG>(xa + ((k - 1) & 1) * kXFloats, lane, h, a);
      if constexpr (NJ == 4) {
#pragma unroll
        for (int q = 0; q < NG; ++q) {
          f2 aq[NJ], zq[NJ];
#pragma unroll
          for (int c = 0; c < NJ; ++c) aq[c] = a[q * NJ + c];
          sigma_fwd2<NJ>(aq, zq, amax);
#pragma unroll
          for (int c = 0; c < NJ; ++c) z[q * NJ + c] = zq[c];
        }
      } else {
        sigma_fwd_vals<NJ * NG>(a, z, amax);
      }
      xput2<NJ * NG>(xz + ((k - 1) & 1) * kXFloats, lane, h, z);
    }
    __syncthreads();
  }
}

// M2 forward: y' += V^T z for block k - 2
template <int NJ, int RGM, int RGO, int NG>
__device__ __forceinline__ void m2_fwd_loop(const SmemWS& sm, const float* xz, int Gs, int li,
                                            int lane, f4 (&y)[NJ][RGM]) {
  for (int k = 0; k < Gs + 2; ++k) {
    if (k >= 2) {
      f4 z[NJ * NG];
      xget<NJ * NG>(xz + (k & 1) * kXFloats, lane, z);
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        f4 zq[NJ];
#pragma unroll
        for (int c = 0; c < NJ; ++c) zq[c] = z[q * NJ + c];
        rows_t_times<NJ, RGM, RGO>(sm.Vs, 4 * ((k - 2) * NG + q), li, zq, y);
      }
    }
    __syncthreads();
  }
}

// M2 reverse: zbar = V ybar for block k
template <int NJ, int RGM, int RGO, int NG>
__device__ __forceinline__ void m2_bwd_loop(const SmemWS& sm, float* xz, int Gs, int li,
                                            int lane, const f4 (&yb)[NJ][RGM]) {
  for (int k = 0; k < Gs + 2; ++k) {
    if (k < Gs) {
      f4 zb[NJ * NG];
      rows_times_ng<NJ, RGM, RGO, false, NG>(sm.Vs, nullptr, 4 * k * NG, li, yb, zb);
      xput<NJ * NG>(xz + (k & 1) * kXFloats, lane, zb);
    }
    __syncthreads();
  }
}

// S0 reverse: adjoint of the sin jets and the db row for block k - 1
// (bbar_row + c * col_stride is the db row of value column c)
template <int NJ, int NG>
__device__ __forceinline__ void s0_bwd_loop(const float* xa, const float* xz, float* xg, int Gs,
                                            int lane, float* __restrict__ bbar_row,
                                            int col_stride, float& amax) {
  const int comp = sum4_component(lane);
  for (int k = 0; k < Gs + 2; ++k) {
    if (k >= 1 && k <= Gs) {
      const int slot = ((k - 1) & 1) * kXFloats;
      f4 a[NJ * NG], zb[NJ * NG], ab[NJ * NG];
      xget<NJ * NG>(xa + slot, lane, a);
      xget<NJ * NG>(xz + slot, lane, zb);
      if constexpr (NJ == 4) {
#pragma unroll
        for (int q = 0; q < NG; ++q) {
          f4 aq[NJ], zq[NJ], gq[NJ];
#pragma unroll
          for (int c = 0; c < NJ; ++c) {
            aq[c] = a[q * NJ + c];
            zq[c] = zb[q * NJ + c];
          }
          sigma_bwd<NJ, false>(aq, zq, gq, amax);
#pragma unroll
          for (int c = 0; c < NJ; ++c) ab[q * NJ + c] = gq[c];
        }
      } else {
        sigma_bwd_vals<NJ * NG>(a, zb, ab, amax);
      }
      xput<NJ * NG>(xg + slot, lane, ab);
      // db: the value jet of a four-jet tile; every column of a value tile
      constexpr int NB = NJ == 4 ? 1 : NJ;
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const float bsum = wave_sum4(ab[q * NJ + c], lane);
          if ((lane & 15) == 0) bbar_row[c * col_stride + 4 * ((k - 1) * NG + q) + comp] = bsum;
        }
    }
    __syncthreads();
  }
}

// S1 reverse: wbar += U^T abar for block k - 2
template <int NJ, int RGM, int RGI, int NG>
__device__ __forceinline__ void s1_bwd_loop(const SmemWS& sm, const float* xg, int Gs, int li,
                                            int lane, f4 (&wb)[NJ][RGM]) {
  for (int k = 0; k < Gs + 2; ++k) {
    if (k >= 2) {
      f4 ab[NJ * NG];
      xget<NJ * NG>(xg + (k & 1) * kXFloats, lane, ab);
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        f4 gq[NJ];
#pragma unroll
        for (int c = 0; c < NJ; ++c) gq[c] = ab[q * NJ + c];
        rows_t_times<NJ, RGM, RGI>(sm.Us, 4 * ((k - 2) * NG + q), li, gq, wb);
      }
    }
    __syncthreads();
  }
}

// One rank group of a checkpointed jet array.
template <int NJ, int RGM>
__device__ __forceinline__ void ckpt_load_g(const float* __restrict__ base, int lane, int g,
                                            f4 (&y)[NJ]) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
    y[c] = *reinterpret_cast<const f4*>(base + ((c * RGM + g) * 64 + lane) * 4);
}

// Rank group 0 of the input layer's jets (V^1T (x, t) and its constant jets).
template <int NJ>
__device__ __forceinline__ void input_jets_g0(const KNet& net, float x, float t, f4 (&y)[NJ]) {
  const int r1 = net.r[1];
  const float* V1 = net.V + net.offV[1];
  const float v00 = V1[0], v10 = V1[r1];
  const float v01 = r1 > 1 ? V1[1] : 0.f, v11 = r1 > 1 ? V1[r1 + 1] : 0.f;
  y[0] = f4{v00 * x + v10 * t, v01 * x + v11 * t, 0.f, 0.f};
  if constexpr (NJ == 4) {
    y[1] = f4{v00, v01, 0.f, 0.f};
    y[2] = f4{v10, v11, 0.f, 0.f};
    y[3] = zero4();
  }
}

// y^1 = V^1T (x, t) of NC independent points (value-only columns).
template <int NC, int RGM>
__device__ __forceinline__ void input_vals(const KNet& net, const float (&x)[NC],
                                           const float (&t)[NC], f4 (&y)[NC][RGM]) {
  const int r1 = net.r[1];
  const float* V1 = net.V + net.offV[1];
  const float v00 = V1[0], v10 = V1[r1];
  const float v01 = r1 > 1 ? V1[1] : 0.f, v11 = r1 > 1 ? V1[r1 + 1] : 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int g = 0; g < RGM; ++g) y[c][g] = zero4();
    y[c][0] = f4{v00 * x[c] + v10 * t[c], v01 * x[c] + v11 * t[c], 0.f, 0.f};
  }
}

template <int NC>
__device__ __forceinline__ void input_vals_g0(const KNet& net, const float (&x)[NC],
                                              const float (&t)[NC], f4 (&y)[NC]) {
  const int r1 = net.r[1];
  const float* V1 = net.V + net.offV[1];
  const float v00 = V1[0], v10 = V1[r1];
  const float v01 = r1 > 1 ? V1[1] : 0.f, v11 = r1 > 1 ? V1[r1 + 1] : 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    y[c] = f4{v00 * x[c] + v10 * t[c], v01 * x[c] + v11 * t[c], 0.f, 0.f};
}

// A tile's reduced jets (NJ x RGM f4 per lane) handed from one wave to another
// at a layer boundary through the tile's exchange slots, five slots of 4 f4
// per lane in the order xz[0], xz[1], xg[0], xg[1], xa[1].  At the first step
// of the next layer only xa[0] (M1, forward and reverse) and xz[0] (M2,
// reverse, after its own read) are written, so the reader takes them at that
// step and nothing else touches them before the step's barrier.
__device__ __forceinline__ float* yx_slot(float* xa, float* xz, float* xg, int i) {
  const int q = i >> 2;
  float* base = q == 0 ? xz : q == 1 ? xz + kXFloats : q == 2 ? xg : q == 3 ? xg + kXFloats
                                                                         : xa + kXFloats;
  return base + (i & 3) * 64 * 4;
}

template <int NJ, int RGM>
__device__ __forceinline__ void yx_put(float* xa, float* xz, float* xg, int lane,
                                       const f4 (&y)[NJ][RGM]) {
  static_assert(NJ * RGM <= 20, "five exchange slots of 4 f4 per lane");
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGM; ++g)
      *reinterpret_cast<f4*>(yx_slot(xa, xz, xg, c * RGM + g) + lane * 4) = y[c][g];
}

template <int NJ, int RGM>
__device__ __forceinline__ void yx_get_g(float* xa, float* xz, float* xg, int lane, int g,
                                         f4 (&y)[NJ]) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
    y[c] = *reinterpret_cast<const f4*>(yx_slot(xa, xz, xg, c * RGM + g) + lane * 4);
}

template <int NJ, int RGM>
__device__ __forceinline__ void yx_get(float* xa, float* xz, float* xg, int lane,
                                       f4 (&y)[NJ][RGM]) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGM; ++g)
      y[c][g] = *reinterpret_cast<const f4*>(yx_slot(xa, xz, xg, c * RGM + g) + lane * 4);
}

// ---------------------------------------------------------------------------
// Workgroup driver (MODE_GRAD / MODE_VJP, fast sin/cos with range tracking).
//
// NJ = 4: four-jet interior tile (one point per lane).  NJ < 4: value-only
// IC/BC tiles with NJ independent points per lane ("columns"); column c of
// workgroup wg covers tile NJ wg + c of its kind and reduces into that tile's
// own record (tiles[c]), so records, flags and the accurate relaunch are the
// same whatever the number of columns.  n_tiles is the number of tiles of
// this kind (a trailing column beyond it writes nothing).
// ---------------------------------------------------------------------------
template <int RP, int NJ, bool VJP>
__device__ void ws_run(const KNet& net, const KInst& inst, int64_t ckpt_per_wave, int Wmax_p,
                       const KTile* tiles, int kind, int wg, int n_tiles,
                       const float* __restrict__ s, const float* __restrict__ mu,
                       const SmemWS& sm) {
  constexpr bool JET = NJ == 4;
  constexpr int NC = JET ? 1 : NJ;              // points per lane
  constexpr int RGM = RP / 4;
  constexpr int NG = 4 / NJ;                    // 4-neuron groups per step
  constexpr int64_t kSlot = 4 * RGM * 64 * 4;  // floats per checkpoint slot
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 3;
  const int trip = wave & 3, role = wave >> 2;  // 0: M1, 1: M2, 2: S0, 3: S1
  const int L = net.L;
  const int Wm = Wmax_p;

  // ---- the lane's points (the four waves of a tile own the same points) ----
  float x[NC], t[NC];
  bool valid[NC], tile_ok[NC];
  int64_t p[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int u = wg * NC + c;
    tile_ok[c] = u < n_tiles;
    x[c] = 0.f;
    t[c] = 0.f;
    if (kind == 0) {
      p[c] = (int64_t)u * kPtsPerWG + trip * 64 + lane;
      valid[c] = p[c] < inst.n_r;
      if (valid[c]) {
        x[c] = inst.xt_r[2 * p[c]];
        t[c] = inst.xt_r[2 * p[c] + 1];
      }
    } else if (kind == 1) {
      p[c] = (int64_t)u * kPtsPerWG + trip * 64 + lane;
      valid[c] = p[c] < inst.n_0;
      if (valid[c]) x[c] = inst.x_0[p[c]];
    } else {
      p[c] = (int64_t)u * kBcPairsPerWG + trip * 32 + (lane >> 1);
      valid[c] = p[c] < inst.n_b;
      x[c] = (lane & 1) ? LRNR_TWO_PI_F : 0.f;
      if (valid[c]) t[c] = inst.t_b[p[c]];
    }
  }
  float* ckbase = tiles[0].ck + trip * ckpt_per_wave;
  float* xa = sm.xa + trip * 2 * kXFloats;
  float* xz = sm.xz + trip * 2 * kXFloats;
  float* xg = sm.xg + trip * 2 * kXFloats;
  float amax = 0.f;
  // M1: s * y^l;  M2: y^{l+1} (forward), ybar^{l+1} (reverse);  S1: wbar (reverse)
  f4 y[NJ][RGM];

  // ---- forward sweep ----------------------------------------------------------
  // Layer 1 is staged here; every later layer by waves 0-3 and 8-15 while M2
  // stores the layer's output, which it also hands to M1 through the tile's
  // exchange slots (the global checkpoint is for the reverse sweep).
  __syncthreads();
  stage_layer<kWsThreads>(net, s, 1, 4, L - 1 == 1 ? 4 : RP, sm.Us, sm.Vs, sm.bs, sm.ss + RP);
  for (int l = 1; l <= L - 1; ++l) {
    const bool first = l == 1, last = l == L - 1;
    const int Gs = (((net.M[l] + 3) & ~3) / 4 + NG - 1) / NG;
    __syncthreads();
    if (role == 0) {
      if (first) {
        if constexpr (JET)
          input_jets<NJ, RGM>(net, x[0], t[0], y);
        else
          input_vals<NC, RGM>(net, x, t, y);
      } else {
        yx_get<NJ, RGM>(xa, xz, xg, lane, y);
      }
      const int RGI = first ? 1 : RGM;
#pragma unroll
      for (int g = 0; g < RGM; ++g) {
        if (g < RGI) {
          const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + (l & 1) * RP + 4 * g);
#pragma unroll
          for (int c = 0; c < NJ; ++c) y[c][g] *= s4;
        }
      }
      if (first)
        m1_loop<NJ, RGM, 1, NG, 2>(sm, xa, Gs, Gs + 2, li, lane, y);
      else
        m1_loop<NJ, RGM, RGM, NG>(sm, xa, Gs, Gs + 2, li, lane, y);
    } else if (role >= 2) {
      s_fwd_loop<NJ, NG>(xa, xz, Gs, lane, role - 2, amax);
    } else {
#pragma unroll
      for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int g = 0; g < RGM; ++g) y[c][g] = zero4();
      if (last)
        m2_fwd_loop<NJ, RGM, 1, NG>(sm, xz, Gs, li, lane, y);
      else
        m2_fwd_loop<NJ, RGM, RGM, NG>(sm, xz, Gs, li, lane, y);
      if (!last) {
        ckpt_store<NJ, RGM>(ckbase + (l - 1) * kSlot, lane, y);
        yx_put<NJ, RGM>(xa, xz, xg, lane, y);
      }
    }
    // the loops of this layer are over: the next layer's factors go to LDS
    // (threads of waves 0-3 and 8-15 numbered 0..767)
    if (!last && role != 1)
      stage_layer<kWsThreads - 256>(net, s, l + 1, RP, l + 1 == L - 1 ? 4 : RP, sm.Us, sm.Vs,
                                    sm.bs, sm.ss + ((l + 1) & 1) * RP,
                                    role == 0 ? tid : tid - 256);
  }

  // ---- output layer, residual and loss adjoints (M2) --------------------------
  const float UL = net.U[net.offU[L]];
  const float sL = s[net.offS[L]];
  const float bL = net.b[net.offB[L]];
  const float cL = UL * sL;
  const int comp = sum4_component(lane);
  if (role == 1) {
    float u[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) u[c] = cL * y[c][0][0];
    if constexpr (JET) {
      u[0] += bL;
    } else {
#pragma unroll
      for (int c = 0; c < NJ; ++c) u[c] += bL;
    }
    const int form = inst.form;
    float lsum[NC];
    float ub[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) ub[c] = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) lsum[c] = 0.f;
    if constexpr (VJP) {
      // cotangent of the jets supplied by the caller (interior points only)
      if (valid[0]) {
        const int64_t n = inst.n_r;
#pragma unroll
        for (int c = 0; c < NJ; ++c) ub[c] = inst.cot[c * n + p[0]];
      }
    } else if constexpr (JET) {
      const float beta = mu[0], nu = mu[1], rho = mu[2];
      const float res = u[2] + beta * u[1] - nu * u[3] - rho * u[0] * (1.f - u[0]);
      const float phi = form == 0 ? res * res : fabsf(res);
      const float dphi = form == 0 ? 2.f * res : (res > 0.f ? 1.f : (res < 0.f ? -1.f : 0.f));
      const float g = valid[0] ? inst.wr_n * dphi : 0.f;
      lsum[0] = valid[0] ? phi : 0.f;
      ub[0] = -rho * (1.f - 2.f * u[0]) * g;
      ub[1] = beta * g;
      ub[2] = g;
      ub[3] = -nu * g;
    } else if (kind == 1) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float e0 = u[c] - sinf(x[c]);
        const float phi = form == 0 ? e0 * e0 : fabsf(e0);
        const float dphi = form == 0 ? 2.f * e0 : (e0 > 0.f ? 1.f : (e0 < 0.f ? -1.f : 0.f));
        lsum[c] = valid[c] ? phi : 0.f;
        ub[c] = valid[c] ? inst.w0_n * dphi : 0.f;
      }
    } else {
      const bool right = lane & 1;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float other = __shfl_xor(u[c], 1);
        const float eb = right ? other - u[c] : u[c] - other;
        const float phi = form == 0 ? eb * eb : fabsf(eb);
        const float dphi = form == 0 ? 2.f * eb : (eb > 0.f ? 1.f : (eb < 0.f ? -1.f : 0.f));
        lsum[c] = (valid[c] && !right) ? phi : 0.f;
        ub[c] = valid[c] ? (right ? -inst.wb_n : inst.wb_n) * dphi : 0.f;
      }
    }
    if constexpr (JET) {
      float sLb = 0.f;
#pragma unroll
      for (int c = 0; c < NJ; ++c) sLb += ub[c] * y[c][0][0];
      const float tot = wave_sum4(f4{lsum[0], UL * sLb, ub[0], 0.f}, lane);
      if ((lane & 15) == 0) sm.lw[trip * 4 + comp] = tot;
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float tot = wave_sum4(f4{lsum[c], UL * (ub[c] * y[c][0][0]), ub[c], 0.f}, lane);
        if ((lane & 15) == 0) sm.lw[16 * c + trip * 4 + comp] = tot;
      }
    }
    // ybar^L for the reverse sweep of the last hidden layer
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
#pragma unroll
      for (int g = 0; g < RGM; ++g) y[c][g] = zero4();
      y[c][0] = f4{cL * ub[c], 0.f, 0.f, 0.f};
    }
  }

  // ---- reverse sweep -----------------------------------------------------------
  // Layer L-1 is still staged from the forward sweep.  Every later layer is staged by waves 0-11 while S1 finishes
  // the ds term of the layer before (s^l, which that term still reads, after
  // the following barrier); S1 hands ybar^l to the next layer's M2 through
  // the tile's exchange slots.
  __syncthreads();
  {
    if (tid < 4 * NC) {
      const int c = tid >> 2, e = tid & 3;
      const float* lw = sm.lw + 16 * c;
      const float v = ((lw[e] + lw[4 + e]) + lw[8 + e]) + lw[12 + e];
      float* rec = tiles[c].rec;
      if (tile_ok[c]) {
        if (e == 0) {
          rec[0] = kind == 0 ? v : 0.f;
          rec[1] = kind == 1 ? v : 0.f;
          rec[2] = kind == 2 ? v : 0.f;
          rec[3] = 0.f;
        } else if (e == 1) {
          rec[4 + net.offS[L]] = v;
        } else if (e == 2) {
          rec[4 + net.r_total + net.offB[L]] = v;
        }
      }
    }
  }
  for (int l = L - 1; l >= 1; --l) {
    const bool first = l == 1, last = l == L - 1;
    const int Gs = (((net.M[l] + 3) & ~3) / 4 + NG - 1) / NG;
    __syncthreads();
    if (role == 0) {
      if (first) {
        if constexpr (JET)
          input_jets<NJ, RGM>(net, x[0], t[0], y);
        else
          input_vals<NC, RGM>(net, x, t, y);
      } else {
        ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
      }
      const int RGI = first ? 1 : RGM;
#pragma unroll
      for (int g = 0; g < RGM; ++g) {
        if (g < RGI) {
          const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + (l & 1) * RP + 4 * g);
#pragma unroll
          for (int c = 0; c < NJ; ++c) y[c][g] *= s4;
        }
      }
      if (first)
        m1_loop<NJ, RGM, 1, NG, 2>(sm, xa, Gs, Gs + 2, li, lane, y);
      else
        m1_loop<NJ, RGM, RGM, NG>(sm, xa, Gs, Gs + 2, li, lane, y);
    } else if (role == 1) {
      // wbar^{l+1} from S1 at the end of layer l+1, through the exchange
      // slots; ybar^{l+1} = s^{l+1} * wbar^{l+1} (s^{l+1} is in the other
      // s buffer)
      if (!last) {
        yx_get<NJ, RGM>(xa, xz, xg, lane, y);
#pragma unroll
        for (int g = 0; g < RGM; ++g) {
          const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + ((l + 1) & 1) * RP + 4 * g);
#pragma unroll
          for (int c = 0; c < NJ; ++c) y[c][g] = s4 * y[c][g];
        }
      }
      if (last)
        m2_bwd_loop<NJ, RGM, 1, NG>(sm, xz, Gs, li, lane, y);
      else
        m2_bwd_loop<NJ, RGM, RGM, NG>(sm, xz, Gs, li, lane, y);
    } else if (role == 2) {
      s0_bwd_loop<NJ, NG>(xa, xz, xg, Gs, lane, sm.bbar + trip * Wm, 4 * Wm, amax);
    } else {
#pragma unroll
      for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int g = 0; g < RGM; ++g) y[c][g] = zero4();
      if (first)
        s1_bwd_loop<NJ, RGM, 1, NG>(sm, xg, Gs, li, lane, y);
      else
        s1_bwd_loop<NJ, RGM, RGM, NG>(sm, xg, Gs, li, lane, y);
      // dL/ds^l = sum_c wbar_c * y_c^l over the jets of a point (per column
      // for value tiles), one rank group at a time.  Above the input layer
      // wbar^l first goes to the next layer's M2 through the exchange slots,
      // which frees its registers for y^l, read in one round trip; wbar is
      // read back from LDS group by group.
      if (first) {
        f4 yl[NJ];
        if constexpr (JET)
          input_jets_g0<NJ>(net, x[0], t[0], yl);
        else
          input_vals_g0<NC>(net, x, t, yl);
        if constexpr (JET) {
          f4 acc = zero4();
#pragma unroll
          for (int c = 0; c < NJ; ++c) acc += y[c][0] * yl[c];
          const float tot = wave_sum4(acc, lane);
          if ((lane & 15) == 0) sm.sbar[trip * RP + comp] = tot;
        } else {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const float tot = wave_sum4(y[c][0] * yl[c], lane);
            if ((lane & 15) == 0) sm.sbar[c * 4 * RP + trip * RP + comp] = tot;
          }
        }
      } else {
        yx_put<NJ, RGM>(xa, xz, xg, lane, y);
        ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
#pragma unroll
        for (int g = 0; g < RGM; ++g) {
          f4 wg[NJ];
          yx_get_g<NJ, RGM>(xa, xz, xg, lane, g, wg);
          if constexpr (JET) {
            f4 acc = zero4();
#pragma unroll
            for (int c = 0; c < NJ; ++c) acc += wg[c] * y[c][g];
            const float tot = wave_sum4(acc, lane);
            if ((lane & 15) == 0) sm.sbar[trip * RP + 4 * g + comp] = tot;
          } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const float tot = wave_sum4(wg[c] * y[c][g], lane);
              if ((lane & 15) == 0) sm.sbar[c * 4 * RP + trip * RP + 4 * g + comp] = tot;
            }
          }
        }
      }
    }
    // waves 0-11: U^{l-1}, V^l and b^{l-1} of the next layer (this layer's
    // loops are over, and S1's ds term reads only the checkpoints and the
    // exchange slots)
    if (role != 3 && !first)
      stage_layer<kWsThreads - 256>(net, s, l - 1, l - 1 == 1 ? 4 : RP, RP, sm.Us, sm.Vs,
                                    sm.bs, nullptr);
    __syncthreads();
    if (!first) {
      const int KIn = l - 1 == 1 ? 4 : RP, rn = net.r[l - 1];
      float* ssn = sm.ss + ((l - 1) & 1) * RP;
      for (int i = tid; i < KIn; i += kWsThreads) ssn[i] = i < rn ? s[net.offS[l - 1] + i] : 0.f;
    }
    const int W = net.M[l], rl = net.r[l];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!tile_ok[c]) continue;
      float* rec = tiles[c].rec;
      const float* bb = sm.bbar + c * 4 * Wm;
      const float* sb = sm.sbar + c * 4 * RP;
      for (int i = tid; i < W; i += kWsThreads)
        rec[4 + net.r_total + net.offB[l] + i] =
            ((bb[i] + bb[Wm + i]) + bb[2 * Wm + i]) + bb[3 * Wm + i];
      for (int i = tid; i < rl; i += kWsThreads)
        rec[4 + net.offS[l] + i] = ((sb[i] + sb[RP + i]) + sb[2 * RP + i]) + sb[3 * RP + i];
    }
  }
  // flag the tiles for the accurate relaunch if any lane met |a| > kFastRange
  const bool bad = __any(!(amax <= kFastRange));
  __syncthreads();
  if (lane == 0) sm.lw[16 * kMaxCols + wave] = bad ? 1.f : 0.f;
  __syncthreads();
  if (tid == 0) {
    float any = 0.f;
    for (int w = 0; w < kWsWaves; ++w) any += sm.lw[16 * kMaxCols + w];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (tile_ok[c]) *tiles[c].flag = any > 0.f ? 1 : 0;
  }
}

// Value-only tiles of the plain gradient kernel take NCV points per lane (NCV
// tiles per workgroup).  With two, every factor entry read from LDS feeds two
// MFMAs and the IC/BC workgroups are half as many, but each takes longer: it
// pays when the value tiles outnumber the CUs (they would otherwise run in
// more than one round after the interior ones), and one column is faster
// when they fit in a single round.
__host__ __device__ inline int ws_value_wgs(int G, int ncv) { return (G + ncv - 1) / ncv; }
__host__ __device__ inline int ws_grid_inst(const KGrid& g, int ncv) {
  return g.G_r + ws_value_wgs(g.G_0, ncv) + ws_value_wgs(g.G_b, ncv);
}

template <int RP, int NCV>
__global__ __launch_bounds__(kWsThreads) void lrnr_grad_ws_kernel(KNet net, KInst inst,
                                                                  KGrid grid) {
  extern __shared__ float4 smem_raw[];
  const SmemWS sm = ws_smem(reinterpret_cast<float*>(smem_raw), grid.Wmax_p, RP);

  const int g0 = ws_value_wgs(grid.G_0, NCV);
  const int per_inst = grid.G_r + g0 + ws_value_wgs(grid.G_b, NCV);
  const int inst_id = blockIdx.x / per_inst;
  int wg = blockIdx.x - inst_id * per_inst;
  int kind = 0;
  if (wg >= grid.G_r + g0) {
    kind = 2;
    wg -= grid.G_r + g0;
  } else if (wg >= grid.G_r) {
    kind = 1;
    wg -= grid.G_r;
  }
  const float* s = inst.s + inst_id * grid.s_stride;
  const float* mu = inst.mu ? inst.mu + 3 * inst_id : nullptr;
  // records and flags are per tile of the full grid (G_inst per instance)
  const int64_t first = (int64_t)inst_id * grid.G_inst +
                        (kind == 0 ? 0 : kind == 1 ? grid.G_r : grid.G_r + grid.G_0);
  float* ck = grid.ckpt + (int64_t)blockIdx.x * kWaves * grid.ckpt_per_wave;
  if (kind == 0) {
    KTile tile;
    tile.rec = grid.partials + (first + wg) * grid.P;
    tile.ck = ck;
    tile.flag = grid.flags + first + wg;
    ws_run<RP, 4, false>(net, inst, grid.ckpt_per_wave, grid.Wmax_p, &tile, 0, wg, grid.G_r, s,
                         mu, sm);
  } else {
    KTile tiles[NCV];
#pragma unroll
    for (int c = 0; c < NCV; ++c) {
      const int64_t u = first + (int64_t)wg * NCV + c;
      tiles[c].rec = grid.partials + u * grid.P;
      tiles[c].ck = ck;
      tiles[c].flag = grid.flags + u;
    }
    ws_run<RP, NCV, false>(net, inst, grid.ckpt_per_wave, grid.Wmax_p, tiles, kind, wg,
                           kind == 1 ? grid.G_0 : grid.G_b, s, mu, sm);
  }
}

// Rank tiles above this run the single-role kernel for the reverse modes:
// four jets of 24 or 32 ranks per role do not fit four waves per SIMD (at
// rank 20 a few long-lived values are spilled outside the MFMA loops).
constexpr int kWsMaxRP = 20;

// Which kernel runs the reverse modes.  The four-role kernel hides latency
// with four waves per SIMD but pays a workgroup barrier per neuron step; the
// single-role kernel (one wave owns its points through the whole layer, no
// per-step barrier) runs two waves per SIMD up to rank tile 8 and one above.
// Measured on the MI355X (loss + gradient, 4 hidden layers, 65536 points,
// widths 32-256): the single-role kernel is faster at rank tiles 4 and 8 at
// every width (by 22-31 % at widths 128-256), and at rank tile 16 only while
// Wmax_p * RP <= 512; the four-role kernel is faster above that (by 5-27 %).
template <int RP>
inline bool four_role(int Wmax_p) {
  if constexpr (RP > kWsMaxRP)
    return false;
  else
    return RP > 8 && Wmax_p * RP > 512;
}

// ---------------------------------------------------------------------------
// Task-table launches: a persistent grid strides over the tiles of all tasks.
// ---------------------------------------------------------------------------

// The task owning a tile: the largest t with start[t] <= tile (start is
// non-decreasing, so the ballot of start[i] <= tile is a prefix of the lanes).
__device__ __forceinline__ int find_task(const int* __restrict__ start, int n_tasks, int tile) {
  const int lane = threadIdx.x & 63;
  int t = 0;
  for (int c = 0; c < n_tasks; c += 64) {
    const int i = c + lane;
    const bool le = i < n_tasks && start[i] <= tile;
    const int cnt = __popcll(__ballot(le));
    if (cnt > 0) t = c + cnt - 1;
    if (cnt < 64) break;
  }
  return __builtin_amdgcn_readfirstlane(t);
}

struct TileRef {
  const KTask* task;
  int kind, wg, local;
};

__device__ __forceinline__ TileRef decode_tile(const KTableGrid& tg, int n_tasks, int tile) {
  const int* start = reinterpret_cast<const int*>(tg.table + sizeof(KTableHdr));
  const int t = find_task(start, n_tasks, tile);
  TileRef r;
  r.task = reinterpret_cast<const KTask*>(tg.table + tg.off_tasks) + t;
  r.local = tile - start[t];
  r.wg = r.local;
  r.kind = 0;
  const int Gr = r.task->G_r, G0 = r.task->G_0;
  if (r.wg >= Gr + G0) {
    r.kind = 2;
    r.wg -= Gr + G0;
  } else if (r.wg >= Gr) {
    r.kind = 1;
    r.wg -= Gr;
  }
  return r;
}

// A task whose Adam counter reached its limit is finished: its tiles are skipped.
__device__ __forceinline__ bool task_finished(const KTask* T) {
  return T->step != nullptr && T->steps_max > 0 && *T->step >= T->steps_max;
}

template <int RP, bool VJP>
__global__ __launch_bounds__(kWsThreads) void lrnr_grad_ws_table_kernel(KTableGrid tg) {
  extern __shared__ float4 smem_raw[];
  const SmemWS sm = ws_smem(reinterpret_cast<float*>(smem_raw), tg.Wmax_p, RP);
  const KTableHdr* hdr = reinterpret_cast<const KTableHdr*>(tg.table);
  const int n_tasks = hdr->n_tasks, n_tiles = hdr->n_tiles;
  float* ck = tg.ckpt + (int64_t)blockIdx.x * kWaves * tg.ckpt_per_wave;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const TileRef r = decode_tile(tg, n_tasks, tile);
    const KTask* T = r.task;
    if (task_finished(T)) continue;
    KTile kt;
    kt.rec = tg.partials + T->rec0 + (int64_t)r.local * T->P;
    kt.ck = ck;
    kt.flag = tg.flags + tile;
    if (r.kind == 0)
      ws_run<RP, 4, VJP>(T->net, T->inst, tg.ckpt_per_wave, tg.Wmax_p, &kt, 0, r.wg, r.wg + 1,
                         T->inst.s, T->inst.mu, sm);
    else if constexpr (!VJP)
      ws_run<RP, 1, false>(T->net, T->inst, tg.ckpt_per_wave, tg.Wmax_p, &kt, r.kind, r.wg,
                           r.wg + 1, T->inst.s, T->inst.mu, sm);
    __syncthreads();
  }
}

template <int RP, int MODE, int SC>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(fused_waves_per_simd<RP, MODE, true>()))) void lrnr_table_kernel(
    KTableGrid tg) {
  extern __shared__ float4 smem_raw[];
  const Smem sm = make_smem(reinterpret_cast<float*>(smem_raw), tg.Wmax_p, RP, tg.res_layers);
  const KTableHdr* hdr = reinterpret_cast<const KTableHdr*>(tg.table);
  const int n_tasks = hdr->n_tasks, n_tiles = hdr->n_tiles;
  float* ck = tg.ckpt ? tg.ckpt + (int64_t)blockIdx.x * kWaves * tg.ckpt_per_wave : nullptr;
  int staged = -1;  // net_id whose factors the resident slabs hold
  auto run_tile = [&](int tile) {
    const TileRef r = decode_tile(tg, n_tasks, tile);
    const KTask* T = r.task;
    if constexpr (reverse_mode(MODE))
      if (task_finished(T)) return;
    KTile kt;
    kt.rec = tg.partials ? tg.partials + T->rec0 + (int64_t)r.local * T->P : nullptr;
    kt.ck = ck;
    kt.flag = tg.flags ? tg.flags + tile : nullptr;
    kt.stage_net = T->net_id != staged || T->net_id < 0;
    staged = T->net_id;
    run_kind<RP, MODE, SC, true>(T->net, T->inst, tg.ckpt_per_wave, tg.Wmax_p, kt, r.kind, r.wg,
                                 T->inst.s, T->inst.mu, sm);
    __syncthreads();
  };
  if constexpr (SC == SC_ACC) {
    // only the tiles the fast pass flagged: a workgroup tests kThreads flags
    // at once, so a launch with nothing flagged is one pass per workgroup
    for (int base = blockIdx.x * kThreads; base < n_tiles; base += gridDim.x * kThreads) {
      const int t = base + (int)threadIdx.x;
      if (!__syncthreads_or(t < n_tiles && tg.flags[t] != 0)) continue;
      const int end = min(base + kThreads, n_tiles);
      for (int tile = base; tile < end; ++tile)
        if (tg.flags[tile] != 0) run_tile(tile);
    }
  } else {
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) run_tile(tile);
  }
}

// Raises a kernel's dynamic-LDS limit once per kernel and size (so that
// launches recorded into a graph make no attribute calls after the first).
template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  std::lock_guard<std::mutex> lock(mu);
  const void* key = (const void*)kernel;
  auto it = done.find(key);
  if (it != done.end() && it->second >= lds) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) done[key] = lds;
  return e;
}

// Compute units of the current device (cached per device).
static int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cus;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cus.find(dev);
  if (it != cus.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
    n = 256;
  cus[dev] = n;
  return n;
}

template <typename K>
static int resident_grid(K kernel, int threads, size_t lds) {
  if (set_lds(kernel, lds) != hipSuccess) return -1;
  int per_cu = 0, dev = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kernel, threads, lds) !=
      hipSuccess)
    return -1;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return -1;
  return std::max(1, per_cu) * prop.multiProcessorCount;
}

// Resident workgroups of the kernel that does most of a mode's work.
template <int RP>
int table_grid_rp(int mode, int Wmax_p) {
  if (reverse_mode(mode)) {
    if constexpr (RP <= kWsMaxRP) {
      if (four_role<RP>(Wmax_p)) {
        const size_t lds = ws_lds_floats(RP, Wmax_p) * sizeof(float);
        return mode == MODE_VJP
                   ? resident_grid(lrnr_grad_ws_table_kernel<RP, true>, kWsThreads, lds)
                   : resident_grid(lrnr_grad_ws_table_kernel<RP, false>, kWsThreads, lds);
      }
    }
    const size_t lds = fused_lds_bytes(RP, Wmax_p);
    return mode == MODE_VJP
               ? resident_grid(lrnr_table_kernel<RP, MODE_VJP, SC_TRACK>, kThreads, lds)
               : resident_grid(lrnr_table_kernel<RP, MODE_GRAD, SC_TRACK>, kThreads, lds);
  }
  const size_t lds = fused_lds_bytes(RP, Wmax_p);
  switch (mode) {
    case MODE_JETS: return resident_grid(lrnr_table_kernel<RP, MODE_JETS, SC_REDO>, kThreads, lds);
    case MODE_VALUE:
      return resident_grid(lrnr_table_kernel<RP, MODE_VALUE, SC_REDO>, kThreads, lds);
    default: return resident_grid(lrnr_table_kernel<RP, MODE_LOSS, SC_REDO>, kThreads, lds);
  }
}

template <int RP, int MODE, int SC>
static hipError_t launch_table_one(const KTableGrid& tg, int grid, hipStream_t stream) {
  const size_t lds = fused_lds_bytes(RP, tg.Wmax_p, tg.res_layers);
  hipError_t e = set_lds(lrnr_table_kernel<RP, MODE, SC>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((lrnr_table_kernel<RP, MODE, SC>), dim3(grid), dim3(kThreads), lds, stream,
                     tg);
  return hipGetLastError();
}

template <int RP, bool VJP>
static hipError_t launch_table_rev(const KTableGrid& tg, int grid, hipStream_t stream) {
  constexpr int MODE = VJP ? MODE_VJP : MODE_GRAD;
  if constexpr (RP <= kWsMaxRP) {
    if (four_role<RP>(tg.Wmax_p)) {
      const size_t lds = ws_lds_floats(RP, tg.Wmax_p) * sizeof(float);
      hipError_t e = set_lds(lrnr_grad_ws_table_kernel<RP, VJP>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((lrnr_grad_ws_table_kernel<RP, VJP>), dim3(grid), dim3(kWsThreads), lds,
                         stream, tg);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      // tiles that met |a| > kFastRange are recomputed with ocml's sin/cos
      return launch_table_one<RP, MODE, SC_ACC>(tg, grid, stream);
    }
  }
  hipError_t e = launch_table_one<RP, MODE, SC_TRACK>(tg, grid, stream);
  if (e != hipSuccess) return e;
  return launch_table_one<RP, MODE, SC_ACC>(tg, grid, stream);
}

// grid: persistent workgroups; the checkpoint slab holds grid * kWaves slabs.
template <int RP>
hipError_t launch_table_rp(int mode, const KTableGrid& tg, int grid, hipStream_t stream) {
  switch (mode) {
    case MODE_JETS: return launch_table_one<RP, MODE_JETS, SC_REDO>(tg, grid, stream);
    case MODE_VALUE: return launch_table_one<RP, MODE_VALUE, SC_REDO>(tg, grid, stream);
    case MODE_LOSS: return launch_table_one<RP, MODE_LOSS, SC_REDO>(tg, grid, stream);
    case MODE_VJP: return launch_table_rev<RP, true>(tg, grid, stream);
    default: return launch_table_rev<RP, false>(tg, grid, stream);
  }
}

template <int RP>
hipError_t launch_grad_ws(const KNet& net, const KInst& inst, const KGrid& grid,
                          hipStream_t stream) {
  bool ws = false;
  if constexpr (RP <= kWsMaxRP) ws = four_role<RP>(grid.Wmax_p);
  if (!ws) {
    if constexpr (RP <= 8) {
      if ((int64_t)grid.B * grid.G_inst > 2 * (int64_t)device_cus()) {
        // more workgroups than two per CU: three waves per SIMD, as in the
        // task tables (fast pass, then the flagged workgroups recomputed)
        hipError_t e = launch_one<RP, MODE_GRAD, SC_TRACK, true>(net, inst, grid, stream);
        if (e != hipSuccess) return e;
        return launch_one<RP, MODE_GRAD, SC_ACC>(net, inst, grid, stream);
      }
      // a wave that meets |a| > kFastRange redoes that layer pass with
      // ocml's sin/cos at once: no relaunch of flagged workgroups
      return launch_one<RP, MODE_GRAD, SC_REDO>(net, inst, grid, stream);
    }
    hipError_t e = launch_one<RP, MODE_GRAD, SC_TRACK>(net, inst, grid, stream);
    if (e != hipSuccess) return e;
    return launch_one<RP, MODE_GRAD, SC_ACC>(net, inst, grid, stream);
  }
  if constexpr (RP <= kWsMaxRP) {
    const int64_t value_tiles = (int64_t)grid.B * (grid.G_0 + grid.G_b);
    const bool two = value_tiles > device_cus();
    const dim3 blocks((unsigned)(grid.B * ws_grid_inst(grid, two ? 2 : 1))), threads(kWsThreads);
    const size_t lds = ws_lds_floats(RP, grid.Wmax_p) * sizeof(float);
    hipError_t e;
    if (two) {
      e = set_lds(lrnr_grad_ws_kernel<RP, 2>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((lrnr_grad_ws_kernel<RP, 2>), blocks, threads, lds, stream, net, inst,
                         grid);
    } else {
      e = set_lds(lrnr_grad_ws_kernel<RP, 1>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((lrnr_grad_ws_kernel<RP, 1>), blocks, threads, lds, stream, net, inst,
                         grid);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // workgroups that met |a| > kFastRange are recomputed with ocml's sin/cos
    return launch_one<RP, MODE_GRAD, SC_ACC>(net, inst, grid, stream);
  }
  return hipSuccess;
}

template <int RP>
hipError_t launch_rp(int mode, const KNet& net, const KInst& inst, const KGrid& grid,
                     hipStream_t stream) {
  switch (mode) {
    case MODE_JETS: return launch_one<RP, MODE_JETS, SC_REDO>(net, inst, grid, stream);
    case MODE_VALUE: return launch_one<RP, MODE_VALUE, SC_REDO>(net, inst, grid, stream);
    case MODE_LOSS: return launch_one<RP, MODE_LOSS, SC_REDO>(net, inst, grid, stream);
    default: return launch_grad_ws<RP>(net, inst, grid, stream);
  }
}

}  // namespace lrnr
