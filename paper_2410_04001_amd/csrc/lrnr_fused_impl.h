// Fused LRNR / FastLRNR kernel for gfx950: forward jets, CDR residual loss and
// reverse sweep to s and b (arXiv 2410.04001: eq. 2.1-2.2 for the chain, eq. 2.8
// for the reduced chain, eq. 3.5-3.7 for the loss, eq. 4.1 for the residual).
//
// Work mapping.  One lane owns one collocation point for the whole chain, and
// keeps the point's jets (value, d/dx, d/dt, d2/dx2) in registers.  Every
// contraction is a v_mfma_f32_4x4x1_16b_f32 whose 16 blocks of 4 columns are
// the 64 lanes of the wave, so the MFMA result of lane p is always point p:
//
//  * U side, a_c[p][w0+i] += (U diag(s))[w0+i][k] * y_c[p][k]: A operand lane
//    4b+i holds (U diag(s))[w0+i][k] (a row staged in LDS), B operand lane p
//    its own y[k]; accumulator GPR i holds neuron w0+i.
//  * V side, y'_c[p][4g+i] += V[w][4g+i] * z_c[p][w]: A operand is a 4-rank
//    slice of row w of V, B operand is z of the lane's own point; accumulator
//    GPR i holds rank 4g+i.
//
// The reduced coordinates y^l = V^lT z^{l-1} (r_l floats per jet) are the only
// per-point state carried between layers; in the gradient mode they are
// checkpointed to global scratch in the forward sweep and the W-wide
// activations are recomputed in the reverse sweep.  The factors are staged
// into LDS (zero-padded to 4-aligned widths and the compiled rank tile RP),
// every hidden layer at once when they fit, else one layer at a time, which
// lets the same code run the full LRNR (width M_l) and the FastLRNR (width
// r_hat_l).
#pragma once

#include "lrnr_internal.h"

namespace lrnr {

typedef float f4 __attribute__((ext_vector_type(4)));

#define LRNR_TWO_PI_F 6.28318530717958647692f

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 zero4() { return f4{0.f, 0.f, 0.f, 0.f}; }

// ---------------------------------------------------------------------------
// sin and cos of one argument, branch-free.  Cody & Waite reduction by pi/2
// split into three FP32 parts (P1 = fl(pi/2), P2 = fl(pi/2 - P1),
// P3 = fl(pi/2 - P1 - P2)), applied with fused multiply-adds, then the Taylor
// polynomials of sin (to degree 11) and cos (to degree 10) on [-pi/4, pi/4],
// whose truncation errors there are below 1e-10.  Absolute error below 7.1e-8
// for |x| <= kFastRange; larger arguments take ocml's sincosf (sin/cos policy
// below).
// ---------------------------------------------------------------------------
constexpr float kFastRange = 1.0e6f;
constexpr float kTwoOverPi = 0.63661974668502807617f;
constexpr float kP1 = 1.57079637050628662109f;
constexpr float kP2 = -4.37113882867379300296e-08f;
constexpr float kP3 = -1.71512451000588191836e-15f;
constexpr float kS3 = -1.0f / 6.0f, kS5 = 1.0f / 120.0f, kS7 = -1.0f / 5040.0f;
constexpr float kS9 = 1.0f / 362880.0f, kS11 = -1.0f / 39916800.0f;
constexpr float kC2 = -0.5f, kC4 = 1.0f / 24.0f, kC6 = -1.0f / 720.0f;
constexpr float kC8 = 1.0f / 40320.0f, kC10 = -1.0f / 3628800.0f;

__device__ __forceinline__ void sincos_fast(float x, float& s, float& c) {
  const float k = __builtin_rintf(x * kTwoOverPi);
  float r = __builtin_fmaf(-k, kP1, x);
  r = __builtin_fmaf(-k, kP2, r);
  r = __builtin_fmaf(-k, kP3, r);
  const float r2 = r * r;
  float ps = __builtin_fmaf(r2, kS11, kS9);
  ps = __builtin_fmaf(r2, ps, kS7);
  ps = __builtin_fmaf(r2, ps, kS5);
  ps = __builtin_fmaf(r2, ps, kS3);
  const float sn = __builtin_fmaf(r2 * r, ps, r);
  float pc = __builtin_fmaf(r2, kC10, kC8);
  pc = __builtin_fmaf(r2, pc, kC6);
  pc = __builtin_fmaf(r2, pc, kC4);
  pc = __builtin_fmaf(r2, pc, kC2);
  const float cs = __builtin_fmaf(r2, pc, 1.0f);
  const int q = (int)k;  // quadrant; two's complement bits give q mod 4
  const float a = (q & 1) ? cs : sn;
  const float b = (q & 1) ? sn : cs;
  s = (q & 2) ? -a : a;
  c = ((q + 1) & 2) ? -b : b;
}

template <bool ACC>
__device__ __forceinline__ void sincos_sel(float x, float& s, float& c) {
  if constexpr (ACC)
    sincosf(x, &s, &c);
  else
    sincos_fast(x, s, c);
}

// How a kernel instance evaluates sin/cos:
//  SC_REDO  fast path; a wave that met |a| > kFastRange redoes the layer with
//           ocml's sincosf (forward-only modes, where registers are plentiful);
//  SC_TRACK fast path only; the largest |a| is tracked and reported so that a
//           following SC_ACC launch recomputes the flagged workgroups;
//  SC_ACC   ocml's sincosf throughout.
enum SinCos { SC_REDO = 0, SC_TRACK = 1, SC_ACC = 2 };

// ---------------------------------------------------------------------------
// Wave reduction of four values per lane.  Lanes 32-63 of one value swap with
// lanes 0-31 of another (v_permlane32_swap), then odd 16-lane rows with even
// rows (v_permlane16_swap), then a row sum by DPP row rotations.  On return
// every lane of 16-lane row q holds the 64-lane total of component
// sum4_component(16 q).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum4(f4 v, int /*lane*/) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[0]), __float_as_uint(v[1]),
                                                  false, false);
  const float t01 = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2]), __float_as_uint(v[3]),
                                                  false, false);
  const float t23 = __uint_as_float(q[0]) + __uint_as_float(q[1]);
  const auto w = __builtin_amdgcn_permlane16_swap(__float_as_uint(t01), __float_as_uint(t23),
                                                  false, false);
  float x = __uint_as_float(w[0]) + __uint_as_float(w[1]);
  x += dpp_mov<0x128>(x);  // row_ror:8
  x += dpp_mov<0x124>(x);  // row_ror:4
  x += dpp_mov<0x122>(x);  // row_ror:2
  x += dpp_mov<0x121>(x);  // row_ror:1
  return x;
}

__device__ __forceinline__ int sum4_component(int lane) {
  return ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1);
}

// ---------------------------------------------------------------------------
// Contraction pieces for one group of four neurons w0..w0+3.  In every MFMA
// the B operand is the lane's own point value, the A operand a 4-vector of
// factor entries broadcast from LDS.
// ---------------------------------------------------------------------------

// The factor entries of one group are read from LDS into registers before
// any of its MFMAs issue, so that only the first read's latency is exposed
// (reading them one by one between MFMA batches stalls the wave on each).

// Position of a hidden layer in the chain, as flags.  The first hidden layer
// reads y^1 = V^1T (x, t): its rank is at most 2 (the input width), so the
// U-side contraction needs two of the tile's four k, and its d2/dx2 jet is
// zero, so a_xx = 0 and that jet's U^T adjoint is never used (ds^1 weights
// it by y^1_xx = 0, and nothing is propagated below the first layer).  The
// last hidden layer's V side has rank r_L = 1 (a scalar output): one column
// of the 4-wide tile, contracted on the VALU instead of by MFMAs that would
// be three quarters padding.
constexpr int kEdgeFirst = 1, kEdgeLast = 2;

// a_c = U[w0..w0+3] (s*y_c) (+ b for the value jet)
template <int NJ, int RGM, int RGI, int EDGE = 0>
__device__ __forceinline__ void u_side(const float* __restrict__ Us, const float* __restrict__ bs,
                                       int w0, int li, const f4 (&y)[NJ][RGM], f4 (&a)[NJ]) {
  constexpr bool FIRST = EDGE & kEdgeFirst;
  constexpr int KK = FIRST ? 2 : 4;
  constexpr int NJM = FIRST && NJ == 4 ? 3 : NJ;
  constexpr int KI = 4 * RGI;
  const float* urow = Us + (w0 + li) * KI;
  f4 u4[RGI];
#pragma unroll
  for (int g = 0; g < RGI; ++g) u4[g] = *reinterpret_cast<const f4*>(urow + 4 * g);
  a[0] = *reinterpret_cast<const f4*>(bs + w0);
#pragma unroll
  for (int c = 1; c < NJ; ++c) a[c] = zero4();
#pragma unroll
  for (int g = 0; g < RGI; ++g)
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
      for (int c = 0; c < NJM; ++c) a[c] = mfma4(u4[g][kk], y[c][g][kk], a[c]);
}

// yo_c += V[w0..w0+3]^T z_c
template <int NJ, int RGM, int RGO, int EDGE = 0>
__device__ __forceinline__ void v_side(const float* __restrict__ Vs, int w0, int li,
                                       const f4 (&z)[NJ], f4 (&yo)[NJ][RGM]) {
  constexpr int KO = 4 * RGO;
  if constexpr ((EDGE & kEdgeLast) != 0) {
    // rank 1: yo_c[0] += sum_j V[w0+j][0] z_c[j]
    float v0[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v0[j] = Vs[(w0 + j) * KO];
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
      float acc = yo[c][0][0];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc = __builtin_fmaf(v0[j], z[c][j], acc);
      yo[c][0][0] = acc;
    }
    return;
  }
  float v[4][RGO];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int g = 0; g < RGO; ++g) v[j][g] = Vs[(w0 + j) * KO + 4 * g + li];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int g = 0; g < RGO; ++g)
#pragma unroll
      for (int c = 0; c < NJ; ++c) yo[c][g] = mfma4(v[j][g], z[c][j], yo[c][g]);
}

// zb_c = V[w0..w0+3] yb_c
template <int NJ, int RGM, int RGO, int EDGE = 0>
__device__ __forceinline__ void v_rev(const float* __restrict__ Vs, int w0, int li,
                                      const f4 (&yb)[NJ][RGM], f4 (&zb)[NJ]) {
  constexpr int KO = 4 * RGO;
  if constexpr ((EDGE & kEdgeLast) != 0) {
    // rank 1: zb_c[j] = V[w0+j][0] yb_c[0]
    f4 v0;
#pragma unroll
    for (int j = 0; j < 4; ++j) v0[j] = Vs[(w0 + j) * KO];
#pragma unroll
    for (int c = 0; c < NJ; ++c) zb[c] = v0 * yb[c][0][0];
    return;
  }
  const float* vrow = Vs + (w0 + li) * KO;
  f4 v4[RGO];
#pragma unroll
  for (int g = 0; g < RGO; ++g) v4[g] = *reinterpret_cast<const f4*>(vrow + 4 * g);
#pragma unroll
  for (int c = 0; c < NJ; ++c) zb[c] = zero4();
#pragma unroll
  for (int g = 0; g < RGO; ++g)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int c = 0; c < NJ; ++c) zb[c] = mfma4(v4[g][kk], yb[c][g][kk], zb[c]);
}

// wb_c += U[w0..w0+3]^T ab_c (the first layer leaves wb_xx at its zero start)
template <int NJ, int RGM, int RGI, int EDGE = 0>
__device__ __forceinline__ void ut_side(const float* __restrict__ Us, int w0, int li,
                                        const f4 (&ab)[NJ], f4 (&wb)[NJ][RGM]) {
  constexpr int NJM = (EDGE & kEdgeFirst) && NJ == 4 ? 3 : NJ;
  constexpr int KI = 4 * RGI;
  float u[4][RGI];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int g = 0; g < RGI; ++g) u[j][g] = Us[(w0 + j) * KI + 4 * g + li];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int g = 0; g < RGI; ++g)
#pragma unroll
      for (int c = 0; c < NJM; ++c) wb[c][g] = mfma4(u[j][g], ab[c][j], wb[c][g]);
}

// Scheduling hint for a pipelined loop body whose first NM MFMAs do not depend
// on the body's VALU work: pair each with two VALU instructions, so that the
// matrix core and the vector ALU of the (single) wave on a SIMD overlap.
template <int NM>
__device__ __forceinline__ void interleave() {
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
  }
}

// sin and cos of small arguments with the hardware v_sin_f32 / v_cos_f32,
// which take revolutions (valid within +-256): rev = x / (2 pi) as a
// two-term product (1/(2 pi) = kInv2PiHi + kInv2PiLo).  Measured on the
// device against FP64 over 2^26 arguments: absolute error below 4.3e-7 for
// |x| <= kHwRange (1.3e-7 for |x| <= 2), the same maxima as with an explicit
// exact reduction rev - rint(rev) first, which the hardware makes redundant.
constexpr float kHwRange = 8.0f;
constexpr float kInv2PiHi = 0.15915493667125701904f;
constexpr float kInv2PiLo = 6.42063824329852652e-09f;

__device__ __forceinline__ void sincos_hw(float x, float& s, float& c) {
  const float rev = __builtin_fmaf(x, kInv2PiHi, x * kInv2PiLo);
  s = __builtin_amdgcn_sinf(rev);
  c = __builtin_amdgcn_cosf(rev);
}

// Range tracking for the sin/cos path choice uses IEEE maximum (gfx950's
// v_maximum3_f32), not fmaxf: it needs no canonicalising moves of its inputs
// (three VALU instructions per neuron group instead of seven), and a NaN
// pre-activation makes the running maximum NaN, which fails every range test
// and so takes the accurate path (fmaxf would drop it).
__device__ __forceinline__ float vmax(float a, float b) {
  return __builtin_elementwise_maximum(a, b);
}

// sin/cos of the four pre-activations of a neuron group: the hardware path
// when every lane of the wave is within kHwRange (a wave-uniform choice),
// otherwise the Cody-Waite polynomial; ACC selects ocml's sincosf.
template <bool ACC>
__device__ __forceinline__ void sincos4(const f4& a, f4& sn, f4& cs, float& amax) {
  const float m = vmax(vmax(fabsf(a[0]), fabsf(a[1])), vmax(fabsf(a[2]), fabsf(a[3])));
  amax = vmax(amax, m);
  if constexpr (ACC) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float s, c;
      sincosf(a[j], &s, &c);
      sn[j] = s;
      cs[j] = c;
    }
  } else {
    if (__all(m <= kHwRange)) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float s, c;
        sincos_hw(a[j], s, c);
        sn[j] = s;
        cs[j] = c;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float s, c;
        sincos_fast(a[j], s, c);
        sn[j] = s;
        cs[j] = c;
      }
    }
  }
}

// z jets = sin jets of a (value, d/dx, d/dt, d2/dx2); tracks max |a_v|
template <int NJ, bool ACC>
__device__ __forceinline__ void sigma_fwd(const f4 (&a)[NJ], f4 (&z)[NJ], float& amax) {
  f4 sn, cs;
  sincos4<ACC>(a[0], sn, cs, amax);
  z[0] = sn;
  if constexpr (NJ == 4) {
    const f4 ax = a[1];
    z[1] = cs * ax;
    z[2] = cs * a[2];
    z[3] = cs * a[3] - sn * ax * ax;
  }
}

// adjoints of the a jets from those of the z jets
template <int NJ, bool ACC>
__device__ __forceinline__ void sigma_bwd(const f4 (&a)[NJ], const f4 (&zb)[NJ], f4 (&ab)[NJ],
                                          float& amax) {
  f4 sn, cs;
  sincos4<ACC>(a[0], sn, cs, amax);
  if constexpr (NJ == 4) {
    const f4 ax = a[1], at = a[2], axx = a[3];
    const f4 zv = zb[0], zx = zb[1], zt = zb[2], zxx = zb[3];
    ab[3] = cs * zxx;
    ab[2] = cs * zt;
    ab[1] = cs * zx - 2.f * sn * ax * zxx;
    ab[0] = cs * zv - sn * (ax * zx + at * zt + axx * zxx) - cs * ax * ax * zxx;
  } else {
    ab[0] = cs * zb[0];
  }
}

// ---------------------------------------------------------------------------
// One hidden layer, forward: ys = s * y (in place), yo = V^T sin-jets(U ys + b).
// With PIPE the loop is software-pipelined: the U-side MFMAs of the next
// neuron group are issued next to the VALU sin-jet work of the current one.
// That pays in the reverse-mode kernels (two waves per SIMD, where the
// forward sweep is not the register peak); the forward-only kernels run
// three waves per SIMD, where the extra accumulators only add spills.
// Returns the largest |a_v| seen (to select the accurate sin/cos path if
// needed).
// ---------------------------------------------------------------------------
template <int NJ, int RGM, int RGI, int RGO, bool ACC, bool PIPE, int EDGE>
__device__ __forceinline__ float layer_fwd_pass(const float* __restrict__ Us,
                                                const float* __restrict__ Vs,
                                                const float* __restrict__ bs, int Wp, int li,
                                                const f4 (&ys)[NJ][RGM], f4 (&yo)[NJ][RGM]) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGO; ++g) yo[c][g] = zero4();
  float amax = 0.f;
  f4 a[NJ], z[NJ];
  if constexpr (!PIPE) {
    for (int w0 = 0; w0 < Wp; w0 += 4) {
      u_side<NJ, RGM, RGI, EDGE>(Us, bs, w0, li, ys, a);
      sigma_fwd<NJ, ACC>(a, z, amax);
      v_side<NJ, RGM, RGO, EDGE>(Vs, w0, li, z, yo);
    }
    return amax;
  }
  u_side<NJ, RGM, RGI, EDGE>(Us, bs, 0, li, ys, a);
  for (int w0 = 0; w0 < Wp - 4; w0 += 4) {
    f4 an[NJ];
    u_side<NJ, RGM, RGI, EDGE>(Us, bs, w0 + 4, li, ys, an);
    sigma_fwd<NJ, ACC>(a, z, amax);
    v_side<NJ, RGM, RGO, EDGE>(Vs, w0, li, z, yo);
#pragma unroll
    for (int c = 0; c < NJ; ++c) a[c] = an[c];
    interleave<NJ * 4 * RGI>();
  }
  sigma_fwd<NJ, ACC>(a, z, amax);
  v_side<NJ, RGM, RGO, EDGE>(Vs, Wp - 4, li, z, yo);
  return amax;
}

// Uss is U^l diag(s^l) as staged, so that the U side contracts y itself.
template <int NJ, int RGM, int RGI, int RGO, int SC, bool PIPE, int EDGE>
__device__ __forceinline__ void layer_fwd(const float* __restrict__ Uss,
                                          const float* __restrict__ Vs,
                                          const float* __restrict__ bs, int Wp, int li,
                                          const f4 (&y)[NJ][RGM], f4 (&yo)[NJ][RGM],
                                          float& amax) {
  const float* __restrict__ Us = Uss;
  if constexpr (SC == SC_ACC) {
    layer_fwd_pass<NJ, RGM, RGI, RGO, true, PIPE, EDGE>(Us, Vs, bs, Wp, li, y, yo);
  } else {
    const float m = layer_fwd_pass<NJ, RGM, RGI, RGO, false, PIPE, EDGE>(Us, Vs, bs, Wp, li, y, yo);
    amax = vmax(amax, m);
    if constexpr (SC == SC_REDO) {
      if (__builtin_expect(__any(!(m <= kFastRange)), 0))
        layer_fwd_pass<NJ, RGM, RGI, RGO, true, PIPE, EDGE>(Us, Vs, bs, Wp, li, y, yo);
    }
  }
}

// ---------------------------------------------------------------------------
// One hidden layer, reverse: recompute a = (U diag(s)) y + b, pull
// yb = dL/dy^{l+1} back through V and the sin jets, write the layer's dL/db
// row, and return wb = U^T abar (so that dL/ds = sum_c wb * y and
// dL/dy^l = s * wb).  The
// loop is not software-pipelined: carrying the next group's a and zb beside
// the current ones spilled at the two-waves-per-SIMD register budget and
// measured 3-7 % slower than this plain loop.
// ---------------------------------------------------------------------------
template <int NJ, int RGM, int RGI, int RGO, bool ACC, int EDGE>
__device__ __forceinline__ float layer_bwd_pass(const float* __restrict__ Us,
                                                const float* __restrict__ Uss,
                                                const float* __restrict__ Vs,
                                                const float* __restrict__ bs, int Wp, int li,
                                                int lane, const f4 (&y)[NJ][RGM],
                                                const f4 (&yb)[NJ][RGM], f4 (&wb)[NJ][RGM],
                                                float* __restrict__ bbar_row) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGI; ++g) wb[c][g] = zero4();
  const int comp = sum4_component(lane);
  float amax = 0.f;
  f4 a[NJ], zb[NJ], ab[NJ];
  for (int w0 = 0; w0 < Wp; w0 += 4) {
    u_side<NJ, RGM, RGI, EDGE>(Uss, bs, w0, li, y, a);
    v_rev<NJ, RGM, RGO, EDGE>(Vs, w0, li, yb, zb);
    sigma_bwd<NJ, ACC>(a, zb, ab, amax);
    const float bsum = wave_sum4(ab[0], lane);
    if ((lane & 15) == 0) bbar_row[w0 + comp] = bsum;
    ut_side<NJ, RGM, RGI, EDGE>(Us, w0, li, ab, wb);
  }
  return amax;
}

template <int NJ, int RGM, int RGI, int RGO, int SC, int EDGE>
__device__ __forceinline__ void layer_bwd(const float* __restrict__ Us,
                                          const float* __restrict__ Uss,
                                          const float* __restrict__ Vs,
                                          const float* __restrict__ bs, int Wp, int li,
                                          int lane, const f4 (&y)[NJ][RGM],
                                          const f4 (&yb)[NJ][RGM], f4 (&wb)[NJ][RGM],
                                          float* __restrict__ bbar_row, float& amax) {
  if constexpr (SC == SC_ACC) {
    layer_bwd_pass<NJ, RGM, RGI, RGO, true, EDGE>(Us, Uss, Vs, bs, Wp, li, lane, y, yb, wb,
                                                  bbar_row);
  } else {
    const float m = layer_bwd_pass<NJ, RGM, RGI, RGO, false, EDGE>(Us, Uss, Vs, bs, Wp, li, lane,
                                                                   y, yb, wb, bbar_row);
    amax = vmax(amax, m);
    if constexpr (SC == SC_REDO) {
      if (__builtin_expect(__any(!(m <= kFastRange)), 0))
        layer_bwd_pass<NJ, RGM, RGI, RGO, true, EDGE>(Us, Uss, Vs, bs, Wp, li, lane, y, yb, wb,
                                                      bbar_row);
    }
  }
}

// ---------------------------------------------------------------------------
// Workgroup driver
// ---------------------------------------------------------------------------
// LDS of a workgroup.  Per layer slab: U [Wmax_p][RP], U diag(s) [Wmax_p][RP],
// V [Wmax_p][RP], b [Wmax_p], s [RP]; then per slab the waves' b and s
// gradient rows.  With
// one slab (lstride == 0) the layers are staged one at a time; with resident
// layers, hidden layer l lives in slab l - 1, lstride floats apart, for the
// whole tile.
struct Smem {
  float* Us;
  float* Uss;    // U diag(s)
  float* Vs;
  float* bs;
  float* ss;
  float* bbar;   // [slabs][kWaves][Wmax_p]
  float* sbar;   // [slabs][kWaves][RP]
  float* lw;     // [kWaves][4] wave sums, then [kWaves] range flags
  int lstride;   // floats between layer slabs; 0: one slab
};

__device__ __forceinline__ Smem make_smem(float* base, int Wm, int RP, int n_slabs) {
  const int n = n_slabs > 0 ? n_slabs : 1;
  const int slab = Wm * RP * 3 + Wm + RP;
  Smem sm;
  sm.Us = base;
  sm.Uss = sm.Us + Wm * RP;
  sm.Vs = sm.Uss + Wm * RP;
  sm.bs = sm.Vs + Wm * RP;
  sm.ss = sm.bs + Wm;
  sm.bbar = base + n * slab;
  sm.sbar = sm.bbar + n * kWaves * Wm;
  sm.lw = sm.sbar + n * kWaves * RP;
  sm.lstride = n_slabs > 0 ? slab : 0;
  return sm;
}

// The slab of hidden layer l (the one slab when layers are staged in turn).
__device__ __forceinline__ Smem layer_smem(const Smem& sm, int l, int Wm, int RP) {
  if (sm.lstride == 0) return sm;
  Smem v = sm;
  const int o = (l - 1) * sm.lstride;
  v.Us += o;
  v.Uss += o;
  v.Vs += o;
  v.bs += o;
  v.ss += o;
  v.bbar += (l - 1) * kWaves * Wm;
  v.sbar += (l - 1) * kWaves * RP;
  return v;
}

// dst[i] = src[i] for i < n (float4), two loads in flight per thread.
template <int NT>
__device__ __forceinline__ void copy_f4(f4* __restrict__ dst, const f4* __restrict__ src, int n,
                                        int tx) {
  int i = tx;
  for (; i + NT < n; i += 2 * NT) {
    const f4 a = src[i], b = src[i + NT];
    dst[i] = a;
    dst[i + NT] = b;
  }
  if (i < n) dst[i] = src[i];
}

// Stage layer l's U^l [Wp][KI], V^{l+1} [Wp][KO], b^l [Wp] and s^l [KI] into
// LDS with zero padding.  NT threads cooperate, numbered by tix in [0, NT)
// (threadIdx.x by default); ss == nullptr leaves s^l out.
template <int NT>
__device__ void stage_layer(const KNet& net, const float* __restrict__ s, int l, int KI,
                            int KO, float* __restrict__ Us, float* __restrict__ Vs,
                            float* __restrict__ bs, float* __restrict__ ss, int tix = -1) {
  const int tx = tix < 0 ? (int)threadIdx.x : tix;
  // rows padded to a multiple of 16 (value-only tiles step over 16 neurons)
  const int W = net.M[l], Wp = (W + 15) & ~15, rl = net.r[l], ro = net.r[l + 1];
  const float* __restrict__ U = net.U + net.offU[l];
  const float* __restrict__ V = net.V + net.offV[l + 1];
  const float* __restrict__ b = net.b + net.offB[l];
  // a factor whose rank fills the tile is one contiguous block: copied as
  // float4 when 16-byte aligned, which takes a quarter of the round trips
  if (rl == KI && (reinterpret_cast<uintptr_t>(U) & 15) == 0) {
    copy_f4<NT>(reinterpret_cast<f4*>(Us), reinterpret_cast<const f4*>(U), W * KI / 4, tx);
    for (int i = W * KI + tx; i < Wp * KI; i += NT) Us[i] = 0.f;
  } else {
    for (int i = tx; i < Wp * KI; i += NT) {
      const int w = i / KI, k = i - w * KI;
      Us[i] = (w < W && k < rl) ? U[w * rl + k] : 0.f;
    }
  }
  if (ro == KO && (reinterpret_cast<uintptr_t>(V) & 15) == 0) {
    copy_f4<NT>(reinterpret_cast<f4*>(Vs), reinterpret_cast<const f4*>(V), W * KO / 4, tx);
    for (int i = W * KO + tx; i < Wp * KO; i += NT) Vs[i] = 0.f;
  } else {
    for (int i = tx; i < Wp * KO; i += NT) {
      const int w = i / KO, k = i - w * KO;
      Vs[i] = (w < W && k < ro) ? V[w * ro + k] : 0.f;
    }
  }
  for (int i = tx; i < Wp; i += NT) bs[i] = i < W ? b[i] : 0.f;
  if (ss)
    for (int i = tx; i < KI; i += NT) ss[i] = i < rl ? s[net.offS[l] + i] : 0.f;
}

// Stage U^l diag(s^l) [Wp][KI] (zero padded) for the U side, which then
// contracts the unscaled reduced jets.
template <int NT>
__device__ void stage_us(const KNet& net, const float* __restrict__ s, int l, int KI,
                         float* __restrict__ Uss) {
  const int W = net.M[l], Wp = (W + 15) & ~15, rl = net.r[l];
  const float* __restrict__ U = net.U + net.offU[l];
  const float* __restrict__ sl = s + net.offS[l];
  for (int i = threadIdx.x; i < Wp * KI; i += NT) {
    const int w = i / KI, k = i - w * KI;
    Uss[i] = (w < W && k < rl) ? U[w * rl + k] * sl[k] : 0.f;
  }
}

// Resident layers: stage every hidden layer's slab (or, when the factors are
// already there from the previous tile of the same net, only s and U diag(s)).
template <int RP>
__device__ void stage_resident(const KNet& net, const float* __restrict__ s, bool factors,
                               const Smem& sm, int Wm) {
  const int L = net.L, tx = threadIdx.x;
  for (int l = 1; l <= L - 1; ++l) {
    const int KI = l == 1 ? 4 : RP, KO = l == L - 1 ? 4 : RP;
    const Smem ls = layer_smem(sm, l, Wm, RP);
    if (factors) {
      stage_layer<kThreads>(net, s, l, KI, KO, ls.Us, ls.Vs, ls.bs, ls.ss);
    } else {
      const int rl = net.r[l];
      for (int i = tx; i < KI; i += kThreads) ls.ss[i] = i < rl ? s[net.offS[l] + i] : 0.f;
    }
    stage_us<kThreads>(net, s, l, KI, ls.Uss);
  }
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

template <int NJ, int RGM, int SC, bool PIPE>
__device__ __forceinline__ void fwd_dispatch(bool first, bool last, const Smem& sm, int Wp,
                                             int li, f4 (&y)[NJ][RGM],
                                             f4 (&yo)[NJ][RGM], float& amax) {
  constexpr int F = kEdgeFirst, LA = kEdgeLast;
  if (first && last)
    layer_fwd<NJ, RGM, 1, 1, SC, PIPE, F | LA>(sm.Uss, sm.Vs, sm.bs, Wp, li, y, yo, amax);
  else if (first)
    layer_fwd<NJ, RGM, 1, RGM, SC, PIPE, F>(sm.Uss, sm.Vs, sm.bs, Wp, li, y, yo, amax);
  else if (last)
    layer_fwd<NJ, RGM, RGM, 1, SC, PIPE, LA>(sm.Uss, sm.Vs, sm.bs, Wp, li, y, yo, amax);
  else
    layer_fwd<NJ, RGM, RGM, RGM, SC, PIPE, 0>(sm.Uss, sm.Vs, sm.bs, Wp, li, y, yo, amax);
}

template <int NJ, int RGM, int SC>
__device__ __forceinline__ void bwd_dispatch(bool first, bool last, const Smem& sm, int Wp,
                                             int li, int lane, const f4 (&y)[NJ][RGM],
                                             const f4 (&yb)[NJ][RGM], f4 (&wb)[NJ][RGM],
                                             float* bbar_row, float& amax) {
  constexpr int F = kEdgeFirst, LA = kEdgeLast;
  if (first && last)
    layer_bwd<NJ, RGM, 1, 1, SC, F | LA>(sm.Us, sm.Uss, sm.Vs, sm.bs, Wp, li, lane, y, yb, wb,
                                         bbar_row, amax);
  else if (first)
    layer_bwd<NJ, RGM, 1, RGM, SC, F>(sm.Us, sm.Uss, sm.Vs, sm.bs, Wp, li, lane, y, yb, wb,
                                      bbar_row, amax);
  else if (last)
    layer_bwd<NJ, RGM, RGM, 1, SC, LA>(sm.Us, sm.Uss, sm.Vs, sm.bs, Wp, li, lane, y, yb, wb,
                                       bbar_row, amax);
  else
    layer_bwd<NJ, RGM, RGM, RGM, SC, 0>(sm.Us, sm.Uss, sm.Vs, sm.bs, Wp, li, lane, y, yb, wb,
                                        bbar_row, amax);
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

// Waves per SIMD the compiler budgets registers for.  Rank tiles up to 8
// fit two waves (256 registers) in every mode, which hides the latency of
// the one-wave-per-point-group chain: measured 20-27 % faster for the
// gradient at rank tile 8 than at the default budget (one wave, ~310
// registers).  The forward-only modes (jets, value, loss) there take three
// waves (168 registers).  So do the reverse modes of the persistent task-
// table kernel, which always has more tiles than SIMDs in its throughput
// forms: 168 registers with ~40 spilled outside the neuron loops, 6-7 %
// faster per differentiation step than two waves.  The plain launch keeps
// two: at config-3 sizes one wave per SIMD is all there is, and the spills
// only lengthen its chain (5 % slower at three).  Rank tile 16 at two waves
// spills heavily (2x slower).
template <int RP, int MODE, bool TABLE>
constexpr int fused_waves_per_simd() {
  if (RP > 8) return 1;
  return (MODE == MODE_GRAD || MODE == MODE_VJP) && !TABLE ? 2 : 3;
}

template <int RP, int MODE, int NJ, int SC, bool TABLE>
__device__ void run_workgroup(const KNet& net, const KInst& inst, int64_t ckpt_per_wave,
                              int Wmax_p, const KTile& tile, int kind, int wg,
                              const float* __restrict__ s, const float* __restrict__ mu,
                              const Smem& sm) {
  constexpr bool REV = reverse_mode(MODE);
  // the forward group loop is software-pipelined only at the two-wave budget
  constexpr bool PIPE = REV && fused_waves_per_simd<RP, MODE, TABLE>() == 2;
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
  if constexpr (REV) ckbase = tile.ck + wave * ckpt_per_wave;
  constexpr int64_t kSlot = 4 * RGM * 64 * 4;  // floats per checkpointed layer

  // ---- forward sweep ------------------------------------------------------
  // Resident layers: one staging and one barrier for the whole tile (the
  // caller's LDS is free on entry); otherwise two barriers per layer.
  const bool res = sm.lstride != 0;
  if (res) {
    stage_resident<RP>(net, s, tile.stage_net, sm, Wmax_p);
    __syncthreads();
  }
  float amax = 0.f;  // largest |a| met by this lane (sin/cos range check)
  f4 y[NJ][RGM], yo[NJ][RGM];
  input_jets<NJ, RGM>(net, x, t, y);
  for (int l = 1; l <= L - 1; ++l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    const Smem ls = layer_smem(sm, l, Wmax_p, RP);
    if (!res) {
      __syncthreads();
      stage_layer<kThreads>(net, s, l, KI, KO, sm.Us, sm.Vs, sm.bs, sm.ss);
      stage_us<kThreads>(net, s, l, KI, sm.Uss);
      __syncthreads();
    }
    const int Wp = (net.M[l] + 3) & ~3;
    fwd_dispatch<NJ, RGM, SC, PIPE>(first, last, ls, Wp, li, y, yo, amax);
    if constexpr (REV)
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
  if constexpr (MODE == MODE_VJP) {
    // cotangent of the jets supplied by the caller (interior points only)
    if (valid) {
      const int64_t n = inst.n_r;
#pragma unroll
      for (int c = 0; c < NJ; ++c) ub[c] = inst.cot[c * n + p];
    }
  } else if constexpr (NJ == 4) {
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

  float* rec = tile.rec;
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

  // loss sums and the output layer's s and b gradients (after a barrier)
  auto output_record = [&]() {
    if (tid < 4) {
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
  };
  // layer l's s and b gradients, the waves' rows summed in a fixed order
  auto layer_record = [&](const Smem& ls, int l) {
    const int W = net.M[l], rl = net.r[l], Wm = Wmax_p;
    for (int i = tid; i < W; i += kThreads)
      rec[4 + net.r_total + net.offB[l] + i] =
          ((ls.bbar[i] + ls.bbar[Wm + i]) + ls.bbar[2 * Wm + i]) + ls.bbar[3 * Wm + i];
    for (int i = tid; i < rl; i += kThreads)
      rec[4 + net.offS[l] + i] =
          ((ls.sbar[i] + ls.sbar[RP + i]) + ls.sbar[2 * RP + i]) + ls.sbar[3 * RP + i];
  };

  // ---- reverse sweep over the hidden layers --------------------------------
  for (int l = L - 1; l >= 1; --l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    const int Wp = (net.M[l] + 3) & ~3;
    const Smem ls = layer_smem(sm, l, Wmax_p, RP);
    if (!res) {
      __syncthreads();
      if (l == L - 1) output_record();
      stage_layer<kThreads>(net, s, l, KI, KO, sm.Us, sm.Vs, sm.bs, sm.ss);
      stage_us<kThreads>(net, s, l, KI, sm.Uss);
      __syncthreads();
    }
    if (first)
      input_jets<NJ, RGM>(net, x, t, y);
    else
      ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
    bwd_dispatch<NJ, RGM, SC>(first, last, ls, Wp, li, lane, y, yb, wb,
                              ls.bbar + wave * Wmax_p, amax);
    const int RGI = first ? 1 : RGM;
#pragma unroll
    for (int g = 0; g < RGM; ++g) {
      if (g < RGI) {
        f4 acc = zero4();
#pragma unroll
        for (int c = 0; c < NJ; ++c) acc += wb[c][g] * y[c][g];
        const float tot = wave_sum4(acc, lane);
        if ((lane & 15) == 0) ls.sbar[wave * RP + 4 * g + comp] = tot;
      }
    }
    if (!first) {
#pragma unroll
      for (int g = 0; g < RGM; ++g) {
        const f4 s4 = *reinterpret_cast<const f4*>(ls.ss + 4 * g);
#pragma unroll
        for (int c = 0; c < NJ; ++c) yb[c][g] = s4 * wb[c][g];
      }
    }
    if (!res) {
      __syncthreads();
      layer_record(ls, l);
    }
  }
  if (res) {
    __syncthreads();
    output_record();
    for (int l = L - 1; l >= 1; --l) layer_record(layer_smem(sm, l, Wmax_p, RP), l);
  }
  if constexpr (SC == SC_TRACK) {
    // flag the workgroup for the accurate relaunch if any lane met |a| > kFastRange
    // (own slots: the loss sums in lw[0, 16) may still be being read)
    float* fl = sm.lw + 4 * kWaves;
    const bool bad = __any(!(amax <= kFastRange));
    if (lane == 0) fl[wave] = bad ? 1.f : 0.f;
    __syncthreads();
    if (tid == 0) *tile.flag = (fl[0] + fl[1] + fl[2] + fl[3]) > 0.f ? 1 : 0;
  }
}

// Dispatch on the point kind: interior points carry four jets, IC/BC points
// (and plain value evaluation) one.
template <int RP, int MODE, int SC, bool TABLE>
__device__ __forceinline__ void run_kind(const KNet& net, const KInst& inst,
                                         int64_t ckpt_per_wave, int Wmax_p, const KTile& tile,
                                         int kind, int wg, const float* __restrict__ s,
                                         const float* __restrict__ mu, const Smem& sm) {
  if constexpr (MODE == MODE_VALUE) {
    run_workgroup<RP, MODE, 1, SC, TABLE>(net, inst, ckpt_per_wave, Wmax_p, tile, kind, wg, s, mu, sm);
  } else if constexpr (MODE == MODE_JETS || MODE == MODE_VJP) {
    run_workgroup<RP, MODE, 4, SC, TABLE>(net, inst, ckpt_per_wave, Wmax_p, tile, kind, wg, s, mu, sm);
  } else {
    if (kind == 0)
      run_workgroup<RP, MODE, 4, SC, TABLE>(net, inst, ckpt_per_wave, Wmax_p, tile, kind, wg, s, mu,
                                     sm);
    else
      run_workgroup<RP, MODE, 1, SC, TABLE>(net, inst, ckpt_per_wave, Wmax_p, tile, kind, wg, s, mu,
                                     sm);
  }
}


// W3: the three-wave register budget of the task-table kernel, for launches
// with more workgroups than two waves per SIMD hold at once.
template <int RP, int MODE, int SC, bool W3 = false>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(fused_waves_per_simd<RP, MODE, W3>()))) void lrnr_fused_kernel(
    KNet net, KInst inst, KGrid grid) {
  if constexpr (SC == SC_ACC) {
    if (grid.flags[blockIdx.x] == 0) return;  // only workgroups flagged by SC_TRACK
  }
  extern __shared__ float4 smem_raw[];
  const Smem sm = make_smem(reinterpret_cast<float*>(smem_raw), grid.Wmax_p, RP, grid.res_layers);

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
  KTile tile;
  tile.rec = grid.partials + (int64_t)blockIdx.x * grid.P;
  tile.ck = grid.ckpt ? grid.ckpt + (int64_t)blockIdx.x * kWaves * grid.ckpt_per_wave : nullptr;
  tile.flag = grid.flags ? grid.flags + blockIdx.x : nullptr;
  tile.stage_net = true;
  run_kind<RP, MODE, SC, W3>(net, inst, grid.ckpt_per_wave, grid.Wmax_p, tile, kind, wg, s, mu,
                             sm);
}

template <int RP, int MODE, int SC, bool W3 = false>
static hipError_t launch_one(const KNet& net, const KInst& inst, const KGrid& grid,
                             hipStream_t stream) {
  const dim3 blocks((unsigned)(grid.B * grid.G_inst)), threads(kThreads);
  const size_t lds = fused_lds_bytes(RP, grid.Wmax_p, grid.res_layers);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)lrnr_fused_kernel<RP, MODE, SC, W3>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((lrnr_fused_kernel<RP, MODE, SC, W3>), blocks, threads, lds, stream, net,
                     inst, grid);
  return hipGetLastError();
}

}  // namespace lrnr
