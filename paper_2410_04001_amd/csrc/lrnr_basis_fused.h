// Loss gradient with respect to the bases U^l and V^l, fused into the
// forward and reverse sweeps of the hot-path kernel (the meta-learning phase
// of Section 3.1 trains the bases, eq. 3.4):
//   dL/dU^l = sum_p sum_c abar^l_{p,c} (s^l * y^l_{p,c})^T       [M_l][r_l]
//   dL/dV^l = sum_p sum_c z^{l-1}_{p,c} ybar^l_{p,c}^T            [M_{l-1}][r_l]
// with c over the jets (value, d/dx, d/dt, d2/dx2), abar^l the adjoint of the
// pre-activation of layer l, y^l = V^lT z^{l-1}, ybar^l its adjoint and z^0 =
// (x, t) with constant jets.
//
// The sweeps are those of the loss + gradient kernel (one lane per point,
// 4x4x1 MFMA contractions, reduced jets checkpointed, the U side recomputed
// in reverse).  In the reverse pass of hidden layer l, the group of four
// neurons w0..w0+3 already holds abar (4 neurons x jets) and s * y^l (ranks x
// jets) per lane, and recomputes z^l (4 neurons x jets) from sin/cos of a;
// ybar^{l+1} is the pass's input.  Each lane forms its point's outer-product
// terms summed over the jets (VALU), a 64-lane reduction gives the wave's sum
// for four entries at a time, and the wave writes them once into its own
// record.  The records (one per wave) are then summed over the waves, tiles
// and instances in a fixed order in FP64: no atomics, bitwise reproducible.
// The points are the contracted dimension, so the sum over them is a
// reduction across lanes rather than an MFMA contraction.
#pragma once

#include "lrnr_fused_impl.h"

namespace lrnr {

struct KBasis {
  KNet net;
  KInst inst;               // instance 0; instance i reads s + i*s_stride, mu + 3*i
  KGrid grid;               // tiles, checkpoints (partials unused)
  float* wrec;              // [B * G_inst][kWaves][PB] per-wave records
  int PB;                   // floats per wave record: U entries, then V entries
  int U_total;              // offset of the V entries in a record
};

// Four row totals of a 64-lane sum (wave_sum4) into dst[w * ld + k]: lane
// 16q holds the total of component sum4_component(16q), which is neuron
// w0 + that component for the U and V entries.
__device__ __forceinline__ void put_row_totals(float tot, int lane, int w, int W, int k, int rk,
                                               int ld, float* __restrict__ dst) {
  if ((lane & 15) == 0 && w < W && k < rk) dst[w * ld + k] = tot;
}

// dU[w0..w0+3][k] over the wave's points: sum_c abar_c * (s*y)_c[k]
template <int NJ, int RGM, int RGI>
__device__ __forceinline__ void acc_u(const f4 (&ab)[NJ], const f4 (&ys)[NJ][RGM], int w0,
                                      int lane, int W, int rl, float* __restrict__ dU) {
  const int w = w0 + sum4_component(lane);
#pragma unroll
  for (int g = 0; g < RGI; ++g)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      f4 v = ab[0] * ys[0][g][kk];
#pragma unroll
      for (int c = 1; c < NJ; ++c) v += ab[c] * ys[c][g][kk];
      put_row_totals(wave_sum4(v, lane), lane, w, W, 4 * g + kk, rl, rl, dU);
    }
}

// dV^{l+1}[w0..w0+3][k] over the wave's points: sum_c z_c * ybar^{l+1}_c[k]
template <int NJ, int RGM, int RGO>
__device__ __forceinline__ void acc_v(const f4 (&z)[NJ], const f4 (&yb)[NJ][RGM], int w0,
                                      int lane, int W, int ro, float* __restrict__ dV) {
  const int w = w0 + sum4_component(lane);
#pragma unroll
  for (int g = 0; g < RGO; ++g)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      f4 v = z[0] * yb[0][g][kk];
#pragma unroll
      for (int c = 1; c < NJ; ++c) v += z[c] * yb[c][g][kk];
      put_row_totals(wave_sum4(v, lane), lane, w, W, 4 * g + kk, ro, ro, dV);
    }
}

// Adjoints of the a jets (as sigma_bwd) and the z jets of the same group.
template <int NJ, bool ACC>
__device__ __forceinline__ void sigma_bwd_z(const f4 (&a)[NJ], const f4 (&zb)[NJ], f4 (&ab)[NJ],
                                            f4 (&z)[NJ], float& amax) {
  f4 sn, cs;
  sincos4<ACC>(a[0], sn, cs, amax);
  z[0] = sn;
  if constexpr (NJ == 4) {
    const f4 ax = a[1], at = a[2], axx = a[3];
    const f4 zv = zb[0], zx = zb[1], zt = zb[2], zxx = zb[3];
    z[1] = cs * ax;
    z[2] = cs * at;
    z[3] = cs * axx - sn * ax * ax;
    ab[3] = cs * zxx;
    ab[2] = cs * zt;
    ab[1] = cs * zx - 2.f * sn * ax * zxx;
    ab[0] = cs * zv - sn * (ax * zx + at * zt + axx * zxx) - cs * ax * ax * zxx;
  } else {
    ab[0] = cs * zb[0];
  }
}

// One hidden layer l, reverse, with the basis terms: recompute a = U(s y)+b,
// zbar = V^{l+1} ybar, abar; write dU^l and dV^{l+1} entries of this wave;
// return wb = U^T abar (so that ybar^l = s * wb).
template <int NJ, int RGM, int RGI, int RGO, bool ACC>
__device__ __forceinline__ float basis_bwd_pass(const float* __restrict__ Us,
                                                const float* __restrict__ Vs,
                                                const float* __restrict__ bs, int Wp, int W,
                                                int rl, int ro, int li, int lane,
                                                const f4 (&ys)[NJ][RGM], const f4 (&yb)[NJ][RGM],
                                                f4 (&wb)[NJ][RGM], float* __restrict__ dU,
                                                float* __restrict__ dV) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGI; ++g) wb[c][g] = zero4();
  float amax = 0.f;
  for (int w0 = 0; w0 < Wp; w0 += 4) {
    f4 a[NJ], zb[NJ], ab[NJ], z[NJ];
    u_side<NJ, RGM, RGI>(Us, bs, w0, li, ys, a);
    v_rev<NJ, RGM, RGO>(Vs, w0, li, yb, zb);
    sigma_bwd_z<NJ, ACC>(a, zb, ab, z, amax);
    ut_side<NJ, RGM, RGI>(Us, w0, li, ab, wb);
    acc_u<NJ, RGM, RGI>(ab, ys, w0, lane, W, rl, dU);
    acc_v<NJ, RGM, RGO>(z, yb, w0, lane, W, ro, dV);
  }
  return amax;
}

template <int NJ, int RGM, int RGI, int RGO>
__device__ __forceinline__ void basis_bwd(const Smem& sm, int Wp, int W, int rl, int ro, int li,
                                          int lane, f4 (&y)[NJ][RGM], const f4 (&yb)[NJ][RGM],
                                          f4 (&wb)[NJ][RGM], float* dU, float* dV) {
#pragma unroll
  for (int g = 0; g < RGI; ++g) {
    const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + 4 * g);
#pragma unroll
    for (int c = 0; c < NJ; ++c) y[c][g] *= s4;
  }
  const float m = basis_bwd_pass<NJ, RGM, RGI, RGO, false>(sm.Us, sm.Vs, sm.bs, Wp, W, rl, ro,
                                                           li, lane, y, yb, wb, dU, dV);
  // |a| beyond the fast sin/cos range: the layer again with ocml's sincosf
  // (same entries, overwritten)
  if (__builtin_expect(__any(!(m <= kFastRange)), 0))
    basis_bwd_pass<NJ, RGM, RGI, RGO, true>(sm.Us, sm.Vs, sm.bs, Wp, W, rl, ro, li, lane, y, yb,
                                            wb, dU, dV);
}

template <int NJ, int RGM>
__device__ __forceinline__ void basis_bwd_dispatch(bool first, bool last, const Smem& sm, int Wp,
                                                   int W, int rl, int ro, int li, int lane,
                                                   f4 (&y)[NJ][RGM], const f4 (&yb)[NJ][RGM],
                                                   f4 (&wb)[NJ][RGM], float* dU, float* dV) {
  if (first && last)
    basis_bwd<NJ, RGM, 1, 1>(sm, Wp, W, rl, ro, li, lane, y, yb, wb, dU, dV);
  else if (first)
    basis_bwd<NJ, RGM, 1, RGM>(sm, Wp, W, rl, ro, li, lane, y, yb, wb, dU, dV);
  else if (last)
    basis_bwd<NJ, RGM, RGM, 1>(sm, Wp, W, rl, ro, li, lane, y, yb, wb, dU, dV);
  else
    basis_bwd<NJ, RGM, RGM, RGM>(sm, Wp, W, rl, ro, li, lane, y, yb, wb, dU, dV);
}

template <int RP, int NJ>
__device__ void basis_workgroup(const KBasis& kb, const KTile& tile, float* __restrict__ wrec,
                                int kind, int wg, const float* __restrict__ s,
                                const float* __restrict__ mu, const Smem& sm) {
  constexpr int RGM = RP / 4;
  const KNet& net = kb.net;
  const KInst& inst = kb.inst;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 3;
  const int L = net.L;
  float* dUall = wrec;
  float* dVall = wrec + kb.U_total;

  // ---- the lane's point (as the loss + gradient kernel) ------------------
  float x = 0.f, t = 0.f;
  bool valid = false;
  if (kind == 0) {
    const int64_t p = (int64_t)wg * kPtsPerWG + wave * 64 + lane;
    valid = p < inst.n_r;
    if (valid) {
      x = inst.xt_r[2 * p];
      t = inst.xt_r[2 * p + 1];
    }
  } else if (kind == 1) {
    const int64_t p = (int64_t)wg * kPtsPerWG + wave * 64 + lane;
    valid = p < inst.n_0;
    if (valid) x = inst.x_0[p];
  } else {
    const int64_t p = (int64_t)wg * kBcPairsPerWG + wave * 32 + (lane >> 1);
    valid = p < inst.n_b;
    x = (lane & 1) ? LRNR_TWO_PI_F : 0.f;
    if (valid) t = inst.t_b[p];
  }
  float* ckbase = tile.ck + wave * kb.grid.ckpt_per_wave;
  constexpr int64_t kSlot = 4 * RGM * 64 * 4;

  // ---- forward sweep ------------------------------------------------------
  float amax = 0.f;
  f4 y[NJ][RGM], yo[NJ][RGM];
  input_jets<NJ, RGM>(net, x, t, y);
  for (int l = 1; l <= L - 1; ++l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    __syncthreads();
    stage_layer<kThreads>(net, s, l, KI, KO, sm.Us, sm.Vs, sm.bs, sm.ss);
    stage_us<kThreads>(net, s, l, KI, sm.Uss);
    __syncthreads();
    const int Wp = (net.M[l] + 3) & ~3;
    fwd_dispatch<NJ, RGM, SC_REDO, true>(first, last, sm, Wp, li, y, yo, amax);
    if (!last) ckpt_store<NJ, RGM>(ckbase + (l - 1) * kSlot, lane, yo);
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
      for (int g = 0; g < RGM; ++g) y[c][g] = yo[c][g];
  }

  // ---- output layer and the loss adjoint (eq. 4.1, eq. 3.5 / 3.6) --------
  const float UL = net.U[net.offU[L]];
  const float sL = s[net.offS[L]];
  const float bL = net.b[net.offB[L]];
  const float cL = UL * sL;
  float u[NJ];
#pragma unroll
  for (int c = 0; c < NJ; ++c) u[c] = cL * y[c][0][0];
  u[0] += bL;
  const int form = inst.form;
  float ub[NJ];
#pragma unroll
  for (int c = 0; c < NJ; ++c) ub[c] = 0.f;
  if constexpr (NJ == 4) {
    const float beta = mu[0], nu = mu[1], rho = mu[2];
    const float res = u[2] + beta * u[1] - nu * u[3] - rho * u[0] * (1.f - u[0]);
    const float dphi = form == 0 ? 2.f * res : (res > 0.f ? 1.f : (res < 0.f ? -1.f : 0.f));
    const float g = valid ? inst.wr_n * dphi : 0.f;
    ub[0] = -rho * (1.f - 2.f * u[0]) * g;
    ub[1] = beta * g;
    ub[2] = g;
    ub[3] = -nu * g;
  } else if (kind == 1) {
    const float e0 = u[0] - sinf(x);
    const float dphi = form == 0 ? 2.f * e0 : (e0 > 0.f ? 1.f : (e0 < 0.f ? -1.f : 0.f));
    ub[0] = valid ? inst.w0_n * dphi : 0.f;
  } else {
    const float other = __shfl_xor(u[0], 1);
    const bool right = lane & 1;
    const float eb = right ? other - u[0] : u[0] - other;
    const float dphi = form == 0 ? 2.f * eb : (eb > 0.f ? 1.f : (eb < 0.f ? -1.f : 0.f));
    ub[0] = valid ? (right ? -inst.wb_n : inst.wb_n) * dphi : 0.f;
  }

  // dU^L = sum_p sum_c ubar_c s^L y^L_c (M_L = r_L = 1)
  {
    float a = 0.f;
#pragma unroll
    for (int c = 0; c < NJ; ++c) a += ub[c] * y[c][0][0];
    const float tot = wave_sum4(f4{sL * a, 0.f, 0.f, 0.f}, lane);
    if (lane == 0) dUall[net.offU[L]] = tot;
  }
  f4 yb[NJ][RGM], wb[NJ][RGM];
#pragma unroll
  for (int c = 0; c < NJ; ++c) {
#pragma unroll
    for (int g = 0; g < RGM; ++g) yb[c][g] = zero4();
    yb[c][0][0] = cL * ub[c];
  }

  // ---- reverse sweep over the hidden layers ------------------------------
  for (int l = L - 1; l >= 1; --l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    const int W = net.M[l], Wp = (W + 3) & ~3;
    __syncthreads();
    stage_layer<kThreads>(net, s, l, KI, KO, sm.Us, sm.Vs, sm.bs, sm.ss);
    __syncthreads();
    if (first)
      input_jets<NJ, RGM>(net, x, t, y);
    else
      ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
    basis_bwd_dispatch<NJ, RGM>(first, last, sm, Wp, W, net.r[l], net.r[l + 1], li, lane, y, yb,
                                wb, dUall + net.offU[l], dVall + net.offV[l + 1]);
    // ybar^l = s^l * wbar (rank group 0 only in the first layer, r_1 <= 2)
    const int RGI = first ? 1 : RGM;
#pragma unroll
    for (int g = 0; g < RGM; ++g) {
      const f4 s4 = g < RGI ? *reinterpret_cast<const f4*>(sm.ss + 4 * g) : zero4();
#pragma unroll
      for (int c = 0; c < NJ; ++c) yb[c][g] = g < RGI ? s4 * wb[c][g] : zero4();
    }
  }

  // dV^1 = sum_p sum_c z^0_c ybar^1_c: z^0 = (x, t), d/dx (1, 0), d/dt (0, 1)
  {
    const int r1 = net.r[1];
    f4 vx = x * yb[0][0], vt = t * yb[0][0];
    if constexpr (NJ == 4) {
      vx += yb[1][0];
      vt += yb[2][0];
    }
    const int k = sum4_component(lane);
    const float tx = wave_sum4(vx, lane);
    const float tt = wave_sum4(vt, lane);
    float* dV1 = dVall + net.offV[1];
    if ((lane & 15) == 0 && k < r1) {
      dV1[k] = tx;
      dV1[r1 + k] = tt;
    }
  }
}

template <int RP>
constexpr int basis_waves_per_simd() {
  return 1;
}

template <int RP>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(basis_waves_per_simd<RP>()))) void lrnr_basis_kernel(
    KBasis kb) {
  extern __shared__ float4 smem_raw[];
  float* base = reinterpret_cast<float*>(smem_raw);
  const KGrid& grid = kb.grid;
  const int Wm = grid.Wmax_p;
  Smem sm;
  sm.Us = base;
  sm.Uss = sm.Us + Wm * RP;
  sm.Vs = sm.Uss + Wm * RP;
  sm.bs = sm.Vs + Wm * RP;
  sm.ss = sm.bs + Wm;
  sm.bbar = nullptr;
  sm.sbar = nullptr;
  sm.lw = nullptr;
  sm.lstride = 0;
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
  const float* s = kb.inst.s + inst_id * grid.s_stride;
  const float* mu = kb.inst.mu + 3 * inst_id;
  KTile tile;
  tile.rec = nullptr;
  tile.ck = grid.ckpt + (int64_t)blockIdx.x * kWaves * grid.ckpt_per_wave;
  tile.flag = nullptr;
  tile.stage_net = true;
  float* wrec = kb.wrec + ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * kb.PB;
  if (kind == 0)
    basis_workgroup<RP, 4>(kb, tile, wrec, kind, wg, s, mu, sm);
  else
    basis_workgroup<RP, 1>(kb, tile, wrec, kind, wg, s, mu, sm);
}

inline size_t basis_lds_bytes(int RP, int Wmax_p) {
  return ((size_t)Wmax_p * RP * 3 + Wmax_p + RP) * sizeof(float);
}

}  // namespace lrnr
