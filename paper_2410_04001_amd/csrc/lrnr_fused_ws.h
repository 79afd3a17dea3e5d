// Wave-specialised loss + gradient kernel (the LRNR / FastLRNR hot path of
// arXiv 2410.04001: eq. 2.1-2.2 / 2.8 chain with jets, eq. 4.1 residual,
// eq. 3.5-3.7 loss, reverse sweep to s and b).
//
// Why: at the register footprint of rank-20 jets (about 500 registers per
// lane when one wave does everything) only one wave fits on a SIMD, and one
// wave never overlaps its MFMA and VALU work.  Here every 64-point tile is
// owned by a pair of waves on the same SIMD (waves w and w + 4 of the
// 8-wave workgroup):
//
//   forward   M wave: a = U (s y) + b for the next neuron group  (MFMA)
//             E wave: sin jets of a, then y' += V^T z              (VALU, MFMA)
//   reverse   M wave: a (recomputed) and zbar = V ybar for the next group
//             E wave: adjoint of the sin jets, db row, wbar += U^T abar
//
// a and zbar cross from M to E through a double-buffered LDS slot per pair;
// one workgroup barrier per neuron group paces the pipeline, so the M wave's
// MFMAs for group g+1 run while the E wave works on group g.  Each role holds
// only its own rank-sized state (at most about 200 registers), so two waves
// fit per SIMD.  The role loops are separate code paths with the same number
// of barriers (the hardware barrier counts waves, not program locations), so
// the register allocator sees the roles' live ranges apart.
//
// Between layers the reduced jets travel through the global checkpoint slab
// of the pair: E writes y^{l+1} (forward) and ybar^l (reverse), M reads them
// after the next barrier.
#pragma once

#include <algorithm>
#include <map>
#include <mutex>

#include "lrnr_fused_impl.h"

namespace lrnr {

constexpr int kWsWaves = 8;
constexpr int kWsThreads = 64 * kWsWaves;
constexpr int kSlotF4 = 8;                      // f4 per lane in one exchange slot
constexpr int kSlotFloats = kSlotF4 * 64 * 4;   // floats in one exchange slot

struct SmemWS {
  float* Us;
  float* Vs;
  float* bs;
  float* ss;
  float* xbuf;  // [4 pairs][2 slots][kSlotFloats]
  float* bbar;  // [4][Wmax_p]
  float* sbar;  // [4][RP]
  float* lw;    // [4][4]
};

inline size_t ws_lds_floats(int RP, int Wmax_p) {
  return (size_t)Wmax_p * RP * 2 + Wmax_p + RP + (size_t)4 * 2 * kSlotFloats +
         (size_t)4 * Wmax_p + (size_t)4 * RP + 16;
}

template <int N>
__device__ __forceinline__ void xput(float* __restrict__ slot, int lane, const f4 (&v)[N],
                                     int first = 0) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    *reinterpret_cast<f4*>(slot + ((first + i) * 64 + lane) * 4) = v[i];
}

template <int N>
__device__ __forceinline__ void xget(const float* __restrict__ slot, int lane, f4 (&v)[N],
                                     int first = 0) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    v[i] = *reinterpret_cast<const f4*>(slot + ((first + i) * 64 + lane) * 4);
}

// ---------------------------------------------------------------------------
// Forward, one hidden layer.  M: y holds s*y^l (input); E: y accumulates y^{l+1}.
// ---------------------------------------------------------------------------
template <int NJ, int RGM, int RGI>
__device__ __forceinline__ void ws_fwd_M(const SmemWS& sm, float* xb, int G, int li, int lane,
                                         f4 (&y)[NJ][RGM]) {
#pragma unroll
  for (int g = 0; g < RGI; ++g) {
    const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + 4 * g);
#pragma unroll
    for (int c = 0; c < NJ; ++c) y[c][g] *= s4;
  }
  f4 a[NJ];
  u_side<NJ, RGM, RGI>(sm.Us, sm.bs, 0, li, y, a);
  xput<NJ>(xb, lane, a);
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    if (g + 1 < G) {
      u_side<NJ, RGM, RGI>(sm.Us, sm.bs, 4 * (g + 1), li, y, a);
      xput<NJ>(xb + ((g + 1) & 1) * kSlotFloats, lane, a);
    }
    __syncthreads();
  }
}

template <int NJ, int RGM, int RGO>
__device__ __forceinline__ void ws_fwd_E(const SmemWS& sm, const float* xb, int G, int li,
                                         int lane, f4 (&y)[NJ][RGM], float& amax) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGO; ++g) y[c][g] = zero4();
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    f4 a[NJ], z[NJ];
    xget<NJ>(xb + (g & 1) * kSlotFloats, lane, a);
    sigma_fwd<NJ, false>(a, z, amax);
    v_side<NJ, RGM, RGO>(sm.Vs, 4 * g, li, z, y);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Reverse, one hidden layer.  M: ys = s*y^l and yb = ybar^{l+1}; E: wb.
// ---------------------------------------------------------------------------
template <int NJ, int RGM, int RGI, int RGO>
__device__ __forceinline__ void ws_bwd_M(const SmemWS& sm, float* xb, int G, int li, int lane,
                                         f4 (&ys)[NJ][RGM], const f4 (&yb)[NJ][RGM]) {
#pragma unroll
  for (int g = 0; g < RGI; ++g) {
    const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + 4 * g);
#pragma unroll
    for (int c = 0; c < NJ; ++c) ys[c][g] *= s4;
  }
  f4 a[NJ], zb[NJ];
  u_side<NJ, RGM, RGI>(sm.Us, sm.bs, 0, li, ys, a);
  v_rev<NJ, RGM, RGO>(sm.Vs, 0, li, yb, zb);
  xput<NJ>(xb, lane, a);
  xput<NJ>(xb, lane, zb, NJ);
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    if (g + 1 < G) {
      float* slot = xb + ((g + 1) & 1) * kSlotFloats;
      u_side<NJ, RGM, RGI>(sm.Us, sm.bs, 4 * (g + 1), li, ys, a);
      v_rev<NJ, RGM, RGO>(sm.Vs, 4 * (g + 1), li, yb, zb);
      xput<NJ>(slot, lane, a);
      xput<NJ>(slot, lane, zb, NJ);
    }
    __syncthreads();
  }
}

template <int NJ, int RGM, int RGI>
__device__ __forceinline__ void ws_bwd_E(const SmemWS& sm, const float* xb, int G, int li,
                                         int lane, f4 (&wb)[NJ][RGM],
                                         float* __restrict__ bbar_row, float& amax) {
#pragma unroll
  for (int c = 0; c < NJ; ++c)
#pragma unroll
    for (int g = 0; g < RGI; ++g) wb[c][g] = zero4();
  const int comp = sum4_component(lane);
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    const float* slot = xb + (g & 1) * kSlotFloats;
    f4 a[NJ], zb[NJ], ab[NJ];
    xget<NJ>(slot, lane, a);
    xget<NJ>(slot, lane, zb, NJ);
    sigma_bwd<NJ, false>(a, zb, ab, amax);
    const float bsum = wave_sum4(ab[0], lane);
    if ((lane & 15) == 0) bbar_row[4 * g + comp] = bsum;
    ut_side<NJ, RGM, RGI>(sm.Us, 4 * g, li, ab, wb);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Workgroup driver (MODE_GRAD, fast sin/cos with range tracking)
// ---------------------------------------------------------------------------
template <int RP, int NJ, bool VJP>
__device__ void ws_run(const KNet& net, const KInst& inst, int64_t ckpt_per_wave, int Wmax_p,
                       const KTile& tile, int kind, int wg, const float* __restrict__ s,
                       const float* __restrict__ mu, const SmemWS& sm) {
  constexpr int RGM = RP / 4;
  constexpr int64_t kSlot = 4 * RGM * 64 * 4;  // floats per checkpoint slot
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 3;
  const int pair = wave & 3;
  const bool isM = wave < 4;
  const int L = net.L;

  // ---- the lane's point (both waves of a pair own the same 64 points) ----
  float x = 0.f, t = 0.f;
  bool valid = false;
  int64_t p = 0;
  if (kind == 0) {
    p = (int64_t)wg * kPtsPerWG + pair * 64 + lane;
    valid = p < inst.n_r;
    if (valid) {
      x = inst.xt_r[2 * p];
      t = inst.xt_r[2 * p + 1];
    }
  } else if (kind == 1) {
    p = (int64_t)wg * kPtsPerWG + pair * 64 + lane;
    valid = p < inst.n_0;
    if (valid) x = inst.x_0[p];
  } else {
    p = (int64_t)wg * kBcPairsPerWG + pair * 32 + (lane >> 1);
    valid = p < inst.n_b;
    x = (lane & 1) ? LRNR_TWO_PI_F : 0.f;
    if (valid) t = inst.t_b[p];
  }
  float* ckbase = tile.ck + pair * ckpt_per_wave;
  float* xb = sm.xbuf + pair * 2 * kSlotFloats;
  float amax = 0.f;

  // ---- forward sweep --------------------------------------------------------
  f4 y[NJ][RGM];
  for (int l = 1; l <= L - 1; ++l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    const int G = ((net.M[l] + 3) & ~3) / 4;
    __syncthreads();
    stage_layer<kWsThreads>(net, s, l, KI, KO, sm.Us, sm.Vs, sm.bs, sm.ss);
    __syncthreads();
    if (isM) {
      if (first)
        input_jets<NJ, RGM>(net, x, t, y);
      else
        ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, y);
      if (first)
        ws_fwd_M<NJ, RGM, 1>(sm, xb, G, li, lane, y);
      else
        ws_fwd_M<NJ, RGM, RGM>(sm, xb, G, li, lane, y);
    } else {
      if (last)
        ws_fwd_E<NJ, RGM, 1>(sm, xb, G, li, lane, y, amax);
      else
        ws_fwd_E<NJ, RGM, RGM>(sm, xb, G, li, lane, y, amax);
      if (!last) ckpt_store<NJ, RGM>(ckbase + (l - 1) * kSlot, lane, y);
    }
  }

  // ---- output layer, residual and loss adjoints (E waves) ----------------
  const float UL = net.U[net.offU[L]];
  const float sL = s[net.offS[L]];
  const float bL = net.b[net.offB[L]];
  const float cL = UL * sL;
  const int comp = sum4_component(lane);
  if (!isM) {
    float u[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) u[c] = cL * y[c][0][0];
    u[0] += bL;
    const int form = inst.form;
    float lsum = 0.f;
    float ub[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) ub[c] = 0.f;
    if constexpr (VJP) {
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
    float sLb = 0.f;
#pragma unroll
    for (int c = 0; c < NJ; ++c) sLb += ub[c] * y[c][0][0];
    const float tot = wave_sum4(f4{lsum, UL * sLb, ub[0], 0.f}, lane);
    if ((lane & 15) == 0) sm.lw[pair * 4 + comp] = tot;
    f4 ybL[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c) ybL[c] = f4{cL * ub[c], 0.f, 0.f, 0.f};
    xput<NJ>(xb, lane, ybL);
  }
  __syncthreads();

  // ---- reverse sweep --------------------------------------------------------
  float* rec = tile.rec;
  f4 yb[NJ][RGM];  // M: ybar^{l+1};  E: wbar of the current layer
  if (isM) {
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
      for (int g = 0; g < RGM; ++g) yb[c][g] = zero4();
    f4 ybL[NJ];
    xget<NJ>(xb, lane, ybL);
#pragma unroll
    for (int c = 0; c < NJ; ++c) yb[c][0] = ybL[c];
  }
  for (int l = L - 1; l >= 1; --l) {
    const bool first = l == 1, last = l == L - 1;
    const int KI = first ? 4 : RP, KO = last ? 4 : RP;
    const int G = ((net.M[l] + 3) & ~3) / 4;
    __syncthreads();
    if (l == L - 1 && tid < 4) {
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
    stage_layer<kWsThreads>(net, s, l, KI, KO, sm.Us, sm.Vs, sm.bs, sm.ss);
    __syncthreads();
    if (isM) {
      f4 ys[NJ][RGM];
      if (first)
        input_jets<NJ, RGM>(net, x, t, ys);
      else
        ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, ys);
      // ybar^{l+1} was left in slot l by the E wave at the end of layer l+1
      if (!last) ckpt_load<NJ, RGM>(ckbase + l * kSlot, lane, yb);
      if (first && last)
        ws_bwd_M<NJ, RGM, 1, 1>(sm, xb, G, li, lane, ys, yb);
      else if (first)
        ws_bwd_M<NJ, RGM, 1, RGM>(sm, xb, G, li, lane, ys, yb);
      else if (last)
        ws_bwd_M<NJ, RGM, RGM, 1>(sm, xb, G, li, lane, ys, yb);
      else
        ws_bwd_M<NJ, RGM, RGM, RGM>(sm, xb, G, li, lane, ys, yb);
    } else {
      float* brow = sm.bbar + pair * Wmax_p;
      if (first)
        ws_bwd_E<NJ, RGM, 1>(sm, xb, G, li, lane, yb, brow, amax);
      else
        ws_bwd_E<NJ, RGM, RGM>(sm, xb, G, li, lane, yb, brow, amax);
      // dL/ds^l = sum_c wbar_c * y_c, and ybar^l = s * wbar for the layer below
      f4 yl[NJ][RGM];
      if (first)
        input_jets<NJ, RGM>(net, x, t, yl);
      else
        ckpt_load<NJ, RGM>(ckbase + (l - 2) * kSlot, lane, yl);
      const int RGI = first ? 1 : RGM;
#pragma unroll
      for (int g = 0; g < RGM; ++g) {
        if (g < RGI) {
          f4 acc = zero4();
#pragma unroll
          for (int c = 0; c < NJ; ++c) acc += yb[c][g] * yl[c][g];
          const float tot = wave_sum4(acc, lane);
          if ((lane & 15) == 0) sm.sbar[pair * RP + 4 * g + comp] = tot;
        }
      }
      if (!first) {
#pragma unroll
        for (int g = 0; g < RGM; ++g) {
          const f4 s4 = *reinterpret_cast<const f4*>(sm.ss + 4 * g);
#pragma unroll
          for (int c = 0; c < NJ; ++c) yl[c][g] = s4 * yb[c][g];
        }
        // ybar^l goes to slot l-1 (y^{l+1} there is no longer needed)
        ckpt_store<NJ, RGM>(ckbase + (l - 1) * kSlot, lane, yl);
      }
    }
    __syncthreads();
    const int W = net.M[l], rl = net.r[l], Wm = Wmax_p;
    for (int i = tid; i < W; i += kWsThreads)
      rec[4 + net.r_total + net.offB[l] + i] =
          ((sm.bbar[i] + sm.bbar[Wm + i]) + sm.bbar[2 * Wm + i]) + sm.bbar[3 * Wm + i];
    for (int i = tid; i < rl; i += kWsThreads)
      rec[4 + net.offS[l] + i] =
          ((sm.sbar[i] + sm.sbar[RP + i]) + sm.sbar[2 * RP + i]) + sm.sbar[3 * RP + i];
  }
  // flag the workgroup for the accurate relaunch if any lane met |a| > kFastRange
  const bool bad = __any(!(amax <= kFastRange));
  __syncthreads();
  if (lane == 0) sm.lw[wave] = bad ? 1.f : 0.f;
  __syncthreads();
  if (tid == 0) {
    float any = 0.f;
    for (int w = 0; w < kWsWaves; ++w) any += sm.lw[w];
    *tile.flag = any > 0.f ? 1 : 0;
  }
}

// LDS carve-up of the wave-specialised kernels.
__device__ __forceinline__ SmemWS ws_smem(float* base, int Wm, int RP) {
  SmemWS sm;
  sm.Us = base;
  sm.Vs = sm.Us + Wm * RP;
  sm.bs = sm.Vs + Wm * RP;
  sm.ss = sm.bs + Wm;
  sm.xbuf = sm.ss + RP;
  sm.bbar = sm.xbuf + 4 * 2 * kSlotFloats;
  sm.sbar = sm.bbar + 4 * Wm;
  sm.lw = sm.sbar + 4 * RP;
  return sm;
}

template <int RP>
__global__ __launch_bounds__(kWsThreads) void lrnr_grad_ws_kernel(KNet net, KInst inst,
                                                                  KGrid grid) {
  extern __shared__ float4 smem_raw[];
  const SmemWS sm = ws_smem(reinterpret_cast<float*>(smem_raw), grid.Wmax_p, RP);

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
  tile.ck = grid.ckpt + (int64_t)blockIdx.x * kWaves * grid.ckpt_per_wave;
  tile.flag = grid.flags + blockIdx.x;
  if (kind == 0)
    ws_run<RP, 4, false>(net, inst, grid.ckpt_per_wave, grid.Wmax_p, tile, kind, wg, s, mu, sm);
  else
    ws_run<RP, 1, false>(net, inst, grid.ckpt_per_wave, grid.Wmax_p, tile, kind, wg, s, mu, sm);
}

template <int RP>
hipError_t launch_grad_ws(const KNet& net, const KInst& inst, const KGrid& grid,
                          hipStream_t stream) {
  const dim3 blocks((unsigned)(grid.B * grid.G_inst)), threads(kWsThreads);
  const size_t lds = ws_lds_floats(RP, grid.Wmax_p) * sizeof(float);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)lrnr_grad_ws_kernel<RP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((lrnr_grad_ws_kernel<RP>), blocks, threads, lds, stream, net, inst, grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // workgroups that met |a| > kFastRange are recomputed with ocml's sin/cos
  return launch_one<RP, MODE_GRAD, SC_ACC>(net, inst, grid, stream);
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
      ws_run<RP, 4, VJP>(T->net, T->inst, tg.ckpt_per_wave, tg.Wmax_p, kt, 0, r.wg, T->inst.s,
                         T->inst.mu, sm);
    else if constexpr (!VJP)
      ws_run<RP, 1, false>(T->net, T->inst, tg.ckpt_per_wave, tg.Wmax_p, kt, r.kind, r.wg,
                           T->inst.s, T->inst.mu, sm);
    __syncthreads();
  }
}

__device__ __forceinline__ Smem fused_smem(float* base, int Wm, int RP) {
  Smem sm;
  sm.Us = base;
  sm.Vs = sm.Us + Wm * RP;
  sm.bs = sm.Vs + Wm * RP;
  sm.ss = sm.bs + Wm;
  sm.bbar = sm.ss + RP;
  sm.sbar = sm.bbar + kWaves * Wm;
  sm.lw = sm.sbar + kWaves * RP;
  return sm;
}

template <int RP, int MODE, int SC>
__global__ __launch_bounds__(kThreads) void lrnr_table_kernel(KTableGrid tg) {
  extern __shared__ float4 smem_raw[];
  const Smem sm = fused_smem(reinterpret_cast<float*>(smem_raw), tg.Wmax_p, RP);
  const KTableHdr* hdr = reinterpret_cast<const KTableHdr*>(tg.table);
  const int n_tasks = hdr->n_tasks, n_tiles = hdr->n_tiles;
  float* ck = tg.ckpt ? tg.ckpt + (int64_t)blockIdx.x * kWaves * tg.ckpt_per_wave : nullptr;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    if constexpr (SC == SC_ACC) {
      if (tg.flags[tile] == 0) continue;  // only tiles flagged by the fast pass
    }
    const TileRef r = decode_tile(tg, n_tasks, tile);
    const KTask* T = r.task;
    if constexpr (reverse_mode(MODE))
      if (task_finished(T)) continue;
    KTile kt;
    kt.rec = tg.partials ? tg.partials + T->rec0 + (int64_t)r.local * T->P : nullptr;
    kt.ck = ck;
    kt.flag = tg.flags ? tg.flags + tile : nullptr;
    run_kind<RP, MODE, SC>(T->net, T->inst, tg.ckpt_per_wave, tg.Wmax_p, kt, r.kind, r.wg,
                           T->inst.s, T->inst.mu, sm);
    __syncthreads();
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
    const size_t lds = ws_lds_floats(RP, Wmax_p) * sizeof(float);
    return mode == MODE_VJP ? resident_grid(lrnr_grad_ws_table_kernel<RP, true>, kWsThreads, lds)
                            : resident_grid(lrnr_grad_ws_table_kernel<RP, false>, kWsThreads, lds);
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
  const size_t lds = fused_lds_bytes(RP, tg.Wmax_p);
  hipError_t e = set_lds(lrnr_table_kernel<RP, MODE, SC>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((lrnr_table_kernel<RP, MODE, SC>), dim3(grid), dim3(kThreads), lds, stream,
                     tg);
  return hipGetLastError();
}

template <int RP, bool VJP>
static hipError_t launch_table_rev(const KTableGrid& tg, int grid, hipStream_t stream) {
  const size_t lds = ws_lds_floats(RP, tg.Wmax_p) * sizeof(float);
  hipError_t e = set_lds(lrnr_grad_ws_table_kernel<RP, VJP>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((lrnr_grad_ws_table_kernel<RP, VJP>), dim3(grid), dim3(kWsThreads), lds,
                     stream, tg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // tiles that met |a| > kFastRange are recomputed with ocml's sin/cos
  return launch_table_one<RP, VJP ? MODE_VJP : MODE_GRAD, SC_ACC>(tg, grid, stream);
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
