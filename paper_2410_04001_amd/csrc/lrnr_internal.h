// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lrnr.h"

namespace lrnr {

constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kThreads = 64 * kWaves;     // threads per workgroup
constexpr int kPtsPerWG = 64 * kWaves;    // one point per lane
constexpr int kBcPairsPerWG = 32 * kWaves;
constexpr int kRedChunk = 32;             // records summed per first-stage thread

enum Mode { MODE_JETS = 0, MODE_VALUE = 1, MODE_LOSS = 2, MODE_GRAD = 3 };

// Net shape and packed parameter offsets (layer index l = 1..L).
struct KNet {
  int L;
  int M[LRNR_MAX_LAYERS + 1];
  int r[LRNR_MAX_LAYERS + 1];
  int offU[LRNR_MAX_LAYERS + 1];
  int offV[LRNR_MAX_LAYERS + 1];
  int offB[LRNR_MAX_LAYERS + 1];
  int offS[LRNR_MAX_LAYERS + 1];
  int r_total;
  int b_total;
  const float* U;
  const float* V;
  const float* b;
};

// One problem: coefficients, PDE parameters and points.  Batched launches run
// B instances that share the points; instance i reads s + i*s_stride and
// mu + 3*i.
struct KInst {
  const float* s;
  const float* mu;
  const float* xt_r;
  const float* x_0;
  const float* t_b;
  int64_t n_r, n_0, n_b;
  float wr_n, w0_n, wb_n;   // w_r / n_r, w_0 / n_0, w_b / n_b
  int form;                 // 0: squares, 1: absolute values
  float* out;               // JETS: [4][n_r]; VALUE: [n_r]
};

// Launch geometry, partial-sum records and scratch.
struct KGrid {
  int G_r, G_0, G_b;        // workgroups per instance for each point kind
  int G_inst;               // G_r + G_0 + G_b
  int B;                    // instances
  int P;                    // floats per workgroup record
  int Wmax_p;               // widest hidden layer rounded up to 4
  int64_t s_stride;
  float* partials;          // [B * G_inst][P]
  float* ckpt;              // GRAD: [B * G_inst * kWaves][ckpt_per_wave]
  int64_t ckpt_per_wave;
  int* flags;               // GRAD: [B * G_inst] workgroups that met |a| > kFastRange
};

// Record layout: [0..3) loss sums by kind, [3] unused, [4, 4 + r_total) grad s,
// [4 + r_total, 4 + r_total + b_total) grad b.
inline int record_floats(const KNet& n) { return ((4 + n.r_total + n.b_total) + 3) & ~3; }

// Supported padded ranks (compile-time tile heights of the rank dimension).
int padded_rank(int rmax);
size_t fused_lds_bytes(int RP, int Wmax_p);

hipError_t launch_fused(int RP, int mode, const KNet& net, const KInst& inst,
                        const KGrid& grid, hipStream_t stream);

struct KReduce {
  const float* partials;
  double* red1;             // [B][nchunk][P]
  int G_inst, B, P, nchunk;
  int E;                    // leading record elements to reduce (4 for loss only)
  int r_total, b_total;
  int64_t n_r, n_0, n_b;
  float w_r, w_0, w_b, lambda_loc;
  const float* s;           // [B][r_total] (for the locality term)
  const float* s_ref;       // [B][r_total] or null
  int64_t s_stride;
  float* grad_s;            // [B][r_total] or null
  float* grad_b;            // [b_total] (B == 1) or null
  float* loss;              // [B][4] or null
};

hipError_t launch_reduce(const KReduce& kr, hipStream_t stream);

// Detail text returned by lrnr_status_string for the calling thread.
void set_status_detail(const char* text);

hipError_t launch_adam(float* s, float* m, float* v, const float* g, int64_t n, int step,
                       float lr, float beta1, float beta2, float eps, hipStream_t stream);

}  // namespace lrnr
