// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "lrnr.h"

namespace lrnr {

constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kThreads = 64 * kWaves;     // threads per workgroup
constexpr int kPtsPerWG = 64 * kWaves;    // one point per lane
constexpr int kBcPairsPerWG = 32 * kWaves;
constexpr int kRedChunk = 32;             // records summed per first-stage thread

enum Mode { MODE_JETS = 0, MODE_VALUE = 1, MODE_LOSS = 2, MODE_GRAD = 3, MODE_VJP = 4 };

// Modes that run the reverse sweep (and so checkpoint reduced jets).
constexpr bool reverse_mode(int mode) { return mode == MODE_GRAD || mode == MODE_VJP; }

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
  const float* cot;         // VJP: cotangent of the jets, [4][n_r]
};

// Where one 256-point tile keeps its record, checkpoints and range flag.
struct KTile {
  float* rec;               // [P] partial sums (LOSS, GRAD, VJP)
  float* ck;                // [kWaves][ckpt_per_wave] checkpoint slab of the workgroup
  int* flag;                // 1 if the tile met |a| > kFastRange (SC_TRACK writes it)
  bool stage_net;           // resident layers: stage the factors (else only s)
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
  int res_layers;           // single-role kernel: hidden layers whose factors sit in LDS
                            // together for the whole tile (0: staged layer by layer)
};

// Record layout: [0..3) loss sums by kind, [3] unused, [4, 4 + r_total) grad s,
// [4 + r_total, 4 + r_total + b_total) grad b.
inline int record_floats(const KNet& n) { return ((4 + n.r_total + n.b_total) + 3) & ~3; }

// ---------------------------------------------------------------------------
// Task tables: one launch over many independent instances, each with its own
// net, coefficients, PDE parameters, points and outputs.  The device table is
//   [KTableHdr][tile_start: cap + 1 ints][KTask: cap]
// with tile_start ascending (task t owns tiles [tile_start[t], tile_start[t+1])).
// Kernels run a persistent grid that strides over the tiles, so a captured
// launch stays valid while the table's contents change.
// ---------------------------------------------------------------------------
struct KTableHdr {
  int n_tasks;
  int n_tiles;
  int pad[62];
};

struct KTask {
  KNet net;
  KInst inst;
  int G_r, G_0, G_b;        // tiles of each point kind
  int P;                    // floats per record
  int64_t rec0;             // first float of the task's records in the partials
  // reduction
  float w_r, w_0, w_b, lambda_loc;
  const float* s_ref;       // [r_total] or null
  float* grad_s;            // [r_total] or null
  float* grad_b;            // [b_total] or null
  float* loss;              // [4] or null
  // fused Adam (null m: no update)
  float* s_upd;             // the coefficients to update (inst.s)
  float* m;                 // [r_total]
  float* v;                 // [r_total]
  int* step;                // Adam step counter, incremented on the device;
                            // kTaskFailed is or-ed in when the loss or its
                            // gradient turns non-finite (the task stops)
  int steps_max;            // no update once *step reaches this
  int net_id;               // tasks with equal ids share one net (factors staged once)
};

// Launch-wide constants of a table launch.
struct KTableGrid {
  const char* table;        // device table (layout above)
  int64_t off_tasks;        // byte offset of the KTask array
  float* partials;
  float* ckpt;              // [gridDim.x * kWaves][ckpt_per_wave]
  int64_t ckpt_per_wave;
  int* flags;               // [tile capacity]
  int Wmax_p;               // LDS layout width (>= every task's hidden widths)
  int res_layers;           // as in KGrid (for Lmax - 1 hidden layers)
};

inline int64_t table_off_tasks(int cap) {
  return ((int64_t)sizeof(KTableHdr) + (int64_t)(cap + 1) * 4 + 255) & ~(int64_t)255;
}
inline int64_t table_bytes(int cap) {
  return table_off_tasks(cap) + (int64_t)cap * (int64_t)sizeof(KTask);
}

// Resident workgroups of the table kernels (persistent grid), per mode.
int table_grid_size(int RP, int mode, int Wmax_p);

hipError_t launch_table(int RP, int mode, const KTableGrid& tg, int grid, hipStream_t stream);

struct KAdam {
  float lr, beta1, beta2, eps;
};

// Per-task reduction of the records (fixed FP64 order, independent of the
// other tasks) into loss, grad_s, grad_b; then the optional Adam update.
hipError_t launch_table_reduce(const KTableGrid& tg, int cap, int reduce_b, KAdam adam,
                               hipStream_t stream);

// Supported padded ranks (compile-time tile heights of the rank dimension).
int padded_rank(int rmax);
// LDS of the single-role kernel with n_slabs layer slabs (1: one layer staged
// at a time); resident_layers gives the slab count that keeps all L - 1 hidden
// layers of a net resident, or 0 when that would not fit the budget.
size_t fused_lds_bytes(int RP, int Wmax_p, int n_slabs = 1);
int resident_layers(int RP, int Wmax_p, int L);

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

// ---- host-side validation shared by the entry points (set the detail text) ----
int32_t fail(int32_t code, const char* fmt, ...);
int32_t hip_fail(hipError_t e, const char* where);
size_t align256(size_t x);
int32_t make_knet(const lrnr_net* net, KNet* k, int* RP, int* Wmax_p);
int32_t check_points(const lrnr_points* pts);
// sref_elsewhere: the locality reference may come with each task instead.
int32_t check_cfg(const lrnr_loss_cfg* cfg, bool sref_elsewhere = false);

// Persistent workgroups of a reverse-mode table launch never exceed this
// (checkpoint slabs are sized for it): three 4-wave workgroups per CU.
constexpr int kTableGridCap = 768;

// Host image of a task table and the sizes derived from it.
struct TablePlan {
  int RP = 0, Wmax_p = 4, Lmax = 2;
  int n_tiles = 0;
  int64_t rec_floats = 0;     // partial records of all tasks
  int64_t ckpt_per_wave = 0;  // reverse modes
  int grid_cap = 0;           // persistent workgroups the checkpoints allow
  std::vector<KTask> tasks;
  std::vector<int> start;     // [n_tasks + 1]
};

// Writes the device image of a table into host bytes [table_bytes(cap)].
void table_image(const TablePlan& tp, int cap, std::vector<char>& bytes);

// Asynchronous host-to-device copy through a per-thread pinned staging ring
// (the source may be reused as soon as the call returns).
hipError_t upload_async(void* dst, const void* src, size_t n, hipStream_t stream);

// Resident persistent grid for a table launch (cached per device and shape).
int table_grid(int RP, int mode, int Wmax_p);

hipError_t launch_adam(float* s, float* m, float* v, const float* g, int64_t n, int step,
                       float lr, float beta1, float beta2, float eps, hipStream_t stream);

}  // namespace lrnr
