// Task tables: host planning, the device image and the lrnr_tasks_* entry
// points.  One launch covers many instances (own net, s, mu, points and
// outputs); the kernels read the table from device memory, so the same
// launch can be replayed while the table's contents change.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lrnr_internal.h"

namespace lrnr {

namespace {

struct PinnedRing {
  void* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool used[2] = {false, false};
  size_t cap = 0;
  int next = 0;
};

// Created once per thread and never freed: the staging buffers may still be
// read by an in-flight copy when a thread ends.
PinnedRing& ring() {
  thread_local PinnedRing* r = new PinnedRing();
  return *r;
}

}  // namespace

hipError_t upload_async(void* dst, const void* src, size_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  PinnedRing& r = ring();
  const int i = r.next;
  r.next ^= 1;
  hipError_t e;
  if (n > r.cap) {
    for (int k = 0; k < 2; ++k) {
      if (r.used[k] && (e = hipEventSynchronize(r.ev[k])) != hipSuccess) return e;
      if (r.buf[k] && (e = hipHostFree(r.buf[k])) != hipSuccess) return e;
      r.buf[k] = nullptr;
      r.used[k] = false;
    }
    const size_t cap = std::max(n, (size_t)1 << 16);
    for (int k = 0; k < 2; ++k) {
      if ((e = hipHostMalloc(&r.buf[k], cap, hipHostMallocDefault)) != hipSuccess) return e;
      if (!r.ev[k] && (e = hipEventCreateWithFlags(&r.ev[k], hipEventDisableTiming)) != hipSuccess)
        return e;
    }
    r.cap = cap;
  } else if (r.used[i] && (e = hipEventSynchronize(r.ev[i])) != hipSuccess) {
    return e;
  }
  std::memcpy(r.buf[i], src, n);
  if ((e = hipMemcpyAsync(dst, r.buf[i], n, hipMemcpyHostToDevice, stream)) != hipSuccess) return e;
  if ((e = hipEventRecord(r.ev[i], stream)) != hipSuccess) return e;
  r.used[i] = true;
  return hipSuccess;
}

int table_grid(int RP, int mode, int Wmax_p) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  const auto key = std::make_tuple(dev, RP, mode, Wmax_p);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const int g = table_grid_size(RP, mode, Wmax_p);
  if (g > 0) cache[key] = g;
  return g;
}

void table_image(const TablePlan& tp, int cap, std::vector<char>& bytes) {
  const int n = (int)tp.tasks.size();
  bytes.assign((size_t)table_bytes(cap), 0);
  KTableHdr hdr{};
  hdr.n_tasks = n;
  hdr.n_tiles = tp.n_tiles;
  std::memcpy(bytes.data(), &hdr, sizeof hdr);
  std::memcpy(bytes.data() + sizeof(KTableHdr), tp.start.data(), sizeof(int) * (n + 1));
  if (n) std::memcpy(bytes.data() + table_off_tasks(cap), tp.tasks.data(), sizeof(KTask) * n);
}

}  // namespace lrnr

using namespace lrnr;

namespace {

bool valid_mode(int mode) { return mode >= MODE_JETS && mode <= MODE_VJP; }

// Validates nets and tasks and fills the host table.
int32_t plan_tasks(int mode, const lrnr_net* nets, int n_nets, const lrnr_task* tasks,
                   int n_tasks, const lrnr_loss_cfg* cfg, TablePlan* tp) {
  if (!valid_mode(mode)) return fail(LRNR_EINVAL, "mode=%d outside [0,4]", mode);
  if (!nets || n_nets < 1) return fail(LRNR_EINVAL, "no nets");
  if (!tasks || n_tasks < 1) return fail(LRNR_EINVAL, "no tasks");
  const bool lossy = mode == MODE_LOSS || mode == MODE_GRAD;
  if (lossy) {
    int32_t st = check_cfg(cfg, true);
    if (st) return st;
  }
  std::vector<KNet> kn(n_nets);
  int rp = 0, wmax = 4, lmax = 2;
  for (int i = 0; i < n_nets; ++i) {
    int RP, Wp;
    int32_t st = make_knet(&nets[i], &kn[i], &RP, &Wp);
    if (st) return st;
    rp = std::max(rp, RP);
    wmax = std::max(wmax, Wp);
    lmax = std::max(lmax, kn[i].L);
  }
  tp->RP = rp;
  tp->Wmax_p = wmax;
  tp->Lmax = lmax;
  tp->tasks.assign(n_tasks, KTask{});
  tp->start.assign(n_tasks + 1, 0);
  int64_t tiles = 0, rec = 0;
  for (int t = 0; t < n_tasks; ++t) {
    const lrnr_task& in = tasks[t];
    if (in.net < 0 || in.net >= n_nets)
      return fail(LRNR_EINVAL, "task %d: net %d outside [0,%d)", t, in.net, n_nets);
    if (!in.s) return fail(LRNR_EINVAL, "task %d: s is NULL", t);
    lrnr_points pts = in.pts;
    if (!lossy) pts.n_0 = pts.n_b = 0;
    int32_t st = check_points(&pts);
    if (st) return fail(st, "task %d: invalid points", t);
    const KNet& k = kn[in.net];
    KTask& T = tp->tasks[t];
    T.net = k;
    T.net_id = in.net;
    T.inst.s = in.s;
    T.inst.mu = in.mu;
    T.inst.xt_r = pts.xt_r;
    T.inst.x_0 = pts.x_0;
    T.inst.t_b = pts.t_b;
    T.inst.n_r = pts.n_r;
    T.inst.n_0 = pts.n_0;
    T.inst.n_b = pts.n_b;
    T.inst.out = in.out;
    T.inst.cot = in.cot;
    switch (mode) {
      case MODE_JETS:
      case MODE_VALUE:
        if (pts.n_r && !in.out) return fail(LRNR_EINVAL, "task %d: out is NULL", t);
        break;
      case MODE_VJP:
        if (!in.grad_s) return fail(LRNR_EINVAL, "task %d: grad_s is NULL", t);
        if (pts.n_r && !in.cot) return fail(LRNR_EINVAL, "task %d: cot is NULL", t);
        break;
      case MODE_LOSS:
        if (!in.loss) return fail(LRNR_EINVAL, "task %d: loss is NULL", t);
        if (!in.mu) return fail(LRNR_EINVAL, "task %d: mu is NULL", t);
        break;
      default:
        if (!in.grad_s) return fail(LRNR_EINVAL, "task %d: grad_s is NULL", t);
        if (!in.mu) return fail(LRNR_EINVAL, "task %d: mu is NULL", t);
        break;
    }
    if (lossy) {
      T.inst.form = cfg->form;
      T.inst.wr_n = pts.n_r ? (float)((double)cfg->w_r / (double)pts.n_r) : 0.f;
      T.inst.w0_n = pts.n_0 ? (float)((double)cfg->w_0 / (double)pts.n_0) : 0.f;
      T.inst.wb_n = pts.n_b ? (float)((double)cfg->w_b / (double)pts.n_b) : 0.f;
      T.w_r = cfg->w_r;
      T.w_0 = cfg->w_0;
      T.w_b = cfg->w_b;
      T.lambda_loc = cfg->lambda_loc;
      T.s_ref = in.s_ref ? in.s_ref : cfg->s_ref;
      if (T.lambda_loc != 0.f && !T.s_ref)
        return fail(LRNR_EINVAL, "task %d: lambda_loc != 0 needs s_ref", t);
    }
    T.G_r = (int)((pts.n_r + kPtsPerWG - 1) / kPtsPerWG);
    T.G_0 = (int)((pts.n_0 + kPtsPerWG - 1) / kPtsPerWG);
    T.G_b = (int)((pts.n_b + kBcPairsPerWG - 1) / kBcPairsPerWG);
    T.P = record_floats(k);
    T.rec0 = rec;
    if (reverse_mode(mode)) {
      T.grad_s = in.grad_s;
      T.grad_b = in.grad_b;
    }
    if (lossy) T.loss = in.loss;
    const int64_t G = (int64_t)T.G_r + T.G_0 + T.G_b;
    tp->start[t] = (int)tiles;
    tiles += G;
    rec += G * T.P;
    if (tiles > 0x7fffffffLL) return fail(LRNR_EUNSUPPORTED, "more than 2^31 tiles");
  }
  tp->start[n_tasks] = (int)tiles;
  tp->n_tiles = (int)tiles;
  tp->rec_floats = mode == MODE_JETS || mode == MODE_VALUE ? 0 : rec;
  if (reverse_mode(mode)) {
    tp->ckpt_per_wave = (int64_t)(lmax - 1) * 4 * (rp / 4) * 64 * 4;
    tp->grid_cap = std::min<int64_t>(tiles, kTableGridCap);
  }
  return LRNR_OK;
}

struct TaskWs {
  size_t off_table, off_partials, off_ckpt, off_flags, total;
};

TaskWs task_ws(const TablePlan& tp, int n_tasks) {
  TaskWs w{};
  size_t off = 0;
  w.off_table = off;
  off = align256(off + (size_t)table_bytes(n_tasks));
  w.off_partials = off;
  off = align256(off + (size_t)tp.rec_floats * sizeof(float));
  w.off_ckpt = off;
  off = align256(off + (size_t)tp.grid_cap * kWaves * tp.ckpt_per_wave * sizeof(float));
  w.off_flags = off;
  off = align256(off + (tp.ckpt_per_wave ? (size_t)tp.n_tiles * sizeof(int) : 0));
  w.total = std::max(off, (size_t)256);
  return w;
}

}  // namespace

extern "C" {

size_t lrnr_tasks_workspace_size(int32_t mode, const lrnr_net* nets, int32_t n_nets,
                                 const lrnr_task* tasks, int32_t n_tasks) {
  TablePlan tp;
  lrnr_loss_cfg any{0, 1.f, 1.f, 1.f, 0.f, nullptr};
  if (plan_tasks(mode, nets, n_nets, tasks, n_tasks, &any, &tp)) return 0;
  return task_ws(tp, n_tasks).total;
}

int32_t lrnr_tasks_run(int32_t mode, const lrnr_net* nets, int32_t n_nets,
                       const lrnr_task* tasks, int32_t n_tasks, const lrnr_loss_cfg* cfg,
                       void* ws, size_t ws_bytes, void* stream) {
  TablePlan tp;
  int32_t st = plan_tasks(mode, nets, n_nets, tasks, n_tasks, cfg, &tp);
  if (st) return st;
  const TaskWs w = task_ws(tp, n_tasks);
  if (!ws || ws_bytes < w.total)
    return fail(LRNR_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, w.total);
  if ((uintptr_t)ws & 255) return fail(LRNR_EINVAL, "workspace not 256-byte aligned");
  char* base = static_cast<char*>(ws);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  std::vector<char> img;
  table_image(tp, n_tasks, img);
  hipError_t e = upload_async(base + w.off_table, img.data(), img.size(), hs);
  if (e != hipSuccess) return hip_fail(e, "task table upload");
  KTableGrid tg{};
  tg.table = base + w.off_table;
  tg.off_tasks = table_off_tasks(n_tasks);
  tg.partials = tp.rec_floats ? reinterpret_cast<float*>(base + w.off_partials) : nullptr;
  tg.ckpt = tp.ckpt_per_wave ? reinterpret_cast<float*>(base + w.off_ckpt) : nullptr;
  tg.ckpt_per_wave = tp.ckpt_per_wave;
  tg.flags = tp.ckpt_per_wave ? reinterpret_cast<int*>(base + w.off_flags) : nullptr;
  tg.Wmax_p = tp.Wmax_p;
  tg.res_layers = resident_layers(tp.RP, tp.Wmax_p, tp.Lmax);
  if (tp.n_tiles > 0) {
    int grid = table_grid(tp.RP, mode, tp.Wmax_p);
    if (grid <= 0) return fail(LRNR_EHIP, "occupancy query failed");
    grid = std::min(grid, tp.n_tiles);
    if (reverse_mode(mode)) grid = std::min(grid, tp.grid_cap);
    if ((e = launch_table(tp.RP, mode, tg, grid, hs)) != hipSuccess)
      return hip_fail(e, "task kernel launch");
  }
  if (mode == MODE_LOSS || mode == MODE_GRAD || mode == MODE_VJP) {
    if ((e = launch_table_reduce(tg, n_tasks, 1, KAdam{}, hs)) != hipSuccess)
      return hip_fail(e, "task reduction launch");
  }
  return LRNR_OK;
}

}  // extern "C"
