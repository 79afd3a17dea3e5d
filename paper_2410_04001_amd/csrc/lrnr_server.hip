// Serving engine: continuous batching of new-parameter requests on the task
// tables.  Each request is solved by K Adam steps of physics-informed
// fine-tuning of s (eq. 3.5-3.7, residual of eq. 4.1) and an evaluation of
// the tuned net on a grid (the fast-phase solution of Section 3.2).
//
// Device state per request lives in one arena block (srv_sched.h gives the
// layout).  The step table holds the admitted requests in admission order;
// one engine step is [gradient kernel, accurate relaunch, per-task reduction
// + Adam], steps_per_launch of them captured once into a hipGraph whose
// kernels read the table from a fixed device address.  The host rewrites the
// table (an asynchronous copy on the same stream) only when requests join or
// leave, so graph replays see the current set.  A request's Adam step counter
// lives on the device: once it reaches K the kernels skip the request, so a
// multi-step graph never overshoots.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <vector>

#include "lrnr_internal.h"
#include "lrnr_task_status.h"
#include "srv_sched.h"

using namespace lrnr;

namespace {

constexpr int kRing = 8;           // pinned table-image buffers
constexpr int kMaxSlots = 4096;

double clock_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Model {
  KNet k;
  const float* s_init;
};

struct Req {
  lrnr_srv_request in;
  srv::Footprint fp;
  int64_t off = -1;   // arena block
  int slot = -1;
  double admitted = 0;
  int steps_issued = 0;
  bool cancelled = false;
};

struct Batch {       // requests whose evaluation and copies are queued
  std::vector<Req> reqs;
  hipEvent_t ev;
};

}  // namespace

struct lrnr_srv {
  lrnr_srv_cfg cfg{};
  std::vector<Model> models;
  int RP = 0, Wmax_p = 4, Lmax = 2, rt_max = 0;
  int64_t grid_pts = 0;
  int out_stride = 0;                 // floats per slot in the result staging
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  srv::Arena alloc;
  float* ckpt = nullptr;
  int64_t cpw = 0;
  int grid_step = 0, grid_eval = 0;
  int* flags = nullptr;
  char* table = nullptr;              // step table [table_bytes(max_slots)]
  char* etable = nullptr;             // evaluation table
  float* grid_xt = nullptr;           // [grid_pts][2]
  char* ring = nullptr;               // pinned [kRing][table_bytes(max_slots)]
  hipEvent_t ring_ev[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_next = 0;
  float* host_out = nullptr;          // pinned [max_slots][out_stride]
  float* host_mu = nullptr;           // pinned [max_slots][4]
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::mutex mu_wait;
  std::deque<Req> waiting;
  std::vector<Req> active;
  std::deque<Batch> finishing;
  std::deque<hipEvent_t> inflight;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> free_slots;
  int64_t tiles_active = 0;
  bool dirty = true;
  std::vector<lrnr_srv_done> done;
  lrnr_srv_stats st{};
  std::vector<char> img;

  KTableGrid step_grid() const {
    KTableGrid tg{};
    tg.table = table;
    tg.off_tasks = table_off_tasks(cfg.max_slots);
    tg.partials = reinterpret_cast<float*>(arena);
    tg.ckpt = ckpt;
    tg.ckpt_per_wave = cpw;
    tg.flags = flags;
    tg.Wmax_p = Wmax_p;
    tg.res_layers = resident_layers(RP, Wmax_p, Lmax);
    return tg;
  }

  KTableGrid eval_grid() const {
    KTableGrid tg{};
    tg.table = etable;
    tg.off_tasks = table_off_tasks(cfg.max_slots);
    tg.Wmax_p = Wmax_p;
    tg.res_layers = resident_layers(RP, Wmax_p, Lmax);
    return tg;
  }

  hipError_t event(hipEvent_t* e) {
    if (!ev_pool.empty()) {
      *e = ev_pool.back();
      ev_pool.pop_back();
      return hipSuccess;
    }
    return hipEventCreateWithFlags(e, hipEventDisableTiming);
  }

  // Copies a table image to the device through the pinned ring.
  hipError_t upload(char* dst, const std::vector<char>& bytes) {
    const int i = ring_next;
    ring_next = (ring_next + 1) % kRing;
    hipError_t e;
    if (ring_used[i] && (e = hipEventSynchronize(ring_ev[i])) != hipSuccess) return e;
    char* h = ring + (size_t)i * table_bytes(cfg.max_slots);
    std::memcpy(h, bytes.data(), bytes.size());
    if ((e = hipMemcpyAsync(dst, h, bytes.size(), hipMemcpyHostToDevice, stream)) != hipSuccess)
      return e;
    if ((e = hipEventRecord(ring_ev[i], stream)) != hipSuccess) return e;
    ring_used[i] = true;
    ++st.table_uploads;
    return hipSuccess;
  }

  void fill_task(const Req& r, KTask& T) const {
    const Model& md = models[r.in.model];
    char* base = arena + r.off;
    T = KTask{};
    T.net = md.k;
    T.net_id = r.in.model;
    float* s = reinterpret_cast<float*>(base + r.fp.s);
    T.inst.s = s;
    T.inst.mu = reinterpret_cast<const float*>(base + r.fp.mu);
    T.inst.xt_r = reinterpret_cast<const float*>(base + r.fp.xt);
    T.inst.x_0 = reinterpret_cast<const float*>(base + r.fp.x0);
    T.inst.t_b = reinterpret_cast<const float*>(base + r.fp.tb);
    T.inst.n_r = r.in.n_r;
    T.inst.n_0 = r.in.n_0;
    T.inst.n_b = r.in.n_b;
    const lrnr_loss_cfg& c = cfg.loss;
    T.inst.form = c.form;
    T.inst.wr_n = r.in.n_r ? (float)((double)c.w_r / (double)r.in.n_r) : 0.f;
    T.inst.w0_n = r.in.n_0 ? (float)((double)c.w_0 / (double)r.in.n_0) : 0.f;
    T.inst.wb_n = r.in.n_b ? (float)((double)c.w_b / (double)r.in.n_b) : 0.f;
    T.G_r = (int)((r.in.n_r + kPtsPerWG - 1) / kPtsPerWG);
    T.G_0 = (int)((r.in.n_0 + kPtsPerWG - 1) / kPtsPerWG);
    T.G_b = (int)((r.in.n_b + kBcPairsPerWG - 1) / kBcPairsPerWG);
    T.P = record_floats(md.k);
    T.rec0 = (r.off + r.fp.partials) / (int64_t)sizeof(float);
    T.w_r = c.w_r;
    T.w_0 = c.w_0;
    T.w_b = c.w_b;
    T.lambda_loc = c.lambda_loc;
    T.s_ref = c.lambda_loc != 0.f ? md.s_init : nullptr;
    T.loss = reinterpret_cast<float*>(base + r.fp.loss);
    T.s_upd = s;
    T.m = reinterpret_cast<float*>(base + r.fp.m);
    T.v = reinterpret_cast<float*>(base + r.fp.v);
    T.step = reinterpret_cast<int*>(base + r.fp.step);
    T.steps_max = cfg.K;
  }

  hipError_t upload_step_table() {
    TablePlan tp;
    tp.tasks.resize(active.size());
    tp.start.assign(active.size() + 1, 0);
    int tiles = 0;
    for (size_t i = 0; i < active.size(); ++i) {
      fill_task(active[i], tp.tasks[i]);
      tp.start[i] = tiles;
      tiles += active[i].fp.tiles;
    }
    tp.start[active.size()] = tiles;
    tp.n_tiles = tiles;
    table_image(tp, cfg.max_slots, img);
    return upload(table, img);
  }

  hipError_t enqueue_steps() {
    const KTableGrid tg = step_grid();
    const KAdam adam{cfg.lr, cfg.beta1, cfg.beta2, cfg.eps};
    for (int i = 0; i < cfg.steps_per_launch; ++i) {
      hipError_t e = launch_table(RP, MODE_GRAD, tg, grid_step, stream);
      if (e != hipSuccess) return e;
      if ((e = launch_table_reduce(tg, cfg.max_slots, 0, adam, stream)) != hipSuccess) return e;
    }
    return hipSuccess;
  }

  hipError_t admit(Req& r) {
    char* base = arena + r.off;
    hipError_t e;
    const Model& md = models[r.in.model];
    const int rt = md.k.r_total;
    auto h2d = [&](int64_t off, const void* src, int64_t bytes) {
      if (bytes <= 0 || e != hipSuccess) return;
      e = hipMemcpyAsync(base + off, src, (size_t)bytes, hipMemcpyHostToDevice, stream);
    };
    e = hipSuccess;
    h2d(r.fp.xt, r.in.xt_r, r.in.n_r * 8);
    h2d(r.fp.x0, r.in.x_0, r.in.n_0 * 4);
    h2d(r.fp.tb, r.in.t_b, r.in.n_b * 4);
    float* hm = host_mu + (size_t)r.slot * 4;
    hm[0] = r.in.mu[0];
    hm[1] = r.in.mu[1];
    hm[2] = r.in.mu[2];
    hm[3] = 0.f;
    h2d(r.fp.mu, hm, 16);
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyAsync(base + r.fp.s, md.s_init, (size_t)rt * 4, hipMemcpyDeviceToDevice,
                            stream)) != hipSuccess)
      return e;
    // m, v, loss, step counter start at zero (the three blocks are contiguous)
    if ((e = hipMemsetAsync(base + r.fp.m, 0, (size_t)(r.fp.v - r.fp.m) * 2, stream)) !=
        hipSuccess)
      return e;
    return hipMemsetAsync(base + r.fp.loss, 0, (size_t)(r.fp.partials - r.fp.loss), stream);
  }

  // Evaluation on the grid and the copies of the results to pinned memory.
  hipError_t finish(std::vector<Req>& reqs) {
    TablePlan tp;
    tp.tasks.resize(reqs.size());
    tp.start.assign(reqs.size() + 1, 0);
    const int g = (int)((grid_pts + kPtsPerWG - 1) / kPtsPerWG);
    for (size_t i = 0; i < reqs.size(); ++i) {
      const Req& r = reqs[i];
      KTask& T = tp.tasks[i];
      T = KTask{};
      T.net = models[r.in.model].k;
      T.net_id = r.in.model;
      char* base = arena + r.off;
      T.inst.s = reinterpret_cast<const float*>(base + r.fp.s);
      T.inst.xt_r = grid_xt;
      T.inst.n_r = grid_pts;
      T.inst.out = reinterpret_cast<float*>(base + r.fp.u);
      T.G_r = g;
      tp.start[i] = (int)(i * g);
    }
    tp.start[reqs.size()] = (int)(reqs.size() * g);
    tp.n_tiles = (int)(reqs.size() * g);
    table_image(tp, cfg.max_slots, img);
    hipError_t e = upload(etable, img);
    if (e != hipSuccess) return e;
    if ((e = launch_table(RP, MODE_VALUE, eval_grid(), std::min(grid_eval, tp.n_tiles),
                          stream)) != hipSuccess)
      return e;
    for (const Req& r : reqs) {
      float* h = host_out + (size_t)r.slot * out_stride;
      char* base = arena + r.off;
      const int rt = models[r.in.model].k.r_total;
      if ((e = hipMemcpyAsync(h, base + r.fp.u, (size_t)grid_pts * 4, hipMemcpyDeviceToHost,
                              stream)) != hipSuccess ||
          (e = hipMemcpyAsync(h + grid_pts, base + r.fp.s, (size_t)rt * 4,
                              hipMemcpyDeviceToHost, stream)) != hipSuccess ||
          (e = hipMemcpyAsync(h + grid_pts + rt_max, base + r.fp.loss, 16,
                              hipMemcpyDeviceToHost, stream)) != hipSuccess ||
          (e = hipMemcpyAsync(h + grid_pts + rt_max + 4, base + r.fp.step, 4,
                              hipMemcpyDeviceToHost, stream)) != hipSuccess)
        return e;
    }
    ++st.evals;
    return hipSuccess;
  }

  void deliver(Batch& b) {
    const double t = clock_s();
    for (Req& r : b.reqs) {
      lrnr_srv_done d{};
      d.id = r.in.id;
      d.arrival = r.in.arrival;
      d.admitted = r.admitted;
      d.done = t;
      d.model = r.in.model;
      d.tiles = r.fp.tiles;
      if (r.cancelled) {
        d.status = LRNR_SRV_CANCELLED;
        ++st.cancelled;
      } else {
        const float* h = host_out + (size_t)r.slot * out_stride;
        const int rt = models[r.in.model].k.r_total;
        if (r.in.u_out) std::memcpy(r.in.u_out, h, (size_t)grid_pts * 4);
        if (r.in.s_out) std::memcpy(r.in.s_out, h + grid_pts, (size_t)rt * 4);
        if (r.in.loss_out) std::memcpy(r.in.loss_out, h + grid_pts + rt_max, 16);
        int step;
        std::memcpy(&step, h + grid_pts + rt_max + 4, 4);
        d.status = (step & kTaskFailed) ? LRNR_SRV_NONFINITE : LRNR_SRV_OK;
        d.steps = step & ~kTaskFailed;
        if (d.status != LRNR_SRV_OK) ++st.failed;
      }
      done.push_back(d);
      alloc.release(r.off, r.fp.total);
      free_slots.push_back(r.slot);
      ++st.completed;
    }
  }

  // Cancelled admitted requests leave the step table now; their arena blocks
  // are released once the launches already queued (which may still read
  // them) have run.
  hipError_t drop_cancelled() {
    Batch b;
    std::vector<Req> keep;
    keep.reserve(active.size());
    for (Req& r : active) {
      if (r.cancelled) {
        tiles_active -= r.fp.tiles;
        b.reqs.push_back(r);
      } else {
        keep.push_back(r);
      }
    }
    if (b.reqs.empty()) return hipSuccess;
    active.swap(keep);
    dirty = true;
    hipError_t e;
    if ((e = event(&b.ev)) != hipSuccess || (e = hipEventRecord(b.ev, stream)) != hipSuccess)
      return e;
    finishing.push_back(std::move(b));
    return hipSuccess;
  }

  int32_t cancel(int64_t id) {
    {
      std::lock_guard<std::mutex> lock(mu_wait);
      for (auto it = waiting.begin(); it != waiting.end(); ++it) {
        if (it->in.id != id) continue;
        lrnr_srv_done d{};
        d.id = id;
        d.arrival = it->in.arrival;
        d.done = clock_s();
        d.model = it->in.model;
        d.tiles = it->fp.tiles;
        d.status = LRNR_SRV_CANCELLED;
        done.push_back(d);
        waiting.erase(it);
        ++st.cancelled;
        ++st.completed;
        return LRNR_OK;
      }
    }
    for (Req& r : active) {
      if (r.in.id != id || r.cancelled) continue;
      r.cancelled = true;
      return LRNR_OK;
    }
    return fail(LRNR_EINVAL, "request %lld is not waiting or tuning", (long long)id);
  }

  int32_t poll() {
    hipError_t e;
    // 1. deliver finished requests (batches complete in stream order)
    while (!finishing.empty()) {
      e = hipEventQuery(finishing.front().ev);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) return hip_fail(e, "result event");
      deliver(finishing.front());
      ev_pool.push_back(finishing.front().ev);
      finishing.pop_front();
    }
    while (!inflight.empty()) {
      e = hipEventQuery(inflight.front());
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) return hip_fail(e, "step event");
      ev_pool.push_back(inflight.front());
      inflight.pop_front();
    }
    // 2. admit waiting requests, first come first served
    {
      std::lock_guard<std::mutex> lock(mu_wait);
      while (!waiting.empty() && !free_slots.empty()) {
        Req& r = waiting.front();
        if (tiles_active + r.fp.tiles > cfg.max_tiles) break;
        const int64_t off = alloc.alloc(r.fp.total);
        if (off < 0) break;
        r.off = off;
        r.slot = free_slots.back();
        free_slots.pop_back();
        r.admitted = clock_s();
        if ((e = admit(r)) != hipSuccess) return hip_fail(e, "request admission");
        tiles_active += r.fp.tiles;
        active.push_back(r);
        waiting.pop_front();
        dirty = true;
        ++st.admitted;
      }
    }
    if (active.size() > (size_t)st.peak_active) st.peak_active = (int32_t)active.size();
    if ((e = drop_cancelled()) != hipSuccess) return hip_fail(e, "cancellation");
    // 3. queue the next step launch
    if (active.empty() || (int)inflight.size() >= cfg.max_inflight) return LRNR_OK;
    if (dirty) {
      if ((e = upload_step_table()) != hipSuccess) return hip_fail(e, "step table upload");
      dirty = false;
    }
    e = gexec ? hipGraphLaunch(gexec, stream) : enqueue_steps();
    if (e != hipSuccess) return hip_fail(e, "step launch");
    hipEvent_t ev;
    if ((e = event(&ev)) != hipSuccess || (e = hipEventRecord(ev, stream)) != hipSuccess)
      return hip_fail(e, "step event");
    inflight.push_back(ev);
    ++st.launches;
    st.steps += cfg.steps_per_launch;
    // 4. requests that reached K steps leave the table and are evaluated
    std::vector<Req> fin;
    std::vector<Req> keep;
    keep.reserve(active.size());
    for (Req& r : active) {
      r.steps_issued += cfg.steps_per_launch;
      if (r.steps_issued >= cfg.K) {
        fin.push_back(r);
        tiles_active -= r.fp.tiles;
      } else {
        keep.push_back(r);
      }
    }
    if (!fin.empty()) {
      active.swap(keep);
      dirty = true;
      if ((e = finish(fin)) != hipSuccess) return hip_fail(e, "grid evaluation");
      Batch b;
      b.reqs.swap(fin);
      if ((e = event(&b.ev)) != hipSuccess || (e = hipEventRecord(b.ev, stream)) != hipSuccess)
        return hip_fail(e, "result event");
      finishing.push_back(std::move(b));
    }
    return LRNR_OK;
  }

  void fill_stats(lrnr_srv_stats* o) {
    *o = st;
    {
      std::lock_guard<std::mutex> lock(mu_wait);
      o->waiting = (int32_t)waiting.size();
    }
    o->active = (int32_t)active.size();
    int32_t f = 0;
    for (const Batch& b : finishing) f += (int32_t)b.reqs.size();
    o->finishing = f;
    o->arena_used = alloc.used();
    o->arena_peak = alloc.peak();
  }

  void release_all() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : {(void*)arena, (void*)ckpt, (void*)flags, (void*)table, (void*)etable,
                    (void*)grid_xt})
      if (p) (void)hipFree(p);
    for (void* p : {(void*)ring, (void*)host_out, (void*)host_mu})
      if (p) (void)hipHostFree(p);
    for (hipEvent_t ev : ring_ev)
      if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : inflight) (void)hipEventDestroy(ev);
    for (Batch& b : finishing) (void)hipEventDestroy(b.ev);
    for (hipEvent_t ev : ev_pool) (void)hipEventDestroy(ev);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

int32_t check_srv_cfg(const lrnr_srv_cfg* c, std::vector<Model>* models, int* RP, int* Wp,
                      int* Lmax, int* rt_max) {
  if (!c) return fail(LRNR_EINVAL, "cfg is NULL");
  if (c->n_models < 1 || !c->models) return fail(LRNR_EINVAL, "no models");
  if (c->K < 1 || c->steps_per_launch < 1 || c->max_inflight < 1)
    return fail(LRNR_EINVAL, "K, steps_per_launch and max_inflight must be >= 1");
  if (c->max_slots < 1 || c->max_slots > kMaxSlots)
    return fail(LRNR_EINVAL, "max_slots=%d outside [1,%d]", c->max_slots, kMaxSlots);
  if (c->arena_bytes < 4096 || c->max_tiles < 1)
    return fail(LRNR_EINVAL, "arena_bytes or max_tiles too small");
  if (c->grid_nx < 1 || c->grid_nt < 2) return fail(LRNR_EINVAL, "grid needs nx >= 1, nt >= 2");
  int32_t st = check_cfg(&c->loss, true);
  if (st) return st;
  if (!(c->lr > 0.f) || !(c->beta1 >= 0.f && c->beta1 < 1.f) ||
      !(c->beta2 >= 0.f && c->beta2 < 1.f) || !(c->eps > 0.f))
    return fail(LRNR_EINVAL, "Adam hyperparameters out of range");
  models->assign(c->n_models, Model{});
  *RP = 0;
  *Wp = 4;
  *Lmax = 2;
  *rt_max = 0;
  for (int i = 0; i < c->n_models; ++i) {
    int rp, wp;
    if ((st = make_knet(&c->models[i].net, &(*models)[i].k, &rp, &wp))) return st;
    if (!c->models[i].s_init) return fail(LRNR_EINVAL, "model %d: s_init is NULL", i);
    (*models)[i].s_init = c->models[i].s_init;
    *RP = std::max(*RP, rp);
    *Wp = std::max(*Wp, wp);
    *Lmax = std::max(*Lmax, (*models)[i].k.L);
    *rt_max = std::max(*rt_max, (*models)[i].k.r_total);
  }
  return LRNR_OK;
}

srv::Footprint request_fp(const lrnr_srv_cfg* c, const KNet& k, int64_t n_r, int64_t n_0,
                          int64_t n_b) {
  return srv::footprint(n_r, n_0, n_b, k.r_total, record_floats(k),
                        (int64_t)c->grid_nx * c->grid_nt, kPtsPerWG, kBcPairsPerWG);
}

// Grid x_i = 2 pi i / nx, t_j = j / (nt - 1), t-major.
void grid_points(int nx, int nt, std::vector<float>& xt) {
  xt.resize((size_t)nx * nt * 2);
  for (int j = 0; j < nt; ++j)
    for (int i = 0; i < nx; ++i) {
      xt[((size_t)j * nx + i) * 2] = (float)(6.283185307179586 * i / nx);
      xt[((size_t)j * nx + i) * 2 + 1] = (float)((double)j / (nt - 1));
    }
}

}  // namespace

extern "C" {

double lrnr_srv_clock(void) { return clock_s(); }

int64_t lrnr_srv_footprint(const lrnr_srv_cfg* cfg, int32_t model, int64_t n_r, int64_t n_0,
                           int64_t n_b) {
  std::vector<Model> models;
  int RP, Wp, Lmax, rt;
  if (check_srv_cfg(cfg, &models, &RP, &Wp, &Lmax, &rt)) return 0;
  if (model < 0 || model >= cfg->n_models || n_r < 0 || n_0 < 0 || n_b < 0) return 0;
  return request_fp(cfg, models[model].k, n_r, n_0, n_b).total;
}

int32_t lrnr_srv_create(const lrnr_srv_cfg* cfg, lrnr_srv** out) {
  if (!out) return fail(LRNR_EINVAL, "out is NULL");
  *out = nullptr;
  lrnr_srv* S = new lrnr_srv();
  int32_t st = check_srv_cfg(cfg, &S->models, &S->RP, &S->Wmax_p, &S->Lmax, &S->rt_max);
  if (st) {
    delete S;
    return st;
  }
  S->cfg = *cfg;
  S->cfg.models = nullptr;  // copied into S->models
  S->grid_pts = (int64_t)cfg->grid_nx * cfg->grid_nt;
  // per slot: grid values, s, loss [4], the Adam step counter
  S->out_stride = (int)((S->grid_pts + S->rt_max + 5 + 63) & ~63);
  S->alloc.reset(cfg->arena_bytes);
  hipError_t e = hipSuccess;
  auto bad = [&](const char* what) {
    const int32_t code = e == hipErrorOutOfMemory ? LRNR_ENOMEM : LRNR_EHIP;
    fail(code, "%s: %s", what, hipGetErrorString(e));
    S->release_all();
    delete S;
    return code;
  };
  if ((e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking)) != hipSuccess)
    return bad("stream");
  S->grid_step = std::min(table_grid(S->RP, MODE_GRAD, S->Wmax_p), kTableGridCap);
  S->grid_eval = table_grid(S->RP, MODE_VALUE, S->Wmax_p);
  if (S->grid_step <= 0 || S->grid_eval <= 0) {
    e = hipErrorInvalidValue;
    return bad("occupancy query");
  }
  S->cpw = (int64_t)(S->Lmax - 1) * 4 * (S->RP / 4) * 64 * 4;
  const size_t tb = (size_t)table_bytes(cfg->max_slots);
  if ((e = hipMalloc(&S->arena, (size_t)S->alloc.size())) != hipSuccess) return bad("arena");
  if ((e = hipMalloc(&S->ckpt, (size_t)S->grid_step * kWaves * S->cpw * 4)) != hipSuccess)
    return bad("checkpoints");
  if ((e = hipMalloc(&S->flags, (size_t)cfg->max_tiles * 4)) != hipSuccess) return bad("flags");
  if ((e = hipMalloc(&S->table, tb)) != hipSuccess) return bad("table");
  if ((e = hipMalloc(&S->etable, tb)) != hipSuccess) return bad("table");
  if ((e = hipMalloc(&S->grid_xt, (size_t)S->grid_pts * 8)) != hipSuccess) return bad("grid");
  if ((e = hipHostMalloc(&S->ring, tb * kRing, hipHostMallocDefault)) != hipSuccess)
    return bad("pinned staging");
  if ((e = hipHostMalloc(&S->host_out, (size_t)cfg->max_slots * S->out_stride * 4,
                         hipHostMallocDefault)) != hipSuccess)
    return bad("pinned staging");
  if ((e = hipHostMalloc(&S->host_mu, (size_t)cfg->max_slots * 16, hipHostMallocDefault)) !=
      hipSuccess)
    return bad("pinned staging");
  for (int i = 0; i < kRing; ++i)
    if ((e = hipEventCreateWithFlags(&S->ring_ev[i], hipEventDisableTiming)) != hipSuccess)
      return bad("events");
  std::vector<float> g;
  grid_points(cfg->grid_nx, cfg->grid_nt, g);
  if ((e = hipMemcpy(S->grid_xt, g.data(), g.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return bad("grid upload");
  // empty tables: the kernels of a launch with no tasks exit at once
  std::vector<char> zero(tb, 0);
  if ((e = hipMemcpy(S->table, zero.data(), tb, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(S->etable, zero.data(), tb, hipMemcpyHostToDevice)) != hipSuccess)
    return bad("table init");
  // first launches outside capture (kernel attributes, code objects)
  if ((e = S->enqueue_steps()) != hipSuccess || (e = hipStreamSynchronize(S->stream)) != hipSuccess)
    return bad("warm-up");
  if (cfg->use_graph) {
    if ((e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return bad("graph capture");
    hipError_t e2 = S->enqueue_steps();
    e = hipStreamEndCapture(S->stream, &S->graph);
    if (e2 != hipSuccess) e = e2;
    if (e != hipSuccess) return bad("graph capture");
    if ((e = hipGraphInstantiate(&S->gexec, S->graph, nullptr, nullptr, 0)) != hipSuccess)
      return bad("graph instantiation");
  }
  S->free_slots.reserve(cfg->max_slots);
  for (int i = cfg->max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  *out = S;
  return LRNR_OK;
}

int32_t lrnr_srv_submit(lrnr_srv* S, const lrnr_srv_request* req) {
  if (!S || !req) return fail(LRNR_EINVAL, "NULL engine or request");
  if (req->model < 0 || req->model >= (int)S->models.size())
    return fail(LRNR_EINVAL, "model %d outside [0,%zu)", req->model, S->models.size());
  if (!std::isfinite(req->mu[0]) || !std::isfinite(req->mu[1]) || !std::isfinite(req->mu[2]))
    return fail(LRNR_EINVAL, "request %lld: non-finite mu", (long long)req->id);
  lrnr_points pts{req->xt_r, req->n_r, req->x_0, req->n_0, req->t_b, req->n_b};
  int32_t st = check_points(&pts);
  if (st) return st;
  if (!req->u_out) return fail(LRNR_EINVAL, "u_out is NULL");
  Req r;
  r.in = *req;
  r.fp = request_fp(&S->cfg, S->models[req->model].k, req->n_r, req->n_0, req->n_b);
  if (r.fp.total > S->alloc.size() || r.fp.tiles > S->cfg.max_tiles)
    return fail(LRNR_ENOMEM, "request needs %lld arena bytes and %d tiles (limits %lld, %d)",
                (long long)r.fp.total, r.fp.tiles, (long long)S->alloc.size(),
                S->cfg.max_tiles);
  std::lock_guard<std::mutex> lock(S->mu_wait);
  S->waiting.push_back(r);
  ++S->st.submitted;
  return LRNR_OK;
}

int32_t lrnr_srv_poll(lrnr_srv* S, int32_t* n_waiting, int32_t* n_active) {
  if (!S) return fail(LRNR_EINVAL, "NULL engine");
  const int32_t st = S->poll();
  if (n_waiting) {
    std::lock_guard<std::mutex> lock(S->mu_wait);
    *n_waiting = (int32_t)S->waiting.size();
  }
  if (n_active) {
    int32_t f = 0;
    for (const Batch& b : S->finishing) f += (int32_t)b.reqs.size();
    *n_active = (int32_t)S->active.size() + f;
  }
  return st;
}

int32_t lrnr_srv_cancel(lrnr_srv* S, int64_t id) {
  if (!S) return fail(LRNR_EINVAL, "NULL engine");
  return S->cancel(id);
}

int32_t lrnr_srv_take_done(lrnr_srv* S, lrnr_srv_done* out, int32_t cap, int32_t* n) {
  if (!S || !n || (cap > 0 && !out)) return fail(LRNR_EINVAL, "NULL argument");
  const int32_t k = (int32_t)std::min<size_t>(S->done.size(), cap > 0 ? (size_t)cap : 0);
  if (k) std::memcpy(out, S->done.data(), sizeof(lrnr_srv_done) * k);
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *n = k;
  return LRNR_OK;
}

int32_t lrnr_srv_get_stats(const lrnr_srv* S, lrnr_srv_stats* out) {
  if (!S || !out) return fail(LRNR_EINVAL, "NULL argument");
  const_cast<lrnr_srv*>(S)->fill_stats(out);
  return LRNR_OK;
}

int32_t lrnr_srv_destroy(lrnr_srv* S) {
  if (!S) return LRNR_OK;
  S->release_all();
  delete S;
  return LRNR_OK;
}

}  // extern "C"
