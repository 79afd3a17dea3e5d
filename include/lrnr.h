/*
 * lrnr.h - C ABI of the MI355X (gfx950) LRNR / FastLRNR physics-informed hot path.
 *
 * The library evaluates a Low Rank Neural Representation (arXiv 2410.04001,
 * Section 2.1, eq. 2.1-2.4) at collocation points together with its x-, t- and
 * xx-derivative jets, forms the convection-diffusion-reaction residual loss
 * (Section 4, eq. 4.1; loss forms of eq. 3.5-3.7) and back-propagates it to the
 * coefficients s and the biases b.  The same entry points run the FastLRNR of
 * Section 2.2 (eq. 2.6-2.8): a FastLRNR is an LRNR whose hidden widths are the
 * reduced widths r_hat, with operators (U_hat, V_hat, b_hat) from the EIM/DEIM
 * construction of eq. 2.7.
 *
 * Conventions shared by every function:
 *  - Return value: LRNR_OK (0) or a negative status; no exception crosses the ABI.
 *    lrnr_status_string() gives the text, including the HIP error of LRNR_EHIP.
 *  - Pointers marked [dev] are device memory owned by the caller; [host] are
 *    host memory.  The library never frees caller memory.
 *  - stream: a hipStream_t passed as void* (NULL = the default stream).  Calls
 *    are asynchronous on that stream; outputs are valid once it has completed.
 *    Host pointers are read before the call returns.
 *  - Determinism: for identical inputs the outputs are bitwise identical; all
 *    reductions run in a fixed order (no floating-point atomics).
 *  - Calls on distinct streams with distinct workspaces may run concurrently.
 *  - Arithmetic is FP32 on the device; cross-block sums are FP64.
 */
#ifndef LRNR_H
#define LRNR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRNR_MAX_LAYERS 8     /* L: weight layers (L-1 hidden + 1 linear output) */
#define LRNR_MAX_WIDTH 256    /* hidden widths M_l (or reduced widths r_hat_l)   */
#define LRNR_MAX_RANK 32      /* ranks r_l                                        */

enum {
  LRNR_OK = 0,
  LRNR_EINVAL = -1,       /* bad shape, rank, count or pointer                  */
  LRNR_ENOMEM = -2,       /* workspace too small or device allocation failed    */
  LRNR_EHIP = -3,         /* HIP runtime error (text via lrnr_status_string)    */
  LRNR_ESINGULAR = -4,    /* POD/DEIM breakdown (rank-deficient snapshots)      */
  LRNR_EUNSUPPORTED = -5  /* width/rank/depth above the compiled limits         */
};

/*
 * An LRNR with frozen bases (eq. 2.4).  L weight layers, widths M[0..L] with
 * M[0] = 2 (input (x, t)) and M[L] = 1 (scalar u); ranks r[1..L] (r[0] unused)
 * with 1 <= r[l] <= LRNR_MAX_RANK, r[1] <= M[0] and r[L] <= M[L].  A hidden
 * rank may exceed the widths next to it: the reduced net of a FastLRNR has
 * widths r_hat_l that may lie below r_l (eq. 2.7-2.8).  Layer l computes
 * z^l = sin(U^l diag(s^l) V^lT z^{l-1} + b^l) for l < L and the linear
 * u = U^L diag(s^L) V^LT z^{L-1} + b^L (eq. 2.1 with eq. 2.2).
 *  U [dev]: U^1..U^L concatenated, U^l row-major [M[l]][r[l]].
 *  V [dev]: V^1..V^L concatenated, V^l row-major [M[l-1]][r[l]]  (the reading
 *           of eq. 2.2 under which U diag(s) V^T has the shape of W^l).
 *  b [dev]: b^1..b^L concatenated, b^l [M[l]].
 * Coefficients s are passed separately as [r_total] = s^1..s^L concatenated.
 */
typedef struct lrnr_net {
  int32_t L;
  int32_t M[LRNR_MAX_LAYERS + 1];
  int32_t r[LRNR_MAX_LAYERS + 1];
  const float* U;
  const float* V;
  const float* b;
} lrnr_net;

/*
 * Collocation points of one loss (eq. 4.1 on Omega = (0, 2 pi) x (0, 1)):
 *  xt_r [dev] [n_r][2] interior (x, t) pairs -> residual
 *           N[u; mu] = u_t + mu_1 u_x - mu_2 u_xx - mu_3 u (1 - u);
 *  x_0  [dev] [n_0] abscissae of the initial line -> u(x, 0) - sin x;
 *  t_b  [dev] [n_b] times of the periodic boundary -> u(0, t) - u(2 pi, t).
 * Any count may be 0 (its pointer may then be NULL).
 */
typedef struct lrnr_points {
  const float* xt_r;
  int64_t n_r;
  const float* x_0;
  int64_t n_0;
  const float* t_b;
  int64_t n_b;
} lrnr_points;

/*
 * Loss form.  With phi(e) = e^2 (form 0, eq. 3.5) or |e| (form 1, eq. 3.6):
 *   loss = w_r mean phi(N) + w_0 mean phi(IC) + w_b mean phi(BC)
 *          + lambda_loc * sum |s - s_ref|                     (eq. 3.7)
 * The means run over n_r, n_0 and n_b points.  The subgradient of |e| at 0 is
 * taken as 0.  s_ref [dev] [r_total] may be NULL when lambda_loc == 0.
 */
typedef struct lrnr_loss_cfg {
  int32_t form;
  float w_r, w_0, w_b;
  float lambda_loc;
  const float* s_ref;
} lrnr_loss_cfg;

/* Opaque FastLRNR handle: owns the device copies of U_hat, V_hat, b_hat, P. */
typedef struct fastlrnr_handle fastlrnr_handle;

/*
 * Forward jets (Section 2.1 eq. 2.1-2.2, differentiated by the chain rule):
 *  s    [dev] [r_total] coefficients
 *  xt   [dev] [n][2]    points
 *  jets [dev] [4][n]    out: u, u_x, u_t, u_xx (structure of arrays)
 * n may be 0.  No workspace is needed.
 */
int32_t lrnr_forward_jets(const lrnr_net* net, const float* s, const float* xt,
                          int64_t n, float* jets, void* stream);

/* Values only: u [dev] [n] at xt [dev] [n][2] (u_FASTSOL grid evaluation of
 * Section 3.2 when s holds the fast-phase coefficients). */
int32_t lrnr_forward_value(const lrnr_net* net, const float* s, const float* xt,
                           int64_t n, float* u, void* stream);

/*
 * Reduced states (values only): for every hidden layer l = 1..L-1 the
 * r_{l+1} coordinates y^{l+1} = V^{(l+1)T} z^l of z^l = sigma(U^l (s^l * y^l)
 * + b^l) at each point.  On the net of fastlrnr_get_net these are the reduced
 * states z_hat^l of eq. 2.8; on the LRNR, the V^{(l+1)T} z^l they approximate
 * (Section 2.2), so the two calls give the FastLRNR's state error.
 *  xt [dev] [n][2];  y [dev] [sum_{l=2..L} r[l]][n] out (layer by layer,
 *  coordinate-major).  FP32, one thread per point (a diagnostic, not the hot
 *  path).  n may be 0.
 */
int32_t lrnr_reduced_states(const lrnr_net* net, const float* s, const float* xt, int64_t n,
                            float* y, void* stream);

/*
 * Workspace bytes needed by lrnr_residual_loss / lrnr_grad_s for this net and
 * these point counts (batch = number of instances; 1 for the single calls).
 * Returns 0 when the net or counts are invalid.
 */
size_t lrnr_workspace_size(const lrnr_net* net, const lrnr_points* pts, int32_t batch);

/*
 * Physics-informed loss (eq. 3.5 / 3.6 / 3.7 with the residual of eq. 4.1):
 *  mu   [dev] [3]  (mu_1, mu_2, mu_3) = (beta, nu, rho)
 *  loss [dev] [4]  out: total, interior term, initial term, boundary term
 *                  (terms include their weights; total adds the lambda term)
 *  ws   [dev] workspace of at least lrnr_workspace_size() bytes, 256-B aligned.
 */
int32_t lrnr_residual_loss(const lrnr_net* net, const float* s, const float* mu,
                           const lrnr_points* pts, const lrnr_loss_cfg* cfg,
                           float* loss, void* ws, size_t ws_bytes, void* stream);

/*
 * Loss and its gradient (reverse mode through the jets) with respect to the
 * coefficients s (the fine-tuning problem of eq. 3.5) and the biases b:
 *  grad_s [dev] [r_total]        out
 *  grad_b [dev] [sum_l M[l]]     out, may be NULL
 *  loss   [dev] [4]              out, may be NULL
 */
int32_t lrnr_grad_s(const lrnr_net* net, const float* s, const float* mu,
                    const lrnr_points* pts, const lrnr_loss_cfg* cfg,
                    float* grad_s, float* grad_b, float* loss,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * lrnr_grad_s for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, kernels and results (bitwise) as lrnr_grad_s, with the
 * workspace taken from a fixed device array inside the library instead of a
 * caller buffer.  The array holds LRNR_NOALLOC_SCRATCH_BYTES per GPU, set up
 * on the first call on each device and held until the process ends; nothing
 * is allocated or freed on any call.  Sizes whose lrnr_workspace_size exceeds
 * it return LRNR_EUNSUPPORTED before any device work (64 MiB holds the
 * 64-wide rank-8 net up to about 90,000 interior points with N/8 initial and
 * N/8 boundary points, the 256-wide rank-20 net up to about 30,000).  Every
 * call on one GPU shares that GPU's array and leaves its contents behind (no
 * part of it needs to start at zero): calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.  Other
 * arguments as lrnr_grad_s.
 */
#define LRNR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int32_t lrnr_grad_s_noalloc(const lrnr_net* net, const float* s, const float* mu,
                            const lrnr_points* pts, const lrnr_loss_cfg* cfg,
                            float* grad_s, float* grad_b, float* loss, void* stream);

/*
 * Batched loss + gradient for B instances that share the net and the point
 * set but have their own coefficients and PDE parameters:
 *  s      [dev] [B][r_total]
 *  mu     [dev] [B][3]
 *  grad_s [dev] [B][r_total]  out
 *  loss   [dev] [B][4]        out, may be NULL
 *  s_ref in cfg, when used, is [dev] [B][r_total].
 * Instance i's results equal those of lrnr_grad_s on instance i alone, bitwise.
 */
int32_t lrnr_grad_s_batched(const lrnr_net* net, int32_t B, const float* s,
                            const float* mu, const lrnr_points* pts,
                            const lrnr_loss_cfg* cfg, float* grad_s, float* loss,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * Task tables: one launch over many independent instances (the batched
 * differentiation and serving forms built around the method of Sections 2-3).
 * Each task has its own net (an index into nets[]), coefficients, PDE
 * parameters, points and outputs.  The device work runs on a persistent grid
 * that strides over 256-point tiles of all tasks; every task's reduction
 * runs in a fixed order over its own tiles only, so a task's results are
 * bitwise identical whatever other tasks share the launch, and equal those of
 * the single-instance entry points up to the order of FP32 operations.
 *
 * Modes:
 *  LRNR_MODE_JETS  out [4][n_r] = u, u_x, u_t, u_xx at pts.xt_r (as lrnr_forward_jets)
 *  LRNR_MODE_VALUE out [n_r]    = u at pts.xt_r (grid evaluation)
 *  LRNR_MODE_LOSS  loss [4] of eq. 3.5-3.7 with eq. 4.1 (as lrnr_residual_loss)
 *  LRNR_MODE_GRAD  loss [4] (nullable), grad_s [r_total], grad_b (nullable)
 *                  (as lrnr_grad_s)
 *  LRNR_MODE_VJP   grad_s [r_total] (and grad_b, nullable) of the scalar
 *                  sum_c sum_i cot[c][i] * jet_c(x_i), i.e. the vector-Jacobian
 *                  product of the forward jets with a caller cotangent.
 * JETS, VALUE and VJP read pts.xt_r and pts.n_r only.
 */
#define LRNR_MODE_JETS 0
#define LRNR_MODE_VALUE 1
#define LRNR_MODE_LOSS 2
#define LRNR_MODE_GRAD 3
#define LRNR_MODE_VJP 4

typedef struct lrnr_task {
  int32_t net;          /* index into nets[]                                        */
  int32_t reserved;     /* 0                                                        */
  const float* s;       /* [dev] [r_total] coefficients                             */
  const float* mu;      /* [dev] [3] (beta, nu, rho); LOSS and GRAD                 */
  lrnr_points pts;      /* [dev] points                                              */
  const float* s_ref;   /* [dev] [r_total] locality reference; NULL: cfg->s_ref     */
  const float* cot;     /* [dev] [4][n_r] cotangent of (u, u_x, u_t, u_xx); VJP    */
  float* out;           /* [dev] JETS [4][n_r], VALUE [n_r]                         */
  float* grad_s;        /* [dev] [r_total]; GRAD and VJP                            */
  float* grad_b;        /* [dev] [b_total] or NULL; GRAD and VJP                    */
  float* loss;          /* [dev] [4]; LOSS (required), GRAD (nullable)              */
} lrnr_task;

/*
 * Workspace bytes for lrnr_tasks_run with these nets and tasks (0 when the
 * arguments are invalid).  The size depends on the nets, point counts and
 * mode only, never on the device.
 */
size_t lrnr_tasks_workspace_size(int32_t mode, const lrnr_net* nets, int32_t n_nets,
                                 const lrnr_task* tasks, int32_t n_tasks);

/*
 * Runs one mode over n_tasks tasks (n_tasks >= 1; host arrays nets[] and
 * tasks[] are read before the call returns).  cfg (form, weights, lambda_loc)
 * applies to every task of LOSS and GRAD; it may be NULL for the other modes.
 * ws [dev]: at least lrnr_tasks_workspace_size() bytes, 256-B aligned.  Every
 * net of one call is run with the rank tile of the largest rank among them.
 */
int32_t lrnr_tasks_run(int32_t mode, const lrnr_net* nets, int32_t n_nets,
                       const lrnr_task* tasks, int32_t n_tasks, const lrnr_loss_cfg* cfg,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * Serving engine: continuous batching of new-parameter requests, each solved
 * by K steps of physics-informed fine-tuning of the coefficients s (Adam on
 * eq. 3.5-3.7 with the residual of eq. 4.1, through a FastLRNR of Section 2.2
 * for the sparse back-propagation) followed by the evaluation of the tuned
 * network on an nx x nt grid (the fast-phase solution of Section 3.2).
 *
 * Every request keeps its points, s, Adam moments, step counter, partial
 * records and grid output in one block of a device arena; a waiting request
 * is admitted (first come, first served) when a slot, an arena block of its
 * footprint and tile capacity are free.  Each engine step runs all admitted
 * requests in one task-table launch (gradient, per-task reduction and Adam),
 * captured once as a hipGraph of steps_per_launch steps and replayed; the
 * table in device memory changes only when requests join or leave.  A
 * request's results are bitwise identical whatever else is in flight.
 */
typedef struct lrnr_srv lrnr_srv;

typedef struct lrnr_srv_model {
  lrnr_net net;          /* device arrays must outlive the engine              */
  const float* s_init;   /* [dev] [r_total] starting coefficients (and the
                            locality reference of eq. 3.7)                     */
} lrnr_srv_model;

typedef struct lrnr_srv_cfg {
  int32_t n_models;
  const lrnr_srv_model* models;   /* [host] [n_models]; all ranks <= 32        */
  int32_t K;                      /* tuning steps per request (>= 1)            */
  int32_t steps_per_launch;       /* steps per graph launch (>= 1)              */
  int32_t max_slots;              /* requests admitted at once (<= 4096)        */
  int32_t max_inflight;           /* step launches queued ahead of the GPU      */
  int64_t arena_bytes;            /* device memory for request state            */
  int32_t max_tiles;              /* 256-point tiles in flight (admission cap)  */
  int32_t use_graph;              /* 1: replay a captured graph; 0: launch      */
  lrnr_loss_cfg loss;             /* s_ref is ignored (each model's s_init)     */
  float lr, beta1, beta2, eps;    /* Adam                                       */
  int32_t grid_nx, grid_nt;       /* evaluation grid x_i = 2 pi i / nx,
                                     t_j = j / (nt - 1), output [nt][nx]       */
} lrnr_srv_cfg;

typedef struct lrnr_srv_request {
  int64_t id;
  int32_t model;
  int32_t reserved;
  float mu[3];                    /* (beta, nu, rho)                            */
  double arrival;                 /* lrnr_srv_clock() time the request arrived  */
  /* [host] points; pinned memory (hipHostMalloc) keeps the copies
     asynchronous.  They must stay valid until the request completes. */
  const float* xt_r;
  int64_t n_r;
  const float* x_0;
  int64_t n_0;
  const float* t_b;
  int64_t n_b;
  float* u_out;                   /* [host] [nt * nx] grid values, written at completion */
  float* s_out;                   /* [host] [r_total] tuned s, or NULL           */
  float* loss_out;                /* [host] [4] loss at the last step, or NULL   */
} lrnr_srv_request;

/* Completion status of a request (lrnr_srv_done.status). */
#define LRNR_SRV_OK 0         /* K steps taken, outputs written                  */
#define LRNR_SRV_NONFINITE 1  /* the loss or its gradient turned non-finite at
                                 step `steps` + 1: s keeps its last finite value,
                                 the request stops tuning and its outputs
                                 (grid, s, the non-finite loss) are written     */
#define LRNR_SRV_CANCELLED 2  /* cancelled by lrnr_srv_cancel: no outputs       */

typedef struct lrnr_srv_done {
  int64_t id;
  double arrival, admitted, done;  /* lrnr_srv_clock() times (admitted = 0 for a
                                      request cancelled while waiting)          */
  int32_t model, tiles;
  int32_t status;                  /* LRNR_SRV_OK, _NONFINITE or _CANCELLED      */
  int32_t steps;                   /* Adam steps applied to s                    */
} lrnr_srv_done;

typedef struct lrnr_srv_stats {
  int64_t submitted, admitted, completed;   /* completed counts every status   */
  int64_t failed, cancelled;
  int64_t launches, steps, evals, table_uploads;
  int32_t waiting, active, finishing, peak_active;
  int64_t arena_used, arena_peak;
} lrnr_srv_stats;

/* Seconds on the engine's monotonic clock. */
double lrnr_srv_clock(void);

/* Arena bytes one request of this model and these point counts occupies
 * (0 when the arguments are invalid). */
int64_t lrnr_srv_footprint(const lrnr_srv_cfg* cfg, int32_t model, int64_t n_r, int64_t n_0,
                           int64_t n_b);

/* Creates an engine (allocates its arena and buffers, captures its graph)
 * on the current device with a stream of its own. */
int32_t lrnr_srv_create(const lrnr_srv_cfg* cfg, lrnr_srv** out);

/* Queues a request (thread-safe; validation only, no device work).
 * LRNR_EINVAL for a non-finite mu; LRNR_ENOMEM when the request can never fit
 * the arena or tile cap.  Point values are not scanned: a non-finite point
 * makes that request, and only it, complete with LRNR_SRV_NONFINITE. */
int32_t lrnr_srv_submit(lrnr_srv* srv, const lrnr_srv_request* req);

/* Cancels request id (call from the thread that polls).  A waiting request
 * completes at once; an admitted one leaves the step table before the next
 * launch and completes once the launches already queued have run; either way
 * its done record has status LRNR_SRV_CANCELLED and no outputs are written.
 * The other requests are unaffected (bitwise).  LRNR_EINVAL when id is not
 * waiting or tuning (unknown, completed, or already being evaluated). */
int32_t lrnr_srv_cancel(lrnr_srv* srv, int64_t id);

/* One scheduling pass, never waiting on the device except to bound the
 * queued launches: delivers finished requests, admits waiting ones and
 * queues the next step.  Counts of waiting and admitted requests are
 * returned through the (nullable) pointers. */
int32_t lrnr_srv_poll(lrnr_srv* srv, int32_t* n_waiting, int32_t* n_active);

/* Moves up to cap completion records into out[]; *n receives the count. */
int32_t lrnr_srv_take_done(lrnr_srv* srv, lrnr_srv_done* out, int32_t cap, int32_t* n);

int32_t lrnr_srv_get_stats(const lrnr_srv* srv, lrnr_srv_stats* out);

/* Waits for the device and frees everything the engine owns. */
int32_t lrnr_srv_destroy(lrnr_srv* srv);

/*
 * FastLRNR construction (Section 2.2, eq. 2.7; construction of Section 4):
 * snapshots of the hidden states z^l at n_snap points for each of the n_s
 * coefficient vectors, POD basis Xi^l (leading r_hat[l] left singular vectors,
 * FP64), DEIM indices P^l (greedy, ties to the smallest index) and reduced
 * operators U_hat^l = P^T U^l, b_hat^l = P^T b^l,
 * V_hat^{l+1} = (V^{(l+1)T} Xi^l (P^T Xi^l)^{-1})^T.
 *  s_snap  [dev]  [n_s][r_total]
 *  xt_snap [dev]  [n_snap][2]
 *  r_hat   [host] [L-1] reduced widths of hidden layers 1..L-1, each in
 *                 [1, min(M[l], n_s * n_snap, LRNR_MAX_WIDTH)]; a width
 *                 below the layer's rank r_l is allowed (Section 4 uses
 *                 r_hat well below r)
 *  out     [host] receives the handle; free it with fastlrnr_destroy.
 * Synchronises the stream (the selection runs on the device but its result
 * sizes the handle).  The net's device arrays are not referenced afterwards.
 */
int32_t fastlrnr_build(const lrnr_net* net, const float* s_snap, int32_t n_s,
                       const float* xt_snap, int64_t n_snap, const int32_t* r_hat,
                       fastlrnr_handle** out, void* stream);

/* Index selection of fastlrnr_build_sel. */
#define LRNR_SEL_DEIM 0  /* greedy DEIM (as fastlrnr_build)                       */
#define LRNR_SEL_QDEIM 1 /* Q-DEIM: first r_hat pivots of the column-pivoted QR of
                            Xi^T (Drmac & Gugercin 2016; the alternative the
                            fidelity study compares), ties to the smallest index */

/*
 * fastlrnr_build with a choice of index selection (LRNR_SEL_DEIM or
 * LRNR_SEL_QDEIM); the snapshots, POD basis and the reduced operators of
 * eq. 2.7 are the same for both.  Other selection values return
 * LRNR_EINVAL; LRNR_ESINGULAR as fastlrnr_build, or when Q-DEIM finds no row
 * with a nonzero remaining norm (Xi of deficient rank).
 */
int32_t fastlrnr_build_sel(const lrnr_net* net, const float* s_snap, int32_t n_s,
                           const float* xt_snap, int64_t n_snap, const int32_t* r_hat,
                           int32_t selection, fastlrnr_handle** out, void* stream);

/* Reduced net of a handle as an lrnr_net (widths r_hat, device pointers owned
 * by the handle): usable with every lrnr_* entry point. */
int32_t fastlrnr_get_net(const fastlrnr_handle* h, lrnr_net* out);

/* DEIM indices P^1..P^{L-1} concatenated into host [sum_l r_hat[l]]. */
int32_t fastlrnr_get_indices(const fastlrnr_handle* h, int32_t* P);

/*
 * SPInProp: loss and gradient with respect to s of the FastLRNR (eq. 2.8)
 * physics-informed loss (eq. 3.5 or 3.6 with the locality term of eq. 3.7).
 * Arguments as lrnr_grad_s; the workspace is sized by lrnr_workspace_size on
 * the net returned by fastlrnr_get_net.
 */
int32_t fastlrnr_grad_s(const fastlrnr_handle* h, const float* s, const float* mu,
                        const lrnr_points* pts, const lrnr_loss_cfg* cfg,
                        float* grad_s, float* loss, void* ws, size_t ws_bytes,
                        void* stream);

int32_t fastlrnr_destroy(fastlrnr_handle* h);

/*
 * Fused Adam step (Kingma & Ba; the optimiser of Section 4) on n coefficients,
 * in place, bias-corrected with the 1-based step count:
 *  s, m, v [dev] [n] updated; g [dev] [n] gradient.
 */
int32_t lrnr_adam_step(float* s, float* m, float* v, const float* g, int64_t n,
                       int32_t step, float lr, float beta1, float beta2, float eps,
                       void* stream);

/*
 * Measurement aid: the next launch of the fused loss/gradient kernel made by
 * this thread (from lrnr_residual_loss, lrnr_grad_s, lrnr_grad_s_batched or
 * fastlrnr_grad_s) is bracketed by hipEventRecord(start) and
 * hipEventRecord(stop) on the call's stream.  start and stop are hipEvent_t
 * passed as void*; NULL for both cancels a pending request.
 */
int32_t lrnr_time_next_fused(void* start_event, void* stop_event);

/*
 * Factored biases.  Section 2.1 notes that the biases can be factored like
 * the weights (and does not do it); here b^l = B^l s_b^l, so that the biases
 * too are driven by coefficients s_b while the basis B stays fixed.  A basis:
 *  L     layers (the net's L)
 *  M[l]  rows of B^l for l = 1..L (the net's widths; M[0] is not used)
 *  q[l]  columns of B^l, 0..LRNR_MAX_RANK (q[l] = 0: b^l = 0)
 *  B     [dev] layers 1..L packed, each [M[l]][q[l]] row-major
 * Coefficients s_b [sum_l q[l]] and biases b [sum_l M[l]] are packed by layer
 * (b as lrnr_net.b).  A factored-bias step is lrnr_bias_compose into the b
 * array the net points at, lrnr_grad_s with grad_b, then lrnr_bias_grad.
 */
typedef struct lrnr_bias_basis {
  int32_t L;
  int32_t M[LRNR_MAX_LAYERS + 1];
  int32_t q[LRNR_MAX_LAYERS + 1];
  const float* B;
} lrnr_bias_basis;

/* b^l = B^l s_b^l for every layer (FP64 sums over the columns in order):
 *  s_b [dev] [sum_l q[l]];  b [dev] [sum_l M[l]] out.
 * LRNR_EINVAL on a bad basis (L, M[l] > LRNR_MAX_WIDTH, q[l]) or NULL arrays. */
int32_t lrnr_bias_compose(const lrnr_bias_basis* bb, const float* s_b, float* b,
                          void* stream);

/* Chain rule through the factored bias: grad_sb^l = B^lT grad_b^l (FP64 sums
 * over the rows in order):
 *  grad_b [dev] [sum_l M[l]] (from lrnr_grad_s or a GRAD task);
 *  grad_sb [dev] [sum_l q[l]] out. */
int32_t lrnr_bias_grad(const lrnr_bias_basis* bb, const float* grad_b, float* grad_sb,
                       void* stream);

/* The reduced basis of a FastLRNR (eq. 2.7 applied to b = B s_b): for every
 * hidden layer the rows of B^l at the handle's indices P^l, B_hat^l =
 * P^lT B^l [r_hat_l][q[l]]; the output layer's B^L unchanged.
 *  full    basis of the LRNR the handle was built from (M[l] its widths)
 *  B_hat   [dev] out, sum_{l<L} r_hat_l q[l] + M[L] q[L] floats, caller-owned
 *  reduced out (host struct, may be NULL): the basis over B_hat with the
 *          reduced widths, for lrnr_bias_compose / lrnr_bias_grad with the
 *          net of fastlrnr_get_net (whose b is then replaced by the composed one).
 * LRNR_EINVAL when L or M[L] differ from the handle's net or an index is not
 * a row of B^l. */
int32_t fastlrnr_bias_basis(const fastlrnr_handle* h, const lrnr_bias_basis* full,
                            float* B_hat, lrnr_bias_basis* reduced, void* stream);

/*
 * Meta-learning of the coefficient map (Section 3.1, eq. 3.1-3.4) with the
 * bases U, V, b held fixed.  The hypernetwork s = f_hyper(mu; Theta) is a
 * network of the form of eq. 2.1 with the activation sin on its hidden
 * layers and a ReLU on its output (non-negative coefficients):
 *  K     layers, 1..LRNR_MAX_LAYERS
 *  H[k]  widths, H[0] = 3 (mu), H[K] = the net's r_total, each <= 256
 *  theta [dev] per layer k = 1..K: W_k [H[k]][H[k-1]] row-major, then c_k [H[k]]
 */
typedef struct lrnr_hyper {
  int32_t K;
  int32_t H[LRNR_MAX_LAYERS + 1];
  const float* theta;
} lrnr_hyper;

/* s [dev] [B][H[K]] out = f_hyper(mu[b]) for mu [dev] [B][3].  B = 0 is a no-op. */
int32_t lrnr_hyper_forward(const lrnr_hyper* f, int32_t B, const float* mu, float* s,
                           void* stream);

/*
 * Theta gradient of the meta objective (eq. 3.4 with fixed bases)
 *   (1/B) sum_b [ L_b(s_b) + lambda_sparse R_sparse(s_b) ],  s_b = f_hyper(mu_b),
 * given s_bar [dev] [B][r_total] = dL_b/ds_b (e.g. from lrnr_grad_s_batched at
 * s = lrnr_hyper_forward(mu)).  R_sparse (eq. 3.3) = sum_l || ReLU(Gamma^l s^l) ||_1,
 * Gamma^l [(r_l - 1) x r_l] with -1 on the diagonal and gamma above it; the
 * net supplies the ranks r_l.
 *  grad_theta [dev] out, the size of theta (overwritten, not accumulated)
 *  r_sparse   [dev] [1] out, (1/B) sum_b R_sparse(s_b); may be NULL
 *  ws         [dev] workspace of lrnr_hyper_workspace_size(f, B) bytes
 *             (per-sample gradients), 256-B aligned
 * B >= 1.  The per-sample gradients are summed over the samples in a fixed
 * order (FP64): results are bitwise reproducible.  LRNR_EINVAL on shapes that
 * do not match the net, LRNR_ENOMEM on a short workspace.
 */
int32_t lrnr_hyper_backward(const lrnr_hyper* f, const lrnr_net* net, int32_t B, const float* mu,
                            const float* s_bar, float gamma, float lambda_sparse,
                            float* grad_theta, float* r_sparse, void* ws, size_t ws_bytes,
                            void* stream);

/* Workspace bytes of lrnr_hyper_backward for B samples (0 if f or B is invalid). */
size_t lrnr_hyper_workspace_size(const lrnr_hyper* f, int32_t B);

/*
 * Truncation after meta-learning (Section 4): over B parameter samples
 * mu [dev] [B][3], coefficient k of layer l is kept when f_hyper(mu_b)[k] is
 * nonzero for some b (the ReLU output is exactly zero otherwise, decided in
 * FP32); dropped coefficients lose their columns of U^l and V^l and their
 * hypernetwork output (row of W_K, entry of c_K).  A layer with no kept
 * coefficient keeps its first one (zero at every sample, so the network is
 * unchanged).  The widths and the biases stay.
 *  r_out     [host] [L+1] out: the new ranks (r_out[0] = 0)
 *  keep      [host] [r_total] out: 1 for a kept coefficient, else 0; may be NULL
 *  U_out     [dev] out: the truncated U, packed as an lrnr_net with ranks r_out
 *                  (room for the full U); V_out likewise for V
 *  theta_out [dev] out: the truncated hypernetwork (widths H[0..K-1] and
 *                  H[K] = the new r_total; room for the full theta)
 *  ws        [dev] lrnr_truncate_workspace_size(f, B) bytes, 256-B aligned
 * Synchronises the stream (the kept set sizes the outputs).  LRNR_EINVAL when
 * f's output width differs from the net's r_total.
 */
int32_t lrnr_truncate(const lrnr_net* net, const lrnr_hyper* f, int32_t B, const float* mu,
                      int32_t* r_out, int32_t* keep, float* U_out, float* V_out,
                      float* theta_out, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of lrnr_truncate for B samples (0 if f or B is invalid). */
size_t lrnr_truncate_workspace_size(const lrnr_hyper* f, int32_t B);

/*
 * Gradient of the physics-informed loss (eq. 3.5 / 3.6 with eq. 4.1; the
 * locality term does not depend on the bases) with respect to the bases, the
 * parameters the meta-learning phase trains besides Theta and b (eq. 3.4):
 *   grad_U^l = sum_p sum_c abar^l_{p,c} (s^l * y^l_{p,c})^T,
 *   grad_V^l = sum_p sum_c z^{l-1}_{p,c} ybar^l_{p,c}^T   (c over the jets).
 *  grad_U [dev] packed as net.U, out;  grad_V [dev] packed as net.V, out
 *  ws [dev] workspace of lrnr_basis_grad_workspace_size bytes, 256-B aligned:
 *  one record of the U and V entries per wave of 64 points, and the reduced
 *  jets checkpointed between the sweeps.
 * Other arguments as lrnr_grad_s.  The terms are formed inside the fused
 * forward and reverse sweeps (FP32, one lane per point); the per-wave records
 * are summed in a fixed order in FP64 (bitwise reproducible).  LRNR_ENOMEM
 * on a short workspace.
 */
int32_t lrnr_basis_grad(const lrnr_net* net, const float* s, const float* mu,
                        const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_U,
                        float* grad_V, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of lrnr_basis_grad (0 when the net or points are invalid). */
size_t lrnr_basis_grad_workspace_size(const lrnr_net* net, const lrnr_points* pts);

/*
 * The mean over B instances (the samples of the meta objective, eq. 3.4)
 * of lrnr_basis_grad, in one launch: instance b has coefficients
 * s [dev] [B][r_total] row b and PDE parameters mu [dev] [B][3] row b, and
 * all share the net and the points.  grad_U, grad_V as lrnr_basis_grad
 * ((1/B) sum over b).  ws: lrnr_basis_grad_batched_workspace_size bytes.
 */
int32_t lrnr_basis_grad_batched(const lrnr_net* net, int32_t B, const float* s, const float* mu,
                                const lrnr_points* pts, const lrnr_loss_cfg* cfg,
                                float* grad_U, float* grad_V, void* ws, size_t ws_bytes,
                                void* stream);

size_t lrnr_basis_grad_batched_workspace_size(const lrnr_net* net, const lrnr_points* pts,
                                              int32_t B);

/* Orthogonality term of eq. 3.3 on the net's bases:
 *   R_orth = sum_l ||U^lT U^l - I||_F^2 + ||V^lT V^l - I||_F^2  (all L layers),
 * and its gradients 4 U^l (U^lT U^l - I), 4 V^l (V^lT V^l - I).
 *  value  [dev] [1] out, may be NULL
 *  grad_U [dev] packed as net.U, out, may be NULL;  grad_V as net.V, may be NULL
 * FP64 sums in a fixed order (one workgroup). */
int32_t lrnr_orth_reg(const lrnr_net* net, float* value, float* grad_U, float* grad_V,
                      void* stream);

/* Mean over samples, for the bias gradient of the meta objective (the biases
 * are shared by all samples; eq. 3.4 averages over mu): out[e] = (1/B)
 * sum_b x[b][e], summed in sample order in FP64 (bitwise reproducible).
 *  x [dev] [B][n] (e.g. the grad_b rows of B GRAD tasks);  out [dev] [n].
 * B >= 1; n may be 0. */
int32_t lrnr_rows_mean(const float* x, int32_t B, int64_t n, float* out, void* stream);

/*
 * Reference solution of the convection-diffusion-reaction problem of
 * Section 4, eq. 4.1 (u_t + mu_1 u_x - mu_2 u_xx - mu_3 u (1 - u) = 0 on
 * (0, 2 pi) periodic, u(x, 0) = sin x), for B parameter instances at once:
 * the reference against which the test-accuracy comparison of Section 4
 * measures L1 relative errors.  The paper names no solver; this one is
 * Strang splitting R(dt/2) L(dt) R(dt/2) with both sub-flows exact (L in
 * Fourier space on the uniform grid x_j = 2 pi j / n_x, R the logistic
 * flow), FP64, dt = t_end / n_t, second order in dt.
 *  mu     [dev] [B][3]           (beta, nu, rho) per instance, FP64
 *  u      [dev] [B][n_out][n_x]  out, FP64: u(x_j, t_k), t_k = k t_end / (n_out - 1)
 *  status [dev] [B]              out: 0, or the 1-based step n at which the
 *                                instance blew up (a logistic sub-flow left R,
 *                                or |u| > 1e6 or not finite); u is then NaN
 *                                at every output time at or after step n.
 * n_x is a power of two in [8, 1024]; n_out >= 2 and (n_out - 1) divides n_t.
 * One workgroup per instance; B = 0 is a no-op.  LRNR_EINVAL on bad sizes or
 * NULL pointers.  Asynchronous on the stream; no workspace.
 */
int32_t lrnr_cdr_reference(const double* mu, int32_t B, int32_t n_x, int32_t n_t,
                           int32_t n_out, double t_end, double* u, int32_t* status,
                           void* stream);

/*
 * L1 relative error of a prediction against a reference (the error measure of
 * the Section 4 comparison), as two FP64 sums taken in a fixed order:
 *  pred [dev] [n] FP32 (e.g. lrnr_forward_value on the reference grid)
 *  ref  [dev] [n] FP64
 *  out  [dev] [2] out: sum |pred - ref|, sum |ref|  (error = out[0] / out[1])
 * Results are bitwise reproducible.  n may be 0 (both sums 0).
 */
int32_t lrnr_l1_error(const float* pred, const double* ref, int64_t n, double* out,
                      void* stream);

/* Text of a status code (thread-local detail for LRNR_EHIP / LRNR_EINVAL). */
const char* lrnr_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* LRNR_H */
