/*
 * drt.h -- C ABI of the MI355X (gfx950) smoothed differentiable ray tracer.
 *
 * Method: arXiv 2401.11882 (Eertmans, Jacques, Oestges), "Fully Differentiable
 * Ray Tracing via Discontinuity Smoothing for Radio Network Optimization".
 *
 * What one call computes, for every receiver r and every path candidate
 * sigma = (sigma_1..sigma_k), 0 <= k <= max_order, an ordered list of walls
 * with no wall repeated back to back (Sec. V, "exhaustive list of path
 * candidates" from a full visibility matrix):
 *   1. the image method in the relaxed scene of infinite wall lines
 *      (Sec. V and Sec. V-B): images I_0 = tx, I_i = mirror of I_{i-1}
 *      across the line of sigma_i; back-trace X_{k+1} = r, X_i = a + t_i e
 *      = X_{i+1} + u_i (I_i - X_{i+1});
 *   2. the continuous validity of Sec. V-A, with every comparison
 *      x0 > x1 replaced by s(x0 - x1; alpha), s = sigmoid(alpha x)
 *      (Eq. 3, Eq. 4) or the hard sigmoid relu6(alpha x + 3) / 6 (Eq. 5-6),
 *      AND as a product and NOT as 1 - s:
 *        V = prod_i in(t_i) in(u_i) * prod_{legs l} prod_{walls j not at
 *            the leg's ends} (1 - in(tau_lj) in(upsilon_lj)),
 *        in(x) = s(x) s(1 - x);
 *   3. the received power of Eq. 7 with the dyadic coefficient set to the
 *      identity, summed incoherently:
 *        P(r) = sum_sigma V / max(|r - I_k|^2, d_min^2);
 *   4. the loss L = -F of Sec. III, and its gradients with respect to the
 *      transmitter, every wall endpoint and (optionally) every receiver, by
 *      a hand-written adjoint (the paper obtains them by automatic
 *      differentiation, Sec. I and Sec. III).
 *
 * Conventions shared by every entry point
 *   - Pointers named *_dev are DEVICE pointers, owned by the caller; the
 *     library never frees or retains them.  Only drt_plan_create,
 *     drt_plan_set_config, drt_batched_autotune and drt_mlp_create allocate
 *     device memory, which their handle owns (the diagnostic drt_valu_peak
 *     frees what it allocates).  Pointers to drt_* structs are HOST
 *     pointers read during the call only.
 *   - Layouts: walls float32 [n_walls][4] = (ax, ay, bx, by); tx float32 [2];
 *     rx float32 [n_rx][2]; grad_walls float32 [n_walls][4] in the same
 *     order; power / grad_power float32 [n_rx].
 *   - stream is a hipStream_t (NULL = the default stream).  Compute calls
 *     only enqueue kernels on it: no allocation, no host synchronisation, no
 *     memset nodes, so they may be captured into a HIP graph.
 *   - Return value: DRT_OK (0) or a negative drt_status.  Argument checks run
 *     on the host before anything is enqueued, so a failed call leaves all
 *     outputs untouched; drt_last_error() then gives a message (thread-local).
 *     No C++ exception crosses this interface and the library never aborts.
 *   - Results are deterministic: every reduction has a fixed order, so two
 *     identical calls give bitwise-identical outputs.
 */
#ifndef DRT_H
#define DRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DRT_ABI_VERSION 2
#define DRT_MAX_ORDER 3      /* LOS + up to three reflections */
#define DRT_MAX_WALLS 1024

typedef enum drt_status {
  DRT_OK = 0,
  DRT_EINVAL = -1,      /* bad argument: sizes, alpha, order, NULL pointer */
  DRT_EWORKSPACE = -2,  /* workspace NULL or smaller than drt_workspace_size */
  DRT_ENOTSUP = -3,     /* option not implemented */
  DRT_EHIP = -4         /* a HIP runtime call failed */
} drt_status;

typedef enum drt_smoothing {
  DRT_SIGMOID = 0,      /* Eq. 4: 1 / (1 + exp(-alpha x)) */
  DRT_HARD_SIGMOID = 1  /* Eq. 5-6: relu6(alpha x + 3) / 6; every factor is exactly 0 or 1
                           beyond 3 / alpha of its interval's ends, no transcendentals */
} drt_smoothing;

typedef enum drt_loss {
  DRT_LOSS_NONE = 0,               /* no loss, no seed */
  DRT_LOSS_SUM_POWER = 1,          /* L = sum_r P(r) */
  DRT_LOSS_NEG_MEAN_LOG_POWER = 2, /* L = -(1/R) sum_r log(P(r) + log_eps) */
  DRT_LOSS_NEG_MIN_POWER = 3       /* L = -min_r P(r): the objective of Eq. 8 (Sec. VII), to be
                                      maximised, as a loss; dL/dP = -1 at the lowest receiver
                                      index attaining the minimum, 0 elsewhere.  Needs n_rx >= 1
                                      (batched: 1 <= n_rx <= 64 in every scene). */
} drt_loss;

/* One scene.  All array pointers are device pointers. */
typedef struct drt_scene {
  const float* walls_dev;  /* [n_walls][4]; the box walls are ordinary walls */
  int32_t n_walls;         /* 0 .. DRT_MAX_WALLS (0 = free space, LOS only) */
  const float* tx_dev;     /* [2] transmitter */
  const float* rx_dev;     /* [n_rx][2] receivers, or NULL for the receiver
                              grid: the cell centres ((i + 1/2) / nx,
                              (j + 1/2) / ny) of an nx x ny grid over [0, 1]^2,
                              index m = j nx + i, nx = rx_grid_nx,
                              ny = n_rx / nx, computed in FP64 and rounded
                              once to FP32 (the grid needs rx_grid_nx > 0) */
  int32_t n_rx;            /* >= 0 */
  int32_t rx_grid_nx;      /* 0, or the row length when the receivers form a
                              row-major grid (index j*nx + i) with nx % 8 == 0
                              and n_rx % (8*nx) == 0: then each wavefront
                              takes an 8x8 block of neighbouring receivers.
                              With rx_dev given only the work order changes,
                              never the result. */
  int32_t max_order;       /* K, 0 .. DRT_MAX_ORDER */
  float alpha;             /* smoothing sharpness, finite and > 0 (Eq. 3) */
  int32_t smoothing;       /* drt_smoothing */
  float d_min;             /* distance floor, finite and > 0 (e.g. 1e-3) */
} drt_scene;

/* ABI version compiled into the library (DRT_ABI_VERSION). */
int drt_abi_version(void);

/* Static text for a drt_status value. */
const char* drt_status_string(int status);

/* Message of the last failed call on this thread ("" if none). */
const char* drt_last_error(void);

/* Number of candidates 1 + sum_{k=1..K} W (W-1)^(k-1) (Sec. V); host only.
   Returns DRT_EINVAL for out-of-range arguments. */
int drt_num_candidates(int32_t n_walls, int32_t max_order, int64_t* count);

/* Launch-shape override for the tracer kernels (a tuning knob; results do
   not depend on it beyond float summation order).  nw = wavefronts per
   workgroup (0 = automatic, else 2, 4, 8 or 16); cchunk = consecutive
   candidates handed to one wavefront (0 = automatic).  Process-wide. */
int drt_set_launch_config(int32_t nw, int32_t cchunk);

/* Upper bound (bytes) on the contribution cache that drt_workspace_size
   reserves: drt_forward records, per wavefront, the candidates with a
   nonzero contribution and their per-receiver values, so that the adjoint
   can start from them instead of re-evaluating the forward.  A smaller
   limit only costs speed (overflowing wavefronts re-evaluate); 0 disables
   the cache.  Default 32 GiB.  Process-wide; affects later size queries. */
int drt_set_cache_limit(int64_t bytes);

/* Candidate screen on (1, default) or off (0).  With the screen on, each
   wavefront first tests 64 candidates at a time against the bounding box of
   its receivers and drops those whose interaction factor is provably
   exactly 0 at every receiver of the box (a back-trace parameter beyond the
   range where exp(-alpha x) overflows FP32; Sec. V-A, Eq. 3-4).  The same
   switch controls the wall culling of the 2D calls (single scene and
   batched: a (wall, leg) test is skipped when a separating-axis test proves
   the wall's band-extended segment misses the leg's box, so its factor is
   exactly 1 in every lane) and the panel culling of the 3D calls.  None of
   them changes any result beyond the summation order of zero terms; with the
   switch off every (wall, leg) test is evaluated, which exists to verify
   that.  Process-wide. */
int drt_set_screen(int32_t enabled);

/* Contribution cut on (1, default) or off (0), for the 2D calls (single
   scene and batched) and the 3D calls with the sigmoid smoothing (hard-sigmoid
   factors are already exactly 0 beyond a band of 3/alpha; those calls never
   cut).  With the cut on, a receiver drops a candidate as soon as the
   candidate's contribution is provably at most 2^-24 / C times a lower bound
   of that receiver's power, C being the scene's candidate count; the bound is
   the sum of its order-0 and order-1 contributions plus the running sum of the
   candidates already evaluated by the same wavefront (every term is >= 0).
   The forward may stop a candidate's obstruction tests there.  The dropped
   terms of a receiver add up to at most 2^-24 P(r): no more than one FP32
   rounding of P.  Decisions depend only on the receiver, the candidate order
   and the launch shape, so results stay deterministic; the adjoint
   differentiates what the forward summed.  Turning the cut off gives the
   exact (uncut) sums, to verify the bound.  Process-wide. */
int drt_set_cut(int32_t enabled);

/* Workspace bytes that drt_forward / drt_backward / drt_forward_backward
   need for this scene (depends on n_walls, n_rx and the launch shape).
   Host only; reads no device memory. */
int drt_workspace_size(const drt_scene* scene, size_t* bytes);

/* Layout of the contribution cache inside a workspace for this scene under
   the current launch settings (host only; for verification tools).
   slots      wavefront slots, slot = tile * nw + wave;
   capacity   entries per slot (0: no cache);
   off_idx    byte offset of the candidate index lists, int32 [slots][capacity],
              each in increasing candidate order;
   off_n      byte offset of the per-slot counts, int32 [slots] (-1: the slot
              overflowed its capacity).
   The contents are those of the last drt_forward with a seed or of
   drt_forward_backward on that workspace. */
int drt_cache_layout(const drt_scene* scene, int64_t* slots, int64_t* capacity, int64_t* off_idx,
                     int64_t* off_n);

/* Forward pass (steps 1-3 above, and 4's loss value).
   power_dev   out [n_rx]      P(r).
   loss_dev    out [1] or NULL L for loss_kind (ignored for DRT_LOSS_NONE).
   seed_dev    out [n_rx] or NULL: dL/dP(r) for loss_kind.
   log_eps     > 0, the floor inside the log (DRT_LOSS_NEG_MEAN_LOG_POWER).
   ws_dev      workspace of at least drt_workspace_size bytes. */
int drt_forward(const drt_scene* scene, int32_t loss_kind, float log_eps,
                float* power_dev, float* loss_dev, float* seed_dev,
                void* ws_dev, size_t ws_bytes, void* stream);

/* Adjoint pass: given grad_power_dev = dL/dP(r) [n_rx], writes
   grad_tx_dev [2], grad_walls_dev [n_walls][4] and, if not NULL,
   grad_rx_dev [n_rx][2].  Outputs are overwritten, not accumulated.
   flags: 0, or DRT_BWD_REUSE_FORWARD when the workspace still holds what
   the last drt_forward on this same scene (same device inputs, same
   workspace, nothing changed since) recorded; the adjoint then starts from
   the recorded contributions and the wall records the forward prepared.
   With any other history the flag gives wrong gradients: pass 0. */
#define DRT_BWD_REUSE_FORWARD 1
int drt_backward(const drt_scene* scene, const float* grad_power_dev, int32_t flags,
                 float* grad_tx_dev, float* grad_walls_dev, float* grad_rx_dev,
                 void* ws_dev, size_t ws_bytes, void* stream);

/* Forward, loss seed and adjoint in one call (loss_kind must not be NONE).
   Any of grad_rx_dev / loss_dev may be NULL. */
int drt_forward_backward(const drt_scene* scene, int32_t loss_kind, float log_eps,
                         float* power_dev, float* loss_dev,
                         float* grad_tx_dev, float* grad_walls_dev, float* grad_rx_dev,
                         void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   computation as drt_forward_backward, with the workspace taken from a
   64 MiB scratch array that the library holds in each device's memory for
   the life of the process (no hipMalloc, hipFree or allocating call, no
   workspace argument).  Arguments, outputs and errors as drt_forward_backward;
   a scene whose workspace without the contribution cache exceeds 64 MiB
   (about n_rx x (4 + n_walls / 4) bytes: seed, loss and gradient partials) is rejected with
   DRT_EINVAL before anything is enqueued.  The contribution cache gets the
   rest of the array, so wavefronts that overflow it re-evaluate (power is
   bitwise that of drt_forward_backward; gradients agree to FP32 accuracy,
   bitwise with drt_set_cut(0)).  Every call on one device shares that
   device's array: calls that overlap on one device (another stream, another
   thread) race and give wrong results; serialise them.  The first call on a
   device looks up the array's address there (host-side, no allocation). */
int drt_forward_backward_noalloc(const drt_scene* scene, int32_t loss_kind, float log_eps,
                                 float* power_dev, float* loss_dev,
                                 float* grad_tx_dev, float* grad_walls_dev, float* grad_rx_dev,
                                 void* stream);

/* Forward pass with Fermat path tracing instead of the image method
   (Sec. V-B names both as path finders).  For every candidate of order 1 or
   2 the interaction points on the wall lines are found by damped Newton on
   the path length (Fermat's principle), max_iter steps at most per stage of
   a continuation that smooths the length's kinks (a leg of zero length) away
   and then restores them; line-of-sight paths are as in drt_forward.  The
   finder's convergence check compares the MPT loss L (the squared residual
   of the law of reflection summed over the interactions: 0 on a valid path,
   4 (d . n)^2 on a straight pass through a wall line) with 0, smoothed as
   s(1 - L / conv_eps) with the scene's sharpness and smoothing (Sec. V-B).
   It takes the place of the image method's side factor in(u); the other
   factors are as in drt_forward (Sec. V-A): V = prod_i in(t_i) s(1 - L /
   conv_eps) prod over legs of the obstruction factors, power
   sum V / max(l^2, d_min^2) with l the path length.
   max_iter in [1, 64] (16 is ample); conv_eps > 0 (1e-4 rejects passes
   steeper than about 0.3 degrees).  scene->max_order <= 2 (DRT_ENOTSUP
   otherwise); loss_kind NONE, SUM_POWER or NEG_MEAN_LOG_POWER; power_dev
   out [n_rx], loss_dev out [1] or NULL; workspace as drt_workspace_size.
   No contribution cut, cache or candidate screen: every candidate is
   evaluated.  Forward only (no adjoint). */
int drt_forward_fermat(const drt_scene* scene, int32_t max_iter, float conv_eps, int32_t loss_kind,
                       float log_eps, float* power_dev, float* loss_dev, void* ws_dev, size_t ws_bytes,
                       void* stream);

/* One Adam step on the transmitter (torch's Adam with bias correction)
   followed by clamping every coordinate to [lo, hi].
   tx_dev [2] in/out; grad_dev [2] in; m_dev, v_dev [2] in/out (start at 0);
   step_dev: int32 [1] in/out, the number of steps already taken (start at
   0; incremented on the device so a captured graph can be replayed).
   Needs lr > 0, 0 <= b1, b2 < 1, eps > 0, lo <= hi. */
int drt_adam_tx(float* tx_dev, const float* grad_dev, float* m_dev, float* v_dev,
                int32_t* step_dev, float lr, float b1, float b2, float eps,
                float lo, float hi, void* stream);

/* Adam on n_points points at once (2 n_points coordinates), same update and
   clamp as drt_adam_tx with one shared step counter; one launch.
   x_dev, m_dev, v_dev [n_points][2] in/out; grad_dev [n_points][2] in.
   n_points >= 1. */
int drt_adam_points(int32_t n_points, float* x_dev, const float* grad_dev, float* m_dev, float* v_dev,
                    int32_t* step_dev, float lr, float b1, float b2, float eps, float lo, float hi,
                    void* stream);

/* Geometric sharpness schedule of the transmitter optimisation (Sec. VII,
   Fig. 5: alpha grows geometrically from its first to its last value over
   the iterations).  Writes alpha_i = a_first (a_last / a_first)^(i/(n_iter-1))
   with i = min(*step_dev, n_iter - 1) into alpha_dev[0..n), reading the step
   counter on the device (the one drt_adam_points advances), so a loop of
   schedule + trace + Adam can be captured once and replayed.
   n_iter >= 2, 0 < a_first, a_last finite, n >= 1. */
int drt_alpha_schedule(const int32_t* step_dev, int32_t n_iter, float a_first, float a_last,
                       float* alpha_dev, int32_t n, void* stream);

/* ------------------------------------------------------------------------
 * Many scenes in one persistent launch
 *
 * Scenes of uneven wall count and receiver count are traced, seeded with
 * their loss and differentiated in ONE persistent kernel: work items
 * (scene, 64-receiver tile) are sorted longest first when the plan is made;
 * the workgroups that fit on the GPU pull items from a device counter.  Each
 * scene's loss is its own (mean over its receivers).  The launch shape
 * (wavefronts per workgroup, candidate chunk, workgroups per CU, tile width)
 * is chosen by drt_batched_autotune and can be stored in a text cache keyed
 * by device and batch shape.
 * ------------------------------------------------------------------------ */

/* Host-side shape of a batch, read by drt_plan_create only.  Scene s owns
   walls rows [sum_{q<s} n_walls[q], +n_walls[s]) and receivers likewise. */
typedef struct drt_batch_shape {
  int32_t n_scenes;           /* > 0 */
  const int32_t* n_walls;     /* host [n_scenes], each 0 .. DRT_MAX_WALLS */
  const int32_t* n_rx;        /* host [n_scenes], each >= 0 */
  const int32_t* rx_grid_nx;  /* host [n_scenes] or NULL: row length of a
                                 row-major receiver grid (0 = not a grid) */
  int32_t max_order;          /* K for every scene, 0 .. DRT_MAX_ORDER */
} drt_batch_shape;

/* Device data of a batch (layouts follow drt_batch_shape). */
typedef struct drt_batch {
  const float* walls_dev;  /* [sum n_walls][4] */
  const float* tx_dev;     /* [n_scenes][2] */
  const float* rx_dev;     /* [sum n_rx][2] */
  const float* alpha_dev;  /* [n_scenes], each finite and > 0 (not checked
                              on the host: it lives on the device) */
  float d_min;             /* finite, > 0 */
  int32_t smoothing;       /* drt_smoothing, the same for every scene */
} drt_batch;

/* Launch shape of a plan.  nw: 4, 8 or 16 wavefronts per workgroup; cchunk:
   1..64 consecutive candidates per wavefront turn; blocks_per_cu: persistent
   workgroups per CU (0 = as many as fit); tile_w: 8, 16 or 32 receivers per
   tile row on grid scenes. */
typedef struct drt_plan_config {
  int32_t nw, cchunk, blocks_per_cu, tile_w;
} drt_plan_config;

typedef struct drt_plan drt_plan;  /* opaque; owns its device buffers */

/* Builds the work list and allocates the plan's device buffers on the
   current device (allocates and synchronises; not for graph capture).  If
   tune_cache_path names a file with a line for this device and batch shape,
   its launch shape is used, otherwise a default.  *out must be released with
   drt_plan_destroy.  Each workgroup keeps per-wavefront gradient
   accumulators for the largest scene's walls in 64 KiB of LDS, so a batch
   whose largest scene has more than 991 walls is rejected (DRT_EINVAL); a
   launch shape that does not fit is rejected by drt_plan_set_config. */
int drt_plan_create(const drt_batch_shape* shape, const char* tune_cache_path, drt_plan** out);

/* Waits for the device, frees the plan's buffers.  NULL is a no-op. */
int drt_plan_destroy(drt_plan* plan);

/* Current launch shape (blocks_per_cu resolved). */
int drt_plan_get_config(const drt_plan* plan, drt_plan_config* cfg);

/* Sets the launch shape; may reallocate the plan's cache (synchronises). */
int drt_plan_set_config(drt_plan* plan, const drt_plan_config* cfg);

/* Work-list facts: items, total path evaluations (receivers x candidates
   summed over scenes), per-wavefront cache capacity.  Any pointer may be NULL. */
int drt_plan_info(const drt_plan* plan, int64_t* n_items, int64_t* path_evals, int32_t* cache_cap);

/* Forward, per-scene loss and adjoint of every scene in one persistent launch.
   loss_kind: DRT_LOSS_SUM_POWER or DRT_LOSS_NEG_MEAN_LOG_POWER (per scene),
   or DRT_LOSS_NONE for the power maps only (loss and gradient outputs are
   then ignored and may be NULL).
   power_dev out [sum n_rx]; loss_dev out [n_scenes] or NULL;
   grad_tx_dev out [n_scenes][2]; grad_walls_dev out [sum n_walls][4].
   Enqueues only (no allocation, no memset): graph-capturable.  Calls on the
   same plan must not overlap (they share its buffers). */
int drt_batched_forward_backward(drt_plan* plan, const drt_batch* batch, int32_t loss_kind, float log_eps,
                                 float* power_dev, float* loss_dev, float* grad_tx_dev,
                                 float* grad_walls_dev, void* stream);

/* Times every launch shape of a small grid (nw x cchunk x tile_w x
   workgroups per CU) on this batch, keeps the fastest in the plan and, if
   cache_path is not NULL, appends it there.  Synchronises; outputs hold the
   last run's results. */
int drt_batched_autotune(drt_plan* plan, const drt_batch* batch, int32_t loss_kind, float log_eps,
                         float* power_dev, float* loss_dev, float* grad_tx_dev, float* grad_walls_dev,
                         const char* cache_path, void* stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the log smoothed power map
 *
 * yhat(tx, rx) ~ log(P(rx; tx) + eps) for one scene: Fourier features
 * gamma(v) = [sin(2 pi B v), cos(2 pi B v)] of v = (tx, rx) in [0,1]^4 with a
 * fixed B [64][4] (128 inputs), then 5 ReLU layers of width 256 and a linear
 * head (296,449 parameters).  Hidden layers run as BF16 MFMA GEMMs with FP32
 * accumulation; activations are stored in BF16; master weights, biases and
 * Adam moments are FP32.  Trained by MSE on data the tracer generates
 * (drt_batched_forward_backward / drt_log_targets) and used to rank
 * transmitter positions before refinement with the exact tracer.
 *
 * Flat FP32 parameter layout (drt_mlp_num_params floats): for each hidden
 * layer l = 0..4, W_l [in][out] row-major (in = 128 for l = 0, else 256;
 * out = 256) followed by b_l [256]; then the head w [256] and b [1].
 * ------------------------------------------------------------------------ */

typedef struct drt_mlp drt_mlp;  /* opaque; owns its device buffers */

/* Number of parameters (296,449). */
int drt_mlp_num_params(int64_t* n);

/* Creates a network on the current device from host arrays: fourier_B_host
   [64][4], params_host [drt_mlp_num_params] (flat layout above).  max_batch:
   rows per training step / inference chunk, a multiple of 64 (<= 2^24);
   the handle allocates activation buffers for it.  Allocates and
   synchronises. */
int drt_mlp_create(const float* fourier_B_host, const float* params_host, int32_t max_batch, drt_mlp** out);
int drt_mlp_destroy(drt_mlp* mlp);

/* Host copies of the FP32 master parameters (synchronising). */
int drt_mlp_get_params(const drt_mlp* mlp, float* params_host);
int drt_mlp_set_params(drt_mlp* mlp, const float* params_host);

/* Loss L = (1/n) sum (yhat - y)^2 over rows v_dev [n][4], y_dev [n] and its
   gradient w.r.t. every parameter into grads_dev [num_params] (or NULL),
   loss into loss_dev [1] (or NULL).  n: positive multiple of 64, <= max_batch. */
int drt_mlp_grads(drt_mlp* mlp, const float* v_dev, const float* y_dev, int64_t n, float* grads_dev,
                  float* loss_dev, void* stream);

/* drt_mlp_grads followed by one Adam step (beta 0.9 / 0.999, eps 1e-8, torch
   semantics, step count kept on the device) and the BF16 weight copies. */
int drt_mlp_train_step(drt_mlp* mlp, const float* v_dev, const float* y_dev, int64_t n, float lr,
                       float* loss_dev, void* stream);

/* drt_mlp_train_step on the rows rows_dev[0..n) of v_dev / y_dev (int32
   device indices into arrays of any length; the caller keeps them in range):
   a shuffled mini-batch without gathering it first.  Same arithmetic as
   drt_mlp_train_step on the gathered rows.  n as there; rows_dev NULL is
   DRT_EINVAL. */
int drt_mlp_train_step_rows(drt_mlp* mlp, const float* v_dev, const float* y_dev, const int32_t* rows_dev,
                            int64_t n, float lr, float* loss_dev, void* stream);

/* yhat_dev [n] for inputs v_dev [n][4] (any n >= 0; processed in chunks). */
int drt_mlp_forward(drt_mlp* mlp, const float* v_dev, int64_t n, float* yhat_dev, void* stream);

/* F_dev[t] = mean over receivers rx_dev [n_rx][2] of yhat(tx_dev[t], rx), for
   t < n_tx (tx_dev [n_tx][2]).  Needs 0 < n_rx <= max_batch. */
int drt_mlp_scan(drt_mlp* mlp, const float* tx_dev, int32_t n_tx, const float* rx_dev, int32_t n_rx,
                 float* F_dev, void* stream);

/* y_dev[i] = log(power_dev[i] + eps), the surrogate's training target. */
int drt_log_targets(const float* power_dev, int64_t n, float eps, float* y_dev, void* stream);

/* Diagnostic, not part of the method: sustained FP32 VALU rates of the
   current device, measured with two throughput kernels (plain FMA chains and
   v_exp_f32 chains, a few ms each, best of three): fma_tflops in TFLOP/s
   (an FMA counts 2), exp_tlanes in 1e12 lane-operations/s.  They put the
   tracer kernels' rates in context next to the datasheet peak.  Allocates a
   32 MiB buffer, runs on the default stream and synchronises; not for
   graph capture. */
int drt_valu_peak(double* fma_tflops, double* exp_tlanes);

/* ------------------------------------------------------------------------
 * Scenes in three dimensions (Sec. VI: the method makes no assumption on
 * the number of dimensions)
 *
 * The walls become planar parallelogram panels {a + beta (b - a) +
 * gamma (c - a) : beta, gamma in [0, 1]} given by the corner a and its two
 * neighbours b and c.  Each step keeps its 2D meaning: images mirror across
 * the panel's plane (normal (b - a) x (c - a)); the back-trace meets the
 * plane at X_i = X_{i+1} + u_i (I_i - X_{i+1}) with panel coordinates
 * (beta_i, gamma_i); an interaction's factor is in(beta) in(gamma) in(u);
 * panel j obstructs a leg with 1 - in(upsilon) in(beta) in(gamma), upsilon
 * the leg parameter of the plane crossing and (beta, gamma) its panel
 * coordinates (Sec. V-A with Eq. 3-4, or the hard sigmoid of Eq. 5-6).  A panel of
 * zero area contributes no path and never obstructs; a back-trace parallel
 * to a plane gives no path; a leg parallel to a plane is not obstructed by
 * it.  Power, losses, error handling, determinism, graph capture, receiver
 * gradients and the contribution cache (drt_set_cache_limit) are as in the
 * 2D calls above.
 * ------------------------------------------------------------------------ */

#define DRT3_MAX_PANELS 256

/* One 3D scene.  All array pointers are device pointers. */
typedef struct drt3_scene {
  const float* panels_dev;  /* [n_panels][9] = (a, b, c), each (x, y, z) */
  int32_t n_panels;         /* 0 .. DRT3_MAX_PANELS */
  const float* tx_dev;      /* [3] transmitter */
  const float* rx_dev;      /* [n_rx][3] receivers */
  int32_t n_rx;             /* >= 0 */
  int32_t rx_grid_nx;       /* as drt_scene.rx_grid_nx */
  int32_t max_order;        /* K, 0 .. DRT_MAX_ORDER */
  float alpha;              /* finite and > 0 */
  int32_t smoothing;        /* drt_smoothing */
  float d_min;              /* finite and > 0 */
} drt3_scene;

/* Workspace bytes for the drt3_* compute calls on this scene (host only). */
int drt3_workspace_size(const drt3_scene* scene, size_t* bytes);

/* As drt_forward, for a 3D scene: power_dev [n_rx]; loss_dev [1] or NULL;
   seed_dev [n_rx] or NULL. */
int drt3_forward(const drt3_scene* scene, int32_t loss_kind, float log_eps, float* power_dev,
                 float* loss_dev, float* seed_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* As drt_backward: grad_tx_dev [3], grad_panels_dev [n_panels][9] (same
   order as the panels) and, if not NULL, grad_rx_dev [n_rx][3], overwritten.
   flags: 0 or DRT_BWD_REUSE_FORWARD. */
int drt3_backward(const drt3_scene* scene, const float* grad_power_dev, int32_t flags,
                  float* grad_tx_dev, float* grad_panels_dev, float* grad_rx_dev, void* ws_dev,
                  size_t ws_bytes, void* stream);

/* Forward, loss seed and adjoint in one call (loss_kind must not be NONE);
   grad_rx_dev and loss_dev may be NULL. */
int drt3_forward_backward(const drt3_scene* scene, int32_t loss_kind, float log_eps,
                          float* power_dev, float* loss_dev, float* grad_tx_dev,
                          float* grad_panels_dev, float* grad_rx_dev, void* ws_dev, size_t ws_bytes,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DRT_H */
