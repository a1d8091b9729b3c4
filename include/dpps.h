/*
 * dpps.h -- C ABI of the MI355X passing-point search (SBIP-DPPS).
 *
 * The search is the one of arXiv 1909.07717, Sec. 4.2-4.3: for every candidate
 * point of a lattice over the field and every pass variant (kick type and
 * speed) it takes the ideal two-phase ball model of Sec. 4.1, finds each
 * robot's earliest interception along the sampled ball path (SBIP, Sec. 4.2),
 * keeps the pass when the first opponent arrives sufficiently later than the
 * first teammate (Sec. 4.3, delta-time feature), scores it with the weighted
 * sum of Eq. (3) and returns the best one (Sec. 4.3, best pass line).
 *
 * Conventions
 *   - Plain C types only.  Host pointers are read during the call and may be
 *     reused as soon as it returns.  Device pointers are allocated and owned by
 *     the caller (any HIP allocation on the context's device).
 *   - Every entry point returns 0 (DPPS_OK) or a negative DPPS_E_* code; no C++
 *     exception crosses this boundary.  dpps_strerror() names a code and
 *     dpps_last_error() describes the last failure on the calling thread.
 *   - A context is not thread safe: one context per host thread or stream, and
 *     calls on one context are serialised by the caller.
 *   - Units: metres, seconds, m/s, m/s^2, radians.  +x attacks the goal at
 *     x = goal_x.
 */
#ifndef DPPS_H
#define DPPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define DPPS_OK 0
#define DPPS_E_INVALID (-1)     /* bad argument: NaN/Inf input, count or index out of range, window
                                   outside the lattice, spacing that does not divide the field,
                                   K not 64, 128, 192 or 256, v0 <= 0, NULL where required */
#define DPPS_E_NOMEM (-2)       /* a host or device allocation failed */
#define DPPS_E_DEVICE (-3)      /* a HIP call failed (see dpps_last_error) */
#define DPPS_E_BUDGET (-4)      /* the request needs more device memory than the budget allows */
#define DPPS_E_UNSUPPORTED (-5) /* valid but not built (e.g. more than 64 variants in a frame) */

/* ---- pass variants ------------------------------------------------------ */
#define DPPS_FLAT 0 /* flat kick: slides down to slide_ratio * v0, then rolls to rest (Sec. 4.1) */
#define DPPS_CHIP 1 /* chip kick: drag-free flight at chip_angle, then rolls; not interceptable
                       in the air (Sec. 4.3 chip passes; the paper gives no chip model) */

/* ---- output modes (dpps_params.out_flags) ------------------------------ */
#define DPPS_OUT_REDUCED 1u /* per point only: score = best over variants, mask = that variant's
                               index (255: none); layout window-major [ny][nx] */

#define DPPS_MAX_SIDE 16     /* robots per team (the paper assumes 16 a side, Sec. 4.2) */
#define DPPS_MAX_VARIANTS 64 /* pass variants per frame */

typedef struct dpps_ctx dpps_ctx;
typedef struct dpps_batch dpps_batch;

/* Robot state: position (m) and velocity (m/s). */
typedef struct {
    float x, y, vx, vy;
} dpps_robot;

/* A window of the field-centred lattice of spacing h.  The full lattice has
 * Nx = round(field_len/h) + 1 by Ny = round(field_wid/h) + 1 points (h must
 * divide both field dimensions); lattice point (I, J) sits at
 * (h (I - (Nx-1)/2), h (J - (Ny-1)/2)).  The window holds I = i0 .. i0+nx-1,
 * J = j0 .. j0+ny-1. */
typedef struct {
    float h;
    int32_t i0, j0, nx, ny;
} dpps_window;

/* A pass variant: kick type (DPPS_FLAT / DPPS_CHIP) and kick speed v0 (m/s). */
typedef struct {
    int32_t type;
    float v0;
} dpps_variant;

/* One frame of a request.  Its robots are robots[robot_off .. robot_off +
 * n_team + n_opp): the team first (passer included at index `passer` within
 * the team), then the opponents.  Its windows and variants are likewise slices
 * of the window and variant arrays.  out_off is the element offset of the
 * frame's first output (filled in by dpps_layout).  The ball is at
 * (ball_x, ball_y); the passer is never an interceptor. */
typedef struct {
    int32_t n_team, n_opp, passer, robot_off;
    int32_t n_windows, window_off, n_variants, variant_off;
    int64_t out_off;
    float ball_x, ball_y;
} dpps_frame;

/* Geometry, motion limits, ball model and scoring constants, and the sample
 * count K.  The score of a feasible pass is
 *   w_angle * open_goal_angle / pi + w_dist * (1 - |c - goal| / dist_norm)
 *   + w_margin * clamp(t_opp - t_team, 0, margin_cap_s)
 * (Eq. 3 with lengths and angles divided by their upper bound, Sec. 4.3). */
typedef struct {
    float field_len, field_wid, goal_x, goal_width; /* 12, 9, 6, 1.2 */
    float robot_radius, vmax, amax;                 /* 0.09, 3.25 (Sec. 2.1), 3 */
    float slide_decel, roll_decel, slide_ratio;     /* 5, 0.5, 5/7 (Sec. 4.1) */
    float chip_angle, gravity;                      /* pi/4, 9.81 */
    int32_t n_samples;                              /* K: 64, 128, 192 or 256 */
    float margin_s, margin_cap_s;                   /* 0.1, 1.0 */
    float w_angle, w_dist, w_margin, dist_norm;     /* 0.5, 0.3, 0.2, 15 */
    float goal_eps;                                 /* floor of the depth to the goal line, 1e-3 */
    uint32_t out_flags;                             /* 0 or DPPS_OUT_REDUCED */
    uint32_t reserved;                              /* must be 0 */
    uint64_t hbm_budget_bytes;                      /* 0: no limit */
} dpps_params;

/* Device-side outputs of a search.  Element e of a frame is the (window,
 * variant, point) with e = out_off + window base + variant * nx*ny + j*nx + i
 * (window-major, then variant-major, then row-major); with DPPS_OUT_REDUCED
 * the variant axis is dropped.  Any map pointer may be NULL (not written). */
typedef struct {
    uint8_t *mask;  /* 1 where the pass is feasible (REDUCED: best variant or 255) */
    float *score;   /* score where feasible, -inf elsewhere (REDUCED: best score) */
    float *t_team;  /* first-teammate interception time, +inf if none (not with REDUCED) */
    float *t_opp;   /* first-opponent interception time, +inf if none (not with REDUCED) */
    struct dpps_best_s *best; /* one record per frame (required) */
} dpps_outputs;

/* The best pass of a frame: largest score, ties to the lowest element index.
 * found = 0 and score = -inf when no pass is feasible (not an error). */
typedef struct dpps_best_s {
    int32_t found, window, variant, i, j, type;
    float x, y, v0, score, t_team, t_opp, t_ball; /* t_ball: ball time to the point */
    int32_t pad;
} dpps_best;

/* Create a context on HIP device `device` that launches on `hip_stream`
 * (NULL: the context creates its own blocking stream, ordered with the
 * legacy default stream).  Every entry point that takes a stream uses the
 * context's stream when given NULL.  Validates and copies *p. */
int dpps_create(dpps_ctx **out, const dpps_params *p, int device, void *hip_stream);

/* Wait for the context's work and free what it owns (never caller buffers). */
void dpps_destroy(dpps_ctx *c);

/* Assign out_off of n_frames frames (densely, in order) and return the total
 * number of output elements in *total.  Host-only. */
int dpps_layout(const dpps_params *p, int32_t n_frames, dpps_frame *frames,
                const dpps_window *windows, int64_t *total);

/* Device bytes the context's memory needs to hold one dpps_search_batch
 * request of these frames with tile_points points per tile (0: 8): its
 * tables, per-tile records and per-frame best records, without the
 * caller-owned outputs.  Host-only.  A context's memory grows to a quarter
 * above the largest request so far (rounded up to 64 KiB) when its budget
 * allows, else to the request's size exactly. */
int dpps_request_bytes(const dpps_params *p, int32_t n_frames, const dpps_frame *frames,
                       const dpps_window *windows, int32_t tile_points, uint64_t *bytes);

/* Device bytes the context holds now (the figure hbm_budget_bytes limits). */
uint64_t dpps_device_bytes(const dpps_ctx *c);

/* One frame, synchronous: copy the inputs, search, write the maps to the
 * device outputs and the best pass to *h_best (host).  out->best may be NULL
 * here (the context keeps a device record).  frame->out_off is honoured. */
int dpps_search(dpps_ctx *c, const dpps_frame *frame, const dpps_robot *robots,
                const dpps_window *windows, const dpps_variant *variants,
                const dpps_outputs *out, dpps_best *h_best);

/* Many frames, asynchronous on `hip_stream` (NULL: the context's stream):
 * inputs are staged through the context's pinned buffer, then one persistent
 * launch covers every (frame, window, tile).  Results are valid once the
 * stream has completed.  Calls on one context must not overlap. */
int dpps_search_batch(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                      const dpps_robot *robots, const dpps_window *windows,
                      const dpps_variant *variants, const dpps_outputs *out,
                      void *hip_stream);

/* Size in bytes of the fixed device array behind dpps_search_batch_noalloc. */
#define DPPS_NOALLOC_SCRATCH_BYTES (4u << 20)

/* For callers that cannot allocate while they run (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * search as dpps_search_batch, with the same kernels and outputs, that calls
 * no hipMalloc, hipFree, hipHostMalloc or other allocating routine.  Its
 * device state (the frames' tables, the tile list, one best record per tile
 * and the persistent work counter) lives in one fixed array of
 * DPPS_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on
 * holds until the process ends; the tables are staged through host storage
 * and a pinned buffer that dpps_create reserved.  The caller passes the host
 * inputs (read during the call) and the device outputs; out->best is
 * required.  A request whose tables and tile records do not fit the array
 * (about 10^6 points at 8 points per tile, or 24 full 5 cm frames) fails with DPPS_E_BUDGET before anything is copied or launched.
 * Asynchronous on `hip_stream` (NULL: the context's stream); results are
 * valid once the stream has completed.  Every call on one GPU, from any
 * context, shares that GPU's array, which keeps the last call's contents
 * (the work counter is cleared on the stream at the start of each call):
 * calls that overlap on one GPU race, so callers serialise them. */
int dpps_search_batch_noalloc(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                              const dpps_robot *robots, const dpps_window *windows,
                              const dpps_variant *variants, const dpps_outputs *out,
                              void *hip_stream);

/* Device-resident batches: dpps_batch_create validates the frames, builds the
 * tile list and copies everything to device memory owned by the batch
 * (synchronous).  dpps_batch_run only launches (inputs already in HBM);
 * with use_graph != 0 the launches are captured once into a HIP graph keyed
 * by the output pointers and replayed afterwards. */
int dpps_batch_create(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                      const dpps_robot *robots, const dpps_window *windows,
                      const dpps_variant *variants, dpps_batch **out);
int dpps_batch_set_robots(dpps_ctx *c, dpps_batch *b, const dpps_robot *robots, void *hip_stream);
int dpps_batch_run(dpps_ctx *c, dpps_batch *b, const dpps_outputs *out, void *hip_stream,
                   int use_graph);
void dpps_batch_destroy(dpps_batch *b);
int64_t dpps_batch_tiles(const dpps_batch *b);
int64_t dpps_batch_points(const dpps_batch *b);

/* Launch shape: points per tile (a multiple of 8, <= 64) and waves per
 * workgroup (1, 2, 4 or 8); 0 keeps the current value.  wg_per_cu: 1..32
 * persistent workgroups per compute unit, -2 persistent with as many as fit
 * (the default), -1 one workgroup per tile (no persistence), 0 keep.
 * dpps_get_launch reports the resolved workgroups per CU (-1: one per tile). */
int dpps_set_launch(dpps_ctx *c, int32_t tile_points, int32_t waves_per_wg, int32_t wg_per_cu);
int dpps_get_launch(const dpps_ctx *c, int32_t *tile_points, int32_t *waves_per_wg,
                    int32_t *wg_per_cu);

/* Autotuner: time every launch shape (tile points 8/16/32/64 x waves 1/2/4/8
 * x {persistent at occupancy, persistent with 2 or 4 workgroups per CU, one
 * workgroup per tile}) on batch b with `reps` timed runs
 * each, keep the fastest on the context and re-tile b for it.  With
 * cache_path, a previous result for the same class (architecture, K, largest
 * variant and interceptor counts, log2 points per frame, log2 frames, output
 * mode) is reused without timing, and a new result is appended as one JSON
 * line.  *best_ms (may be NULL) receives the winner's average search-kernel
 * time, or -1 when taken from the cache.  Synchronous; overwrites *out. */
int dpps_autotune(dpps_ctx *c, dpps_batch *b, const dpps_outputs *out, void *hip_stream,
                  const char *cache_path, int32_t reps, float *best_ms);

/* Device timing of the last dpps_batch_run / dpps_search_batch main kernel
 * (milliseconds, from HIP events on the launch stream); -1 if unavailable. */
float dpps_last_kernel_ms(dpps_ctx *c);

/* Kernel timing over many runs: dpps_timing_begin arms a ring of max_runs
 * event pairs; each later non-graph run records its search kernel (for
 * dpps_ray_search, its direction-sweep kernel) into the next pair (no host
 * synchronisation); dpps_timing_end waits for them and returns the summed
 * kernel time and the number of runs recorded. */
int dpps_timing_begin(dpps_ctx *c, int32_t max_runs);
int dpps_timing_end(dpps_ctx *c, float *total_ms, int32_t *n_runs);

/* ---- learned surrogate ---------------------------------------------------
 * A multilayer perceptron 66 -> 512 -> 512 -> 512 -> 2806 (GELU) predicts a
 * coarse map of a frame over the 20 cm cells of the 12 m x 9 m field
 * (61 x 46 cells; what it is trained towards is the caller's choice, e.g.
 * the exact score at each cell, or the best exact score among the 5 cm
 * points a re-score of the cell visits (dpps_pool_cells); infeasible as 0)
 * from its robots and ball: team with
 * the passer first and the rest by distance to the ball, 8 slots; opponents
 * by distance to the ball, 8 slots; each (x / 6, y / 4.5, vx / vmax,
 * vy / vmax), missing slots zero; then the ball (x / 6, y / 4.5).  Weights
 * and activations are bfloat16 with float32 accumulation on the matrix cores;
 * master weights, biases, gradients and Adam moments are float32.  The
 * surrogate search keeps the network's top-k cells and re-scores the 5 cm
 * points of each cell (4 x 4 around it) with the exact kernel: a production
 * pattern built on Sec. 4.2-4.3, not part of the paper.
 *
 * Parameters on the host are in the real layout W0 [512][66], b0 [512],
 * W1 [512][512], b1, W2 [512][512], b2, W3 [2806][512], b3 [2806]
 * (dpps_mlp_param_count() floats).  Frames come from a dpps_batch of the
 * same context. */
typedef struct dpps_mlp dpps_mlp;

int64_t dpps_mlp_param_count(void);
/* max_frames: largest batch; max_k: largest top-k (<= 256); He-uniform
 * initialisation from `seed`. */
int dpps_mlp_create(dpps_ctx *c, int32_t max_frames, int32_t max_k, uint64_t seed,
                    dpps_mlp **out);
void dpps_mlp_destroy(dpps_mlp *m);
int dpps_mlp_set_params(dpps_mlp *m, const float *host, int64_t n);
int dpps_mlp_get_params(dpps_mlp *m, float *host, int64_t n);
/* Parameter gradients of the last dpps_mlp_loss_grad (real layout). */
int dpps_mlp_get_grads(dpps_mlp *m, float *host, int64_t n);
int dpps_mlp_get_adam(dpps_mlp *m, float *host_m, float *host_v, int64_t n, int64_t *step);
int dpps_mlp_set_adam(dpps_mlp *m, const float *host_m, const float *host_v, int64_t n,
                      int64_t step);
/* Predicted maps of the batch's frames into d_out [n_frames][ld_out] (f32,
 * device; NULL keeps them internal for dpps_mlp_topk). */
int dpps_mlp_forward(dpps_mlp *m, dpps_batch *b, float *d_out, int64_t ld_out, void *hip_stream);
/* Forward, loss against d_target [n_frames][ld_target] (device f32 score
 * maps, -inf where infeasible) and backward into the parameter gradients.
 * Loss = mean over cells of (1 + pos_weight * t) (y - t)^2 with -inf read as
 * 0, plus ce_weight times the mean over frames of the cross-entropy between
 * softmax(t / tau) over the feasible cells and softmax(y / tau) over all
 * cells.  *loss (may be NULL) receives it (synchronises). */
int dpps_mlp_loss_grad(dpps_mlp *m, dpps_batch *b, const float *d_target, int64_t ld_target,
                       float pos_weight, float ce_weight, float tau, float *loss,
                       void *hip_stream);
/* Coarse-cell labels from fine score maps d_fine [n_frames][fine_ny][fine_nx]:
 * cell (ci, cj) gets the largest fine score over the fine points
 * {4ci-2 .. 4ci+1} x {4cj-2 .. 4cj+1} (the points its re-score visits), -inf
 * if none is feasible; d_coarse [n_frames][coarse_ny][coarse_nx]. */
int dpps_pool_cells(const float *d_fine, int32_t n_frames, int32_t fine_nx, int32_t fine_ny,
                    float *d_coarse, int32_t coarse_nx, int32_t coarse_ny, void *hip_stream);
/* One Adam step on the gradients (bias-corrected; decoupled weight decay
 * added to the gradient of weights only), refreshing the bfloat16 copies. */
int dpps_mlp_adam(dpps_mlp *m, float lr, float beta1, float beta2, float eps, float weight_decay,
                  void *hip_stream);
/* dpps_mlp_loss_grad then Adam (0.9, 0.999, 1e-8, no decay). */
int dpps_mlp_train_step(dpps_mlp *m, dpps_batch *b, const float *d_target, int64_t ld_target,
                        float lr, float pos_weight, float ce_weight, float tau, float *loss,
                        void *hip_stream);
/* The network input of each frame as bfloat16 [n_frames][66] (device). */
int dpps_mlp_features(dpps_mlp *m, dpps_batch *b, uint16_t *d_x, void *hip_stream);
/* Top-k cells (descending prediction, ties to the lower cell) of the last
 * forward pass into d_cells [n_frames][k] (device int32). */
int dpps_mlp_topk(dpps_mlp *m, int32_t n_frames, int32_t k, int32_t *d_cells, void *hip_stream);
/* Surrogate search: forward, top-k cells, exact re-score of their 5 cm points
 * with the frame's variants; best pass per frame into d_best (device).  With
 * fallback != 0, frames where no proposed point is feasible, or whose best
 * re-scored pass scores below fallback_below (-INFINITY: infeasible frames
 * only), are searched exactly on the whole 5 cm lattice; those frames are
 * picked, and their tables built, on the device in stream order, so the
 * call is asynchronous unless n_fallback (may be NULL) is given, in which
 * case it returns once the stream has finished and *n_fallback counts them.
 * The batch's own windows are not used.  A NaN fallback_below is
 * DPPS_E_INVALID. */
int dpps_surrogate_search(dpps_ctx *c, dpps_mlp *m, dpps_batch *b, int32_t k, dpps_best *d_best,
                          int fallback, float fallback_below, int32_t *n_fallback,
                          void *hip_stream);
/* The same from host frames (layout as for dpps_search_batch; the windows are
 * validated but not searched): the tables go through the context's pinned
 * staging into device memory the context keeps, so a steady stream of
 * requests allocates nothing.  n_frames must not exceed the network's
 * max_frames.  h_best (host, n_frames records, may be NULL): when given, the
 * best records are also written there and the call returns once the stream
 * has finished them. */
int dpps_surrogate_search_frames(dpps_ctx *c, dpps_mlp *m, int32_t n_frames,
                                 const dpps_frame *frames, const dpps_robot *robots,
                                 const dpps_window *windows, const dpps_variant *variants,
                                 int32_t k, dpps_best *d_best, int fallback, float fallback_below,
                                 int32_t *n_fallback, dpps_best *h_best,
                                 void *hip_stream);

/* ---- passing power per point (Sec. 4.1, Eq. 1-2) ------------------------
 * Instead of a list of kick speeds, every candidate point gets its own flat
 * pass whose speed follows the receiver: the receiver is the teammate
 * (passer excluded) that reaches the point first, the ball should arrive at
 * its arrival time plus buffer_s; ignoring the sliding phase as Eq. 1 does,
 * the speed after the slide over distance d and time t at the rolling
 * deceleration a is v1 = (d + a t^2 / 2) / t while the ball still rolls at t
 * (else the slowest ball that reaches the point, sqrt(2 a d)); Eq. 2 gives
 * the kick speed v1 / slide_ratio, clamped to the robots' kick range
 * [v_min, v_max].  The pass is then searched as in dpps_search with the full
 * ball model.  Outputs: one element per point (layout of dpps_search with
 * one variant per frame; the frames' variants are not used), d_v0 (may be
 * NULL) the kick speed per point (0 where no teammate can receive), best.v0
 * the chosen pass's speed. */
typedef struct {
    float buffer_s;   /* time added to the receiver's arrival (0.3 s in the paper) */
    float v_min, v_max; /* kick range (1, 6.5 m/s) */
    int32_t reserved; /* must be 0 */
} dpps_power_params;

int dpps_search_power(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                      const dpps_robot *robots, const dpps_window *windows,
                      const dpps_power_params *pp, const dpps_outputs *out, float *d_v0,
                      void *hip_stream);

/* ---- the paper's direction x power form (Sec. 4.2) ----------------------
 * The search as the paper states it, from the passer's point of view: for
 * every kick direction theta_d = 2 pi d / n_dirs (d = 0 .. n_dirs-1, from +x,
 * counterclockwise) and every pass variant of a frame, the ball runs from the
 * ball position along the direction until it stops or leaves the field.  K
 * samples uniform in distance over the part of the ray inside the field,
 * s_k = (k+1) L / K, are shared by all variants; a variant uses the samples
 * its ball reaches (chips: from the landing point on).  Each robot's
 * interception is searched as in dpps_search (Sec. 4.2); the pass is
 * received at the first teammate's interception, the passing point, and is
 * feasible when the first opponent intercepts at least margin_s later, or
 * never.  Its score is Eq. (3) over the five features of Sec. 4.3:
 *   w_angle * open goal angle at the passing point / pi
 *   + w_dist * (1 - distance from the passing point to the goal centre / dist_norm)
 *   + w_margin * clamp(t_opp - t_team, 0, margin_cap_s)
 *   - w_time * t_team (seconds)
 *   - w_refract * refraction angle / pi,
 * the refraction angle being the angle between the ball's direction and the
 * shot from the passing point to the goal centre.  The frames' windows are
 * not used (n_windows is ignored). */
typedef struct {
    int32_t n_dirs;   /* 1 .. 4096 (the paper: 128, 360/128 = 2.8 degrees) */
    float w_time;     /* weight per second of the first teammate's interception time (>= 0) */
    float w_refract;  /* weight of the refraction angle / pi (>= 0) */
    int32_t reserved; /* must be 0 */
} dpps_ray_params;

/* The best pass of a frame: largest score, ties to the lowest (direction,
 * variant) index d * n_variants + v.  found = 0 when none is feasible. */
typedef struct {
    int32_t found, dir, variant, type;
    float theta, v0, x, y; /* direction (rad), kick speed, passing point */
    float score, t_team, t_opp, open_angle, refract;
    int32_t pad;
} dpps_ray_best;

/* Device outputs of dpps_ray_search.  Element (f, d, v) sits at
 * base(f) + d * n_variants(f) + v, base(f) being the sum of n_dirs *
 * n_variants over the frames before f.  Any map pointer may be NULL. */
typedef struct {
    uint8_t *mask;   /* 1 where the pass is feasible */
    float *score;    /* score where feasible, -inf elsewhere */
    float *t_team;   /* first teammate interception (ball) time, +inf if none */
    float *t_opp;    /* first opponent interception time, +inf if none */
    float *s_recv;   /* distance along the ray to the passing point, +inf if none */
    dpps_ray_best *best; /* one record per frame (required) */
} dpps_ray_outputs;

/* Every direction x variant of n_frames frames, asynchronous on the stream
 * (inputs are host arrays staged through the context, as for
 * dpps_search_batch). */
int dpps_ray_search(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                    const dpps_robot *robots, const dpps_variant *variants,
                    const dpps_ray_params *rp, const dpps_ray_outputs *out, void *hip_stream);

/* ---- shooting decision (Sec. 4.4) ----------------------------------------
 * The shot-angle test fused with the interception prediction along the shot.
 * From a shooter position c (the frame's ball, and optionally every point of
 * the frame's windows with the ball placed there):
 *   - the goal mouth spans the directions from c to the two posts (the depth
 *     to the goal line is floored at goal_eps); the frame's opponents
 *     in front of the goal line shadow the directions that pass within
 *     robot_radius of them, as for the open goal angle of dpps_search; a
 *     shooter inside an opponent's radius has no open direction;
 *   - gap = the widest open run of directions, the valid angle of the shot;
 *     the shot aims at its centre (ties to the lower angle), or at the goal
 *     centre when nothing is open;
 *   - the shot is a flat kick at v_shot along the aim to the goal line,
 *     sampled like a pass: K samples uniform in distance, the kick point
 *     excluded, the goal-line point included; slack = the smallest
 *     (earliest opponent arrival - ball time) over the samples the ball gets
 *     to (+inf without opponents); an opponent intercepts exactly when
 *     slack <= 0; teammates never block;
 *   - shoot = gap >= min_angle and the ball reaches the goal line and
 *     slack > margin_s.
 * The frames' variants are not used. */
typedef struct {
    float v_shot;     /* flat kick speed of the shot, m/s (> 0; 6.5 = top of the kick range) */
    float min_angle;  /* threshold on the widest open gap, rad (>= 0) */
    float margin_s;   /* required slack, s (>= 0; 0 = not intercepted) */
    int32_t reserved; /* must be 0 */
} dpps_shot_params;

typedef struct {
    int32_t shoot;     /* the decision */
    int32_t reachable; /* the ball reaches the goal line */
    float aim;         /* direction of the shot, rad from +x */
    float gap;         /* widest open gap, rad */
    float open_angle;  /* sum of the open gaps, rad */
    float length;      /* distance to the goal line along the aim, m */
    float t_goal;      /* ball time to the goal line, s (+inf when it stops short) */
    float slack;       /* s, see above */
} dpps_shot;

/* Decisions from each frame's ball into d_ball (n_frames records, device
 * memory, required) and, when d_map is not NULL, from every point of the
 * frames' windows into d_map: one record per point at the element index
 * dpps_search_batch uses with one variant per frame (out_off + window base +
 * j*nx + i; dpps_layout with n_variants = 1 packs them densely).
 * Asynchronous on the stream; inputs are host arrays staged through the
 * context and may be reused when the call returns.  Errors: DPPS_E_INVALID
 * for bad parameters or frames (as dpps_search_batch), DPPS_E_DEVICE. */
int dpps_shot_decision(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                       const dpps_robot *robots, const dpps_window *windows,
                       const dpps_shot_params *sp, dpps_shot *d_ball, dpps_shot *d_map,
                       void *hip_stream);

/* ---- running points (Sec. 5.2) --------------------------------------------
 * Every vertex of each zone raster (the frames' windows, e.g. four front-field
 * zones at 0.1 m that move with the ball, Sec. 5.1) gets the weighted sum of
 * Eq. (4) over five criteria, each in [0, 1], higher better:
 *   x1 distance to the goal: 1 - |c - goal centre| / dist_norm;
 *   x2 distance to the ball: min(|c - ball| / ball_norm, 1);
 *   x3 angle to the goal: with phi = |bearing of the goal centre from c| (0
 *      straight along +x), 1 inside [ang_lo, ang_hi], falling linearly to 0
 *      over ang_fall outside it;
 *   x4 the opponents' guard time: the segments from c to the two goal posts
 *      first meet the defense area (def_depth deep, def_width wide, in front
 *      of the goal) at P and Q; with t_P, t_Q the earliest opponent arrivals
 *      there (the robot model of dpps_search), min((t_P + t_Q) / guard_norm, 1),
 *      1 without opponents;
 *   x5 avoiding the defense: every opponent nearer to the ball than c marks
 *      c with weight max(0, 1 - |o - c| / mark_radius); 1 - the largest mark.
 * A point strictly inside the defense area cannot be used (score -inf).  The
 * paper names the criteria without formulas or weights: all of the above
 * constants are caller parameters. */
typedef struct {
    float w_goal, w_ball, w_angle, w_guard, w_defense; /* Eq. (4) weights (finite) */
    float ball_norm;                 /* m, > 0 */
    float ang_lo, ang_hi, ang_fall;  /* rad: 0 <= ang_lo <= ang_hi, ang_fall > 0 */
    float guard_norm;                /* s, > 0 */
    float def_depth, def_width;      /* m, >= 0 (SSL 2019 division A: 1.2 x 2.4) */
    float mark_radius;               /* m, > 0 */
    int32_t reserved;                /* must be 0 */
} dpps_run_params;

/* Best running point of one zone: largest score, ties to the lowest
 * row-major index; found = 0 when every point lies in the defense area. */
typedef struct {
    int32_t found, i, j, reserved;
    float x, y, score;
    float goal, ball, angle, guard, defense; /* the five criteria there */
} dpps_run_best;

/* Scores of every zone point into d_score (may be NULL; element order of
 * dpps_search_batch with one variant per frame) and one dpps_run_best per
 * zone into d_best (required; zones in the order of the frames, then of each
 * frame's windows).  Only the ball and the opponents of a frame are used.
 * Asynchronous on the stream; host inputs staged through the context.
 * Errors: DPPS_E_INVALID (parameters, frames, zones outside the lattice),
 * DPPS_E_DEVICE. */
int dpps_running_points(dpps_ctx *c, int32_t n_frames, const dpps_frame *frames,
                        const dpps_robot *robots, const dpps_window *zones,
                        const dpps_run_params *rp, float *d_score, dpps_run_best *d_best,
                        void *hip_stream);

const char *dpps_strerror(int code);
const char *dpps_last_error(void);
int dpps_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DPPS_H */
