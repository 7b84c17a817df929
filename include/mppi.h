/*
 * mppi.h -- C ABI of the MI355X (gfx950) MPPI sampling-step library.
 *
 * One solve is one pass of Model Predictive Path Integral control as defined
 * in Sec. III-B of the paper (Eq. (3)-(5), Alg. 1): K control sequences are
 * sampled around the nominal sequence U*, each is rolled out N steps through
 * the quadrotor dynamics of Sec. III-A (Eq. (2), RK4 with step dt), scored by
 * one objective -- gate progress (Sec. IV-A, Eq. (6)-(7)), trajectory tracking
 * (Sec. IV-B-1, Eq. (8)) or contouring (Sec. IV-B-2, Eq. (9)) -- and the
 * samples are blended by softmax weights into the next nominal sequence.
 * Only the first input is returned for the plant (receding horizon).
 *
 * Conventions shared by every entry point
 *   - State x (13 doubles): p[3] (m, world), v[3] (m/s, world),
 *     q[4] = (w, x, y, z) unit quaternion, Hamilton, body-to-world,
 *     omega[3] (rad/s, body).  Gravity acts along world -z.
 *   - Input u (4 doubles): the four rotor thrusts in N, rotor order of the
 *     torque map of Eq. (2) (X layout).
 *   - Host pointers are caller-owned and only read (or written) during the
 *     call.  Problem data passed to mppi_create is deep-copied to the device.
 *   - Every entry point returns an mppi_status; no exception or abort ever
 *     crosses the ABI.  On any error the context and its warm-start state
 *     are left as they were, and mppi_last_error() describes the failure.
 *   - A context is used by one host thread at a time.  Distinct contexts may
 *     be used concurrently from different threads on different streams.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_N_MAX 256            /* longest horizon                          */
#define MPPI_K_MAX (1 << 24)      /* most samples per solve                   */
#define MPPI_MASK_WORDS 9         /* (MPPI_N_MAX + 1) bits of per-state flags */
#define MPPI_G_MAX 256            /* most gates of a gate track               */
#define MPPI_REQ_DOUBLES 24       /* device request record, see mppi_solve_device */

typedef struct mppi_ctx mppi_ctx;

typedef enum {
    MPPI_OK = 0,
    MPPI_E_INVAL = -1,     /* an argument is out of range or inconsistent         */
    MPPI_E_NOMEM = -2,     /* the device allocation failed                        */
    MPPI_E_DEVICE = -3,    /* a HIP runtime call failed                           */
    MPPI_E_NONFINITE = -4  /* every sample cost was non-finite; nothing updated   */
} mppi_status;

enum { MPPI_OBJ_GATE = 0, MPPI_OBJ_CONTOUR = 1, MPPI_OBJ_TRACK = 2 };
enum { MPPI_FP32 = 0, MPPI_FP64 = 1 };
/* Input models.  MPPI_INPUT_THRUST: the four rotor thrusts are the input (13
 * states).  MPPI_INPUT_RATE: the paper's model (Sec. III-A): the input is the
 * thrusts' time derivative and the thrusts are four more states (17: the 13
 * above, then T[4]); contouring then samples the progress acceleration and
 * carries the progress speed as a state (Sec. IV-B-2, Eq. (9)). */
enum { MPPI_INPUT_THRUST = 0, MPPI_INPUT_RATE = 1 };

/* Quadrotor model of Eq. (2). */
typedef struct {
    double mass;          /* kg, > 0                                           */
    double arm;           /* l in the torque map, m                            */
    double inertia[3];    /* diag(J), kg m^2, each > 0                         */
    double c_tau;         /* yaw torque per unit rotor thrust, m               */
    double drag[3];       /* diag(D) of the rotor-drag term, 1/s (0 disables)  */
    double gravity;       /* m/s^2                                             */
    double t_min, t_max;  /* per-rotor thrust bounds: samples are clipped here */
    double w_max;         /* body-rate bound of the feasibility penalty, rad/s */
} mppi_quad;

/* Sampling parameters (Eq. (3)-(4)) and cost weights. */
typedef struct {
    int32_t K;            /* samples, 1..MPPI_K_MAX                            */
    int32_t N;            /* horizon steps, 1..MPPI_N_MAX                      */
    int32_t objective;    /* MPPI_OBJ_*                                        */
    int32_t precision;    /* MPPI_FP32 (Kahan cost sums) or MPPI_FP64          */
    double dt;            /* integration and prediction step, s, > 0          */
    double lambda;        /* softmax temperature, > 0                          */
    double sigma[4];      /* per-rotor noise standard deviation, N, >= 0       */
    double sigma_v;       /* contouring: progress-speed noise std, m/s, >= 0   */
    uint64_t seed;        /* Philox key                                        */
    double w_lim;         /* weight of the body-rate hinge penalty             */
    double q_near;        /* gate: Q_near of Eq. (7)                           */
    double r_near;        /* gate: radius around the current gate, m           */
    double Q[13];         /* tracking: diag stage weight on x - x_ref          */
    double QN[13];        /* tracking: diag terminal weight                    */
    double R_dT[4];       /* tracking/contouring: diag weight on dT/dt         */
    double q_l, q_c;      /* contouring: lag and contour error weights         */
    double Q_w[3];        /* contouring: body-rate weights                     */
    double r_dv;          /* contouring: weight on the progress acceleration   */
    double mu;            /* contouring: progress reward                       */
    double v_max;         /* contouring: progress-speed bound, m/s             */
    int32_t proj_window;  /* contouring: +- table points searched for theta0   */
    int32_t flags;        /* MPPI_FLAG_* (0 for a stand-alone context)          */
    /* Two standard MPPI variants the paper does not use; zero keeps the
     * paper's method (one iteration, cost of Eq. (6)-(9) alone). */
    int32_t n_iter;       /* MPPI iterations per solve, 0..64 (0 and 1: one).
                             Iterations after the first sample around the
                             previous iteration's solution from the same x0
                             and t_now without shifting it, keep the first
                             iteration's last applied input for the rate
                             terms and draw with the next solve counter; the
                             solve reports the last iteration.            */
    double ctrl_cost;     /* gamma >= 0 of the information-theoretic control
                             cost gamma * sum_k sum_i U*_ki (U_ki - U*_ki) /
                             sigma_i^2 added to each sample's cost (channels
                             with sigma_i > 0, contouring speed included),
                             U* the shifted warm start, U the clipped sample;
                             0: off.  A nonzero gamma needs the sample
                             tensor, so it switches the regenerating average
                             off.                                          */
    /* Input model (MPPI_INPUT_*).  With MPPI_INPUT_RATE each sampled rate is
     * clipped to rate_lim and then to the range that keeps its thrust within
     * [t_min, t_max] over the step; the contouring acceleration likewise to
     * dv_lim and to the range that keeps the progress speed within
     * [0, v_max].  The rate model runs the one-wave rollout with a separate
     * sampling kernel; a batch holding such a context runs all its contexts
     * with one-wave rollouts (a server launches each layout on its own). */
    int32_t input_model;
    int32_t pad_;
    double rate_lim[2];   /* thrust-rate bounds, N/s (lower <= 0 <= upper)    */
    double dv_lim[2];     /* progress-acceleration bounds, m/s^2 (contouring) */
} mppi_params;

/* The context allocates no per-solve workspace (sample tensor, costs,
 * per-tile cost minima); a server lends one to each admitted solve.  Such a
 * context is solved only through a server or mppi_solve_device_noalloc
 * (mppi_solve, mppi_solve_device and mppi_read_samples return MPPI_E_INVAL). */
#define MPPI_FLAG_EXTERNAL_WORKSPACE 1

/* The weighted average of Eq. (5) draws every sample again from the
 * counter-based noise of the solve (the sampling of Eq. (3) repeated with the
 * same counters and the same arithmetic) instead of reading the N x K sample
 * tensor, which the rollout then does not write: the same result bit for
 * bit, with Philox and Box-Muller work in place of 16 B (20 B contouring) of
 * HBM traffic per sample and step.  It takes effect wherever the rollout
 * draws the samples itself: the three- and four-wave layouts and the
 * drawing one-wave layout (mppi_info.regen_average reports it), with thrust
 * as the input and no control-cost term.  Batches choose it per batch
 * (mppi_batch_cfg.regen_average; not with a control-cost term in the
 * batch); served solves keep the tensor.
 * mppi_autotune can choose it instead.  mppi_read_samples then returns the
 * costs only (MPPI_E_INVAL when U_samples is requested). */
#define MPPI_FLAG_REGEN_AVERAGE 2

/* Problem data: the inputs of Alg. 1 (waypoints W, path P_arc, tau_ref). */
typedef struct {
    const double *gates;  /* G x 4 row-major: centre x, y, z, yaw (gate objective) */
    int32_t n_gates;      /* G, 1..MPPI_G_MAX                                  */
    double gate_size;     /* side of the square aperture, m                    */
    const double *path;   /* P x 6 row-major: position, unit tangent; P points
                             uniformly spaced in arc length over a closed path */
    int32_t n_path;
    double path_len;      /* total arc length L, m                             */
    const double *xref;   /* R x 13 row-major full-state reference rows        */
    int32_t n_ref;
    double ref_dt;        /* time between reference rows, s                    */
} mppi_problem;

/* Optional device allocator (e.g. backed by a framework's caching allocator).
 * alloc returns device memory of at least `bytes` bytes aligned to 256 B, or
 * NULL; free releases it.  When the whole struct pointer is NULL the library
 * uses hipMalloc / hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} mppi_allocator;

/* What a solve reports besides the control. */
typedef struct {
    double J_min;          /* smallest finite sample cost                      */
    double S;              /* sum of exp(-(J_m - J_min)/lambda)                */
    double ess;            /* effective sample size 1 / sum w_m^2               */
    double J_nom;          /* cost of the noise-free nominal rollout            */
    double theta0;         /* contouring: arc length the rollouts start from    */
    int32_t status;        /* mppi_status of the solve                          */
    int32_t g0;            /* gate: index of the current target gate            */
    int32_t i0;            /* tracking: reference row of the initial state      */
    int32_t shift;         /* steps the previous solution was shifted by        */
    uint32_t solve_index;  /* Philox counter word of this solve                 */
    int32_t rollout_waves; /* rollout layout of the context's own solves: waves
                              per 64-sample tile (see mppi_batch_cfg)           */
    int32_t regen_average; /* 1: the average draws the samples again
                              (MPPI_FLAG_REGEN_AVERAGE in effect)               */
    int32_t rollout_draw;  /* 1: the one-wave rollout draws its samples itself
                              (binary32, sample tensor larger than 256 MiB)     */
} mppi_info;

/* Warm-start state inherited by the next solve (checkpoint / restore). */
typedef struct {
    int32_t warm;                      /* 0: the next solve starts cold (hover) */
    int32_t g0;                        /* current target gate                   */
    uint32_t solve_index;              /* Philox counter word of the next solve */
    int32_t N;                         /* rows valid in U and V                  */
    uint32_t allow[MPPI_MASK_WORDS];   /* bit j: state j may register the first
                                          gate pass (temporal-consistency rule)  */
    double t_prev;                     /* time of the previous solve, s         */
    double x_prev[13];                 /* state of the previous solve            */
    double theta0;                     /* previous arc length (contouring)       */
    double U[MPPI_N_MAX * 4];          /* previous solution, N x 4               */
    double V[MPPI_N_MAX];              /* previous progress-speed (rate model:
                                          progress-acceleration) solution, N    */
    double vtheta;                     /* rate model, contouring: progress speed
                                          at the previous solve's time          */
} mppi_warm;

/* Create a solver context: the inputs of Alg. 1 (sample count M = K, horizon
 * K = N, temperature lambda, noise covariance Sigma, the waypoints / path /
 * reference of the objective; Sec. III-B and IV) bound to the quadrotor of
 * Eq. (2).  Validates every argument (K, N, dt, lambda, sigma,
 * objective and the data it needs: 1..MPPI_G_MAX gates, P >= 2 path points,
 * R >= 1 reference rows), copies the problem data to the device and allocates all
 * device buffers: the N x K x 4 sample tensor (step-major: sample m of step k
 * at element (k*K + m)*4), K costs, the per-tile cost minima and the
 * warm-start state.  stream is a hipStream_t (NULL: the library creates a non-blocking
 * stream of default priority that it owns).  The context starts cold with
 * target gate 0.  On failure *out is NULL.
 *
 * The rollout layout is chosen here from K, N and the precision and reported
 * in mppi_info (rollout_waves, rollout_draw).  Two environment variables,
 * read at creation, override the choice for testing and measurement:
 * MPPI_ROLLOUT_WAVES (1..4: waves per 64-sample tile) and MPPI_ROLLOUT_DRAW
 * (0 or 1: whether a binary32 one-wave rollout draws its own samples).  The
 * results do not depend on the layout beyond rounding; rollout_draw changes
 * no bit. */
mppi_status mppi_create(const mppi_params *params, const mppi_quad *quad,
                        const mppi_problem *problem, void *stream,
                        const mppi_allocator *allocator, mppi_ctx **out);

/* Release every device and host resource of the context (the end of the
 * receding-horizon loop of Alg. 1).  NULL is a no-op. */
void mppi_destroy(mppi_ctx *ctx);

/* One MPPI step from host memory, synchronous on the context stream: one
 * pass of Alg. 1's loop body (sample Eq. (3), roll out Eq. (2) with the costs
 * of Eq. (6)-(9), weigh Eq. (4), update Eq. (5), shift the warm start).
 * x0: current state (finite, |q| > 0): 13 doubles, or 17 for MPPI_INPUT_RATE
 * (the measured rotor thrusts appended).  t_now: time of x0 in s; the previous
 * solution is shifted by max(1, round((t_now - t_prev)/dt)) steps and, for
 * tracking, the reference row round(t_now / ref_dt) is aligned with x0.
 * u0_out: 4 doubles, the first input of the new solution (required).
 * U_out: N x 4 doubles, the whole new solution (optional, NULL to skip).
 * info: optional report.  Returns MPPI_E_NONFINITE, leaving the warm-start
 * state unchanged, when every sample cost is non-finite. */
mppi_status mppi_solve(mppi_ctx *ctx, const double x0[13], double t_now, double u0_out[4],
                       double *U_out, mppi_info *info);

/* The same step driven entirely from device memory, asynchronous on the
 * context stream (nothing is copied to or from the host, nothing waits).
 * d_req: device pointer to MPPI_REQ_DOUBLES doubles, x0 in [0..12], t_now in
 * [13] and, for MPPI_INPUT_RATE, the measured rotor thrusts in [16..19] (the
 * rest is ignored).  d_u0: device pointer receiving 4 doubles.
 * Both must stay valid until the stream reaches the end of the solve.  The
 * status and report of the solve are read later with mppi_read_info; a solve
 * whose costs are all non-finite leaves the warm-start state unchanged and
 * writes NaN to d_u0.  The call sequence is fixed, so it may be captured in a
 * HIP graph and replayed with new contents of d_req. */
mppi_status mppi_solve_device(mppi_ctx *ctx, const double *d_req, double *d_u0);

/* Allocation-free variant of mppi_solve_device, for callers that cannot
 * allocate device memory during a solve (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The same step with the
 * same arguments, results and stream semantics, but the per-solve workspace
 * (sample tensor, costs, per-tile cost minima, front flags) is a fixed
 * library array of MPPI_SCRATCH_BYTES per GPU instead of the context's own,
 * so it also runs contexts created with MPPI_FLAG_EXTERNAL_WORKSPACE.  The
 * call allocates nothing: the array is a static device variable whose address
 * is looked up once per device on the first call there.
 *   - MPPI_E_INVAL when the context's workspace exceeds MPPI_SCRATCH_BYTES
 *     (binary32 gate or tracking: about 16*K*N + 4*K bytes; contouring
 *     20*K*N + 4*K; binary64 twice that), when the current device is not the
 *     one the context was created on, or when d_req is NULL.
 *   - Every call on a GPU shares that GPU's array.  Two calls whose work
 *     overlaps on one GPU (different streams, no ordering between them) race
 *     on it and their results are undefined; calls ordered on one stream are
 *     safe.  Nothing in the array has to start at zero: a solve writes every
 *     word of it that it reads.
 *   - mppi_read_samples keeps reading the context's own workspace, so it does
 *     not see the costs of a solve made through this entry point. */
#define MPPI_SCRATCH_BYTES ((size_t)32 << 20)
mppi_status mppi_solve_device_noalloc(mppi_ctx *ctx, const double *d_req, double *d_u0);

/* Wait for the context stream and copy the report of the latest solve. */
mppi_status mppi_read_info(mppi_ctx *ctx, mppi_info *info);

/* Result of mppi_autotune. */
typedef struct {
    int32_t regen_average;   /* chosen: 1 the regenerating average, 0 the stored */
    int32_t from_cache;      /* 1: taken from the cache, nothing timed           */
    double ms_stored;        /* mean solve time with the stored average, ms (0:
                                not measured)                                   */
    double ms_regen;         /* the same with the regenerating average (0: not
                                measured or not available in this layout)      */
} mppi_tune_result;

/* Autotuner of one context (Eq. (5) either way): time `reps` solves of the
 * request record d_req (device, layout of mppi_solve_device) with the stored
 * and with the regenerating weighted average, where the context's rollout
 * draws its samples, and keep the faster for the context's later solves; on
 * a cache hit (cache_path, key kind "ctx", no MPPI_TUNE_FORCE) apply the
 * cached choice without timing.  The warm-start state and report are
 * restored after the timed solves.  Synchronous.  MPPI_E_INVAL for a NULL
 * context or request, reps < 1, or a context with an external workspace. */
mppi_status mppi_autotune(mppi_ctx *ctx, const double *d_req, int32_t reps, const char *cache_path, int32_t flags,
                          mppi_tune_result *out);

/* Copy the latest solve's sample costs (K doubles, as computed, in FP64
 * whatever the precision) and optionally the sample controls (N x K x 4
 * doubles, step-major; MPPI_E_INVAL when the context's average regenerates
 * the samples).  Waits for the context stream. */
mppi_status mppi_read_samples(mppi_ctx *ctx, double *J, double *U_samples);

/* Export / import the warm-start state (waits for the context stream).
 * set_warm validates N against the context and the gate index against G. */
mppi_status mppi_get_warm(mppi_ctx *ctx, mppi_warm *out);
mppi_status mppi_set_warm(mppi_ctx *ctx, const mppi_warm *in);

/* Per-kernel timing of solves (instrumentation for benchmarks).  While
 * enabled, every solve records HIP events on the context stream around its
 * three kernels (sample, rollout, average).  mppi_read_profile waits for the
 * stream and returns the mean duration in ms of each kernel over the solves
 * recorded since the last read (at most 4096), and how many there were; it
 * then starts a new collection. */
mppi_status mppi_set_profiling(mppi_ctx *ctx, int32_t enable);
mppi_status mppi_read_profile(mppi_ctx *ctx, double mean_ms[3], int32_t *n_solves);

/* ---- Batches of independent solves (one persistent launch per kernel) ----
 *
 * A batch registers n contexts (all of one precision; objectives, K and N may
 * differ).  Each mppi_batch_solve_device call runs one MPPI step for a chosen
 * subset of them in a single launch sequence: a grid-stride sample kernel, a
 * persistent rollout kernel that pulls 64-sample tiles from a device queue in
 * order of decreasing horizon, a grid-stride control-cost kernel where a
 * context has the term (one unit per context and 64-sample tile), and a
 * grid-stride weighted-average kernel (one unit per context and horizon
 * step), repeated n_iter times (the contexts' shared n_iter), per group
 * of contexts sharing an objective and accumulation type.  Grids are fixed
 * and the work description lives in device memory, so the sequence is
 * captured once in a HIP graph (cfg.use_graph) and replayed for any subset.
 * Each context's result, report and warm-start state are the same as those
 * of mppi_solve_device on that context alone with the same rollout layout. */
typedef struct mppi_batch mppi_batch;

typedef struct {
    int32_t rollout_waves;     /* waves per 64-sample tile: 1 (separate sampling
                                  kernel), 2 (attitude / translation split), 3
                                  (sampling joins the rollout) or 4 (four-stage
                                  pipeline: sampling with body rates, attitude,
                                  translation, sampling with position costs;
                                  chunks of 4 steps with one workgroup per CU,
                                  of 2 with two, the same results);
                                  0: automatic (binary32: 4 for at most two
                                  64-sample tiles per CU, else 1; binary64: 4
                                  for at most one, 2 for at most two, else 1;
                                  the same rule picks a context's layout) */
    int32_t rollout_groups;    /* persistent rollout workgroups; 0: automatic    */
    int32_t sample_groups;     /* workgroups of the sample and reduction kernels;
                                  0: automatic                                   */
    int32_t use_graph;         /* 1: capture the launch sequence in a HIP graph  */
    int32_t regen_average;     /* 1: with three- or four-wave rollouts, no sample
                                  tensor: the weighted average draws the samples
                                  again (see MPPI_FLAG_REGEN_AVERAGE); ignored
                                  with one- and two-wave rollouts             */
} mppi_batch_cfg;

/* Register ctxs[0..n-1] (distinct, same precision and n_iter, each used by
 * no other batch or call while the batch runs: MPPI_E_INVAL otherwise).  stream: hipStream_t of the batch's
 * launches (NULL: one owned by the batch).  cfg NULL: all automatic, graph on.
 * The contexts must outlive the batch. */
mppi_status mppi_batch_create(mppi_ctx *const *ctxs, int32_t n, void *stream, const mppi_batch_cfg *cfg,
                              mppi_batch **out);

/* One MPPI step for the contexts active[0..n_active-1] (indices into the
 * registered list, distinct; NULL with n_active = n: all, in order).  Solve i
 * reads its request record (layout of mppi_solve_device) at
 * d_reqs + MPPI_REQ_DOUBLES i and
 * writes its first input to d_u0s + 4 i; both are device pointers that must
 * stay valid until the stream reaches the end of the step.  Asynchronous. */
mppi_status mppi_batch_solve_device(mppi_batch *b, const int32_t *active, int32_t n_active,
                                    const double *d_reqs, double *d_u0s);

/* Change the launch shape (drops a captured graph). */
mppi_status mppi_batch_set_cfg(mppi_batch *b, const mppi_batch_cfg *cfg);
mppi_status mppi_batch_get_cfg(const mppi_batch *b, mppi_batch_cfg *cfg);

/* Autotuner cache: a JSON object in the file cache_path, one entry per key
 * "<kind>|<gfx arch>|<objective(s)>|<fp32|fp64>|<size buckets>" (size
 * buckets: floor(log2) of K and N for a context; of the instance count and of
 * sum K*N for a batch), each holding the chosen launch settings and the mean
 * time measured for them.  Written through a temporary file and a rename.
 * cache_path NULL: no cache.  MPPI_TUNE_FORCE: time even on a cache hit. */
#define MPPI_TUNE_FORCE 1

/* Autotuner: time every candidate launch shape (rollout waves x persistent
 * rollout workgroups x reduction workgroups, and with three- or four-wave
 * rollouts the stored and the regenerating average) over `reps` steps of the
 * whole batch with the given requests, keep the fastest, and report it and
 * its mean step time in ms; on a cache hit (no MPPI_TUNE_FORCE) apply the
 * cached shape and time nothing (*best_ms: the cached time, *from_cache 1).
 * The timed solves are real solves (they write d_u0s), but the warm-start
 * state and report of every context are restored afterwards. */
mppi_status mppi_batch_autotune(mppi_batch *b, const double *d_reqs, double *d_u0s, int32_t reps,
                                const char *cache_path, int32_t flags, mppi_batch_cfg *best, double *best_ms,
                                int32_t *from_cache);

void mppi_batch_destroy(mppi_batch *b);
const char *mppi_batch_last_error(const mppi_batch *b);

/* ---- Serving: continuous batching of solves from many drones ----
 *
 * The server owns no drone state: it registers contexts created with
 * MPPI_FLAG_EXTERNAL_WORKSPACE (one per drone, all of one precision; each
 * keeps its warm-start state, gate index and problem data resident on the
 * device).  Requests queue per drone in arrival order; a drone has at most
 * one solve in flight, since each solve starts from the previous one's warm
 * state.  mppi_server_progress retires finished launches and then, for every
 * idle launch slot (a stream with its own batch and graph), admits queued
 * heads in arrival order as long as their workspace (sample tensor, costs,
 * tile minima) fits in the free part of a device arena of budget_bytes, and
 * launches them as one batch.  A launch holds the drones of one class, that of
 * the oldest queued head: one rollout layout (mppi_info.rollout_waves and the
 * four-wave chunk, which each context picks from K at creation, or from
 * MPPI_ROLLOUT_WAVES) and one n_iter, and runs them in that layout.  Requests that arrive
 * while others run are admitted as slots and memory free up; the slots' work
 * overlaps on the device.  A solve's result is the same as that of the
 * context stepped alone, bit for bit. */
typedef struct mppi_server mppi_server;

typedef struct {
    double budget_bytes;   /* device arena lent to in-flight solves, > 0        */
    int32_t n_slots;       /* concurrent launches (streams), 1..16               */
    int32_t max_batch;     /* most solves per launch; 0: no limit                */
    int32_t use_graph;     /* capture each slot's launch sequence once           */
    int32_t pad_;
} mppi_server_cfg;

typedef struct {
    uint64_t ticket;       /* as returned by mppi_server_submit                  */
    int32_t drone;
    int32_t status;        /* MPPI_OK or MPPI_E_NONFINITE                        */
    double u0[4];          /* first input of the solution                        */
    double t_arrival;      /* caller's arrival time of the request               */
    double t_launch;       /* caller's clock when the solve was launched         */
    double t_done;         /* caller's clock when it was retired                 */
} mppi_result;

typedef struct {
    uint64_t submitted, completed, launches;
    int64_t queued, in_flight;
    double arena_bytes, peak_bytes_in_flight;
    double rollout_steps;  /* sum of K*N over completed solves                   */
} mppi_server_stats;

mppi_status mppi_server_create(mppi_ctx *const *drones, int32_t n, const mppi_server_cfg *cfg,
                               mppi_server **out);
/* Queue a solve of drone `drone` from state x0 at time t_now (the same
 * arguments as mppi_solve: 13 doubles, or 17 for a drone with the rate input,
 * its four thrusts last); t_arrival only stamps the result.  MPPI_E_NOMEM
 * when that drone's workspace alone exceeds the arena. */
mppi_status mppi_server_submit(mppi_server *s, int32_t drone, const double *x0, double t_now, double t_arrival,
                               uint64_t *ticket);
/* Retire finished launches (non-blocking) and launch what can be admitted;
 * `now` is the caller's clock, used only for the result stamps. */
mppi_status mppi_server_progress(mppi_server *s, double now, int32_t *n_launched);
/* Move up to max finished results into out (oldest first). */
mppi_status mppi_server_poll(mppi_server *s, mppi_result *out, int32_t max, int32_t *n_out);
/* Block until nothing is queued or in flight (calls progress). */
mppi_status mppi_server_drain(mppi_server *s, double now);
mppi_status mppi_server_get_stats(const mppi_server *s, mppi_server_stats *out);
void mppi_server_destroy(mppi_server *s);
const char *mppi_server_last_error(const mppi_server *s);

/* Human-readable description of the last error on this context ("" if none);
 * valid until the next call on the context.  ctx may be NULL (creation). */
const char *mppi_last_error(const mppi_ctx *ctx);

/* Static name of a status code; "MPPI_E_UNKNOWN" for any other integer (the
 * argument is an int so that a value outside the enumeration is defined). */
const char *mppi_status_string(int32_t s);

/* Host FP64 plant step of the paper's rate model (Sec. III-A) for closed-loop
 * simulation: x and x_out hold 17 states (the thrusts last), tdot the rotor
 * thrust rates in N/s held over dt.  Each of the `substeps` equal sub-steps
 * clips the rates to the range that keeps every thrust within [t_min, t_max]
 * (the rotors saturate), integrates the 17-state system with RK4 and
 * renormalises the quaternion.  x_out may alias x. */
mppi_status mppi_plant_step_rate(const mppi_quad *quad, const double x[17], const double tdot[4],
                                 double dt, int32_t substeps, double x_out[17]);

/* Host FP64 plant step for closed-loop simulation (not part of a solve):
 * integrates Eq. (2) with RK4 over dt with the input held, using `substeps`
 * equal sub-steps, and renormalises the quaternion.  x_out may alias x. */
mppi_status mppi_plant_step(const mppi_quad *quad, const double x[13], const double u[4],
                            double dt, int32_t substeps, double x_out[13]);

#ifdef __cplusplus
}
#endif
#endif /* MPPI_H */
