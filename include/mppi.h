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
#define MPPI_REQ_DOUBLES 16       /* device request record, see mppi_solve_device */

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
    int32_t precision;    /* MPPI_FP32 (compensated) or MPPI_FP64              */
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
    int32_t pad_;
} mppi_params;

/* Problem data: the inputs of Alg. 1 (waypoints W, path P_arc, tau_ref). */
typedef struct {
    const double *gates;  /* G x 4 row-major: centre x, y, z, yaw (gate objective) */
    int32_t n_gates;
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
    uint32_t pad_;
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
    double V[MPPI_N_MAX];              /* previous progress-speed solution, N    */
} mppi_warm;

/* Create a solver context.  Validates every argument (K, N, dt, lambda, sigma,
 * objective and the data it needs: G >= 1 gates, P >= 2 path points, R >= 1
 * reference rows), copies the problem data to the device and allocates all
 * device buffers: the N x K x 4 sample tensor (step-major: sample m of step k
 * at element (k*K + m)*4), K costs, the reduction partials and the warm-start
 * state.  stream is a hipStream_t (NULL: the library creates a non-blocking
 * stream of default priority that it owns).  The context starts cold with
 * target gate 0.  On failure *out is NULL. */
mppi_status mppi_create(const mppi_params *params, const mppi_quad *quad,
                        const mppi_problem *problem, void *stream,
                        const mppi_allocator *allocator, mppi_ctx **out);

/* Release every device and host resource of the context.  NULL is a no-op. */
void mppi_destroy(mppi_ctx *ctx);

/* One MPPI step from host memory, synchronous on the context stream.
 * x0: current state (finite, |q| > 0).  t_now: time of x0 in s; the previous
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
 * d_req: device pointer to MPPI_REQ_DOUBLES doubles, x0 in [0..12] and t_now
 * in [13] (the rest is ignored).  d_u0: device pointer receiving 4 doubles.
 * Both must stay valid until the stream reaches the end of the solve.  The
 * status and report of the solve are read later with mppi_read_info; a solve
 * whose costs are all non-finite leaves the warm-start state unchanged and
 * writes NaN to d_u0.  The call sequence is fixed, so it may be captured in a
 * HIP graph and replayed with new contents of d_req. */
mppi_status mppi_solve_device(mppi_ctx *ctx, const double *d_req, double *d_u0);

/* Wait for the context stream and copy the report of the latest solve. */
mppi_status mppi_read_info(mppi_ctx *ctx, mppi_info *info);

/* Copy the latest solve's sample costs (K doubles, as computed, in FP64
 * whatever the precision) and optionally the sample controls (N x K x 4
 * doubles, step-major).  Waits for the context stream. */
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

/* Human-readable description of the last error on this context ("" if none);
 * valid until the next call on the context.  ctx may be NULL (creation). */
const char *mppi_last_error(const mppi_ctx *ctx);

/* Static name of a status code. */
const char *mppi_status_string(mppi_status s);

/* Host FP64 plant step for closed-loop simulation (not part of a solve):
 * integrates Eq. (2) with RK4 over dt with the input held, using `substeps`
 * equal sub-steps, and renormalises the quaternion.  x_out may alias x. */
mppi_status mppi_plant_step(const mppi_quad *quad, const double x[13], const double u[4],
                            double dt, int32_t substeps, double x_out[13]);

#ifdef __cplusplus
}
#endif
#endif /* MPPI_H */
