// Device-side data layout and small helpers of the MPPI step (gfx950).
//
// Memory of one context (all device-resident):
//   ctrl   N x K x 4 Real  sample controls U^m_k, step-major: element (k*K + m)*4 + c,
//          so a wavefront at fixed k reads / writes 64 consecutive 16 B (32 B) records
//   vctrl  N x K Real      contouring progress-speed samples, same order
//   nomU   N x 4 Real      clipped nominal sequence (the noise-free sample, lane K)
//   J      K Real          sample costs
//   tmin   ceil((K+1)/64) Real  smallest finite cost of each 64-sample rollout tile
//   warm   DevWarm + wU (N x 4 double) + wV (N double): what the next solve inherits
//   cur    DevCur: per-solve values decided once by the head and read by every kernel
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

constexpr int kNMax = 256;
constexpr int kMaskWords = 9;   // (kNMax + 1) bits
constexpr int kGMax = 256;      // most gates (the pipelined rollouts stage the table in LDS)
constexpr int kReqDoubles = 24;    // x0[13], t_now, 2 spare, thrusts[4] (rate model), 4 spare
constexpr int kFinalThreads = 1024;  // threads of a block of the weighted-average kernel
constexpr size_t kScratchBytes = (size_t)32 << 20;  // fixed workspace of the allocation-free solve

enum Objective { OBJ_GATE = 0, OBJ_CONTOUR = 1, OBJ_TRACK = 2 };
enum InputModel { INPUT_THRUST = 0, INPUT_RATE = 1 };
constexpr int kReqThrust = 16;      // request slots of the measured thrusts (rate model)
enum Status { ST_OK = 0, ST_INVAL = -1, ST_NOMEM = -2, ST_DEVICE = -3, ST_NONFINITE = -4 };

struct DevWarm {
    int32_t warm, g0;
    uint32_t s;
    int32_t N;
    uint32_t allow[kMaskWords];
    int32_t pad0;
    double t_prev, theta0;
    double x_prev[13];
    double vtheta;              // rate model, contouring: progress speed at the previous solve
};

struct DevCur {
    int32_t g0, i0, shift, warm;
    uint32_t s, pad0[3];
    uint32_t allow[kMaskWords];
    int32_t pad1;
    double theta0, t_now;
    double u_prev[4];
    double v_prev;
    double J_nom;
    double x0[13];
    double pad2;
};

struct DevResult {
    double u0[4];
    double J_min, S, S2, ess, J_nom, theta0;
    int32_t status, g0, i0, shift;
    uint32_t s, pad;
};

// Everything a kernel needs, passed by value (kernel arguments live in SGPRs).
// Floating constants are given in double and converted by the kernel template.
struct KArgs {
    int32_t K, N, G, P, R, objective;
    int32_t C, real_bytes;      // channels (4, 5 contouring); bytes of Real (for ws_layout)
    int32_t n_tiles;            // 64-sample rollout tiles: ceil((K + 1) / 64)
    int32_t ring4_b;            // chunk of the four-wave rollout: 4 or 2 steps (binary32)
    int32_t proj_window, has_drag;
    int32_t rollout_waves;      // 1: one wave per 64 samples; 2: attitude and translation on two waves; 3, 4
    int32_t regen;              // 1: no sample tensor; the weighted average draws the samples again
                                // (three- and four-wave layouts, whose rollout draws them)
    int32_t rollout_draw;       // 1: the one-wave rollout draws its samples (no sample kernel)
    int32_t inner;              // 1: an inner iteration of a control step (no shift, the first
                                // iteration's last applied input)
    int32_t input_model;        // INPUT_THRUST (13 states) or INPUT_RATE (thrust rates, 17 states)
    int32_t pad2_;
    uint32_t seed_lo, seed_hi;
    // model
    double inv_mass, gravity, arm_s, c_tau;
    double inv_J[3], gyro[3];   // 1/J_i and (J_z-J_y)/J_x, (J_x-J_z)/J_y, (J_y-J_x)/J_z
    double drag[3];
    double t_min, t_max, w_max, hover;
    // sampling
    double dt, lambda, sigma[4], sigma_v;
    // costs
    double w_lim, q_near, r_near, gate_half;
    double ctrl_cost;           // gamma of the control-cost term (0: off)
    double rate_lim[2];         // rate model: bounds of the sampled thrust rate, N/s
    double dv_lim[2];           // rate model, contouring: bounds of the progress acceleration
    double inv_sig2[5];         // 1/sigma_i^2 of the four thrusts and the speed, 0 where sigma_i = 0
    double Q[13], QN[13], R_dT[4];
    double q_l, q_c, Q_w[3], r_dv, mu, v_max;
    double path_len, ref_dt;
    // problem data
    const double *gates_d;      // G x 4 (as given), then G x 8 frames (centre, n, h, pad) for the head, FP64
    const void *gates_r;        // G x 8 Real: c, n.xy, h.xy, pad
    const double *path_d;       // P x 6 (head, FP64)
    const void *path_r;         // P x 8 Real: p, t, pad
    const void *xref_r;         // R x 16 Real
    // per-context state
    DevWarm *warm;
    double *wU, *wV;
    DevCur *cur;
    DevResult *res;
    void *ctrl, *vctrl, *nomU, *nomV, *J;
    void *tmin;                 // n_tiles Real: smallest finite sample cost per rollout tile
    uint8_t *front8;            // N + 1 bytes written by the nominal lane
    // per-call
    const double *req;          // x0[13], t_now
    double *u0_out;             // 4 doubles or null
};

// Per-solve scratch of one context, carved out of one block: the sample
// tensor, costs, tile minima and the nominal's front flags.  Offsets are
// multiples of 256 bytes.  rs: bytes of Real.
struct WsLayout {
    size_t ctrl, vctrl, nomU, nomV, J, tmin, front8, total;
};

__host__ __device__ inline WsLayout ws_layout(int K, int N, int C, int rs)
{
    WsLayout l;
    size_t o = 0;
    const size_t k = (size_t)K, n = (size_t)N;
    l.ctrl = o; o += (rs * 4 * k * n + 255) / 256 * 256;
    l.vctrl = o; o += C == 5 ? (rs * k * n + 255) / 256 * 256 : 0;
    l.nomU = o; o += (rs * 4 * n + 255) / 256 * 256;
    l.nomV = o; o += (rs * n + 255) / 256 * 256;
    l.J = o; o += (rs * k + 255) / 256 * 256;
    l.tmin = o; o += (rs * ((k + 1 + 63) / 64) + 255) / 256 * 256;
    l.front8 = o; o += (n + 1 + 255) / 256 * 256;
    l.total = o;
    return l;
}

// One solve of a batch: which context, where its request and first input
// live, and (when the context has none of its own) its workspace.
struct BatchItem {
    int32_t ctx;
    int32_t pad;
    const double *req;
    double *u0_out;
    char *ws;                   // null: the context's own workspace
};

// Work description of one launch group of a batch (one objective and one
// accumulation type), device-resident so that a captured launch sequence
// replays any batch composition.  Items are ordered by horizon, longest first.
struct BatchDesc {
    int32_t n;                  // items
    int32_t n_sample_units;     // sum over items of ceil((K+1)/256)
    int32_t n_tiles;            // sum over items of ceil((K+1)/64)
    int32_t n_steps;            // sum over items of N (units of the weighted-average kernel)
    uint32_t queue;             // rollout tile counter, reset by the sample kernel
    uint32_t sample_queue;      // sample unit counter (both also reset by the
                                // average kernel, for the step's next iteration)
    uint32_t pad[2];
};

struct BArgs {
    const KArgs *table;         // kernel arguments of every registered context
    BatchDesc *desc;
    const BatchItem *items;     // n entries
    const int32_t *sample_prefix, *tile_prefix, *step_prefix;  // n + 1 entries each
};

template <typename T> __device__ __forceinline__ T clampT(T v, T lo, T hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// clampT for a finite v and lo <= hi, in one instruction for binary32
// (median of three); equal to clampT for every finite v.
__device__ __forceinline__ float clamp_finite(float v, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}
__device__ __forceinline__ double clamp_finite(double v, double lo, double hi)
{
    return fmin(fmax(v, lo), hi);
}

// Compensated (Kahan) running sum.  For double the compensation is dropped.
template <typename Real> struct KSum {
    Real s = Real(0), c = Real(0);
    __device__ __forceinline__ void add(Real x)
    {
        Real y = x - c;
        Real t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ Real value() const { return s - c; }
};
template <> struct KSum<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double x) { s += x; }
    __device__ __forceinline__ double value() const { return s; }
};

// 1/sqrt(x): the hardware reciprocal square root in binary32 (about 1 ulp),
// the accurate quotient in binary64.
__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

// Rounding of the warm-start shift and reference row: floor(x + 1/2).
__device__ __forceinline__ int round_half_up(double x) { return (int)floor(x + 0.5); }

__device__ __forceinline__ int solve_shift(int warm, double t_now, double t_prev, double dt)
{
    if (!warm) return 0;
    double el = (t_now - t_prev) / dt;
    if (!(el < 1.0e6)) el = 1.0e6;  // keeps the conversion to int defined
    if (el < 0.0) el = 0.0;
    const int s = round_half_up(el);
    return s < 1 ? 1 : s;
}

}  // namespace mppi
