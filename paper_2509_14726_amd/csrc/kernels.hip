// Kernels of one MPPI step on gfx950 (wave64).
//
//   k_setup          once per context: problem tables -> device layout in Real
//   k_rollout4       (default for small K) a 64-sample tile per workgroup, the
//                    step pipelined over four waves: noise and clipped samples
//                    (Eq. (3)), RK4 of Eq. (2) split into body rates, attitude
//                    and translation, per-step costs fused in (gate Eq. (6)-(7),
//                    tracking Eq. (8), contouring Eq. (9)); cost write and the
//                    smallest cost of the tile
//   k_rollout3       the same over three waves
//   k_sample +       (large K) noise and clipped samples for all (m, k), then
//   k_rollout /      one sample per lane (k_rollout) or attitude and
//   k_rollout_split  translation on two waves (k_rollout_split)
//   k_final          one block per horizon step: J_min from the tile minima,
//                    softmax weights (Eq. (4)), the weighted average (Eq. (5)),
//                    the first input, the report and the warm-start hand-over
//   kb_*             the same bodies as persistent kernels over a batch
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"
#include "noise.hpp"
#include "rollout.hpp"

namespace mppi {

template <typename Real> struct Vec4;
template <> struct Vec4<float> { using T = float4; };
template <> struct Vec4<double> { using T = double4; };

// Streaming (non-temporal) stores of the sample tensor from the pipelined
// rollouts: the tensor is read once, by the weighted-average kernel, and
// written this way it leaves no dirty L2 lines to write back when the rollout
// kernel ends.
__device__ __forceinline__ void store_nt(float4 *p, const float4 v)
{
    typedef float V __attribute__((ext_vector_type(4)));
    const V x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, (V *)p);
}
__device__ __forceinline__ void store_nt(double4 *p, const double4 v)
{
    typedef double V __attribute__((ext_vector_type(4)));
    const V x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, (V *)p);
}
__device__ __forceinline__ void store_nt(float *p, const float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(double *p, const double v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------- setup

template <typename Real> __global__ void k_setup(KArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.G && a.gates_d) {
        // gate frame (centre, normal n, lateral h) in binary64 for the head
        // and in Real for the rollouts; the yaw's cosine and sine are taken
        // once here
        const double *g = a.gates_d + 4 * i;
        double *f = (double *)a.gates_d + 4 * a.G + 8 * i;
        const double cy = cos(g[3]), sy = sin(g[3]);
        f[0] = g[0]; f[1] = g[1]; f[2] = g[2];
        f[3] = cy; f[4] = sy;
        f[5] = -sy; f[6] = cy;
        f[7] = 0.0;
        Real *o = (Real *)a.gates_r + 8 * i;
        o[0] = (Real)g[0]; o[1] = (Real)g[1]; o[2] = (Real)g[2];
        o[3] = (Real)cy; o[4] = (Real)sy;     // normal n
        o[5] = (Real)(-sy); o[6] = (Real)cy;  // lateral h
        o[7] = Real(0);
    }
    if (i < a.P && a.path_d) {
        const double *p = a.path_d + 6 * i;
        Real *o = (Real *)a.path_r + 8 * i;
        for (int c = 0; c < 6; ++c) o[c] = (Real)p[c];
        o[6] = o[7] = Real(0);
    }
    if (i < a.R && a.xref_r) {
        // the FP64 reference was staged in the upper half of the same buffer
        const double *r = (const double *)((const char *)a.xref_r + (size_t)a.R * 16 * sizeof(Real)) + 13 * i;
        Real *o = (Real *)a.xref_r + 16 * i;
        for (int c = 0; c < 13; ++c) o[c] = (Real)r[c];
        o[13] = o[14] = o[15] = Real(0);
    }
}

// ---------------------------------------------------------------- head

// Measured gate pass x_prev -> x0 (same geometry as the in-horizon switch);
// gate = the binary64 frame (centre, n, h) written at set-up.
__device__ bool gate_cross_d(const double *pa, const double *pb, const double *gate, double half)
{
    const double nx = gate[3], ny = gate[4];
    const double hx = gate[5], hy = gate[6];
    const double sa = (pa[0] - gate[0]) * nx + (pa[1] - gate[1]) * ny;
    const double sb = (pb[0] - gate[0]) * nx + (pb[1] - gate[1]) * ny;
    if (!(sa < 0.0 && sb >= 0.0)) return false;
    const double t = sa / (sa - sb);
    const double y0 = pa[0] + t * (pb[0] - pa[0]);
    const double y1 = pa[1] + t * (pb[1] - pa[1]);
    const double y2 = pa[2] + t * (pb[2] - pa[2]);
    const double lat = (y0 - gate[0]) * hx + (y1 - gate[1]) * hy;
    const double ver = y2 - gate[2];
    return fabs(lat) <= half && fabs(ver) <= half;
}

__device__ double wrap_len_d(double th, double L)
{
    double r = fmod(th, L);
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
    return r;
}

// What one solve inherits from the previous one, decided from the request and
// the warm-start state: warm-start shift, current gate and pass mask, start
// arc length, reference row, last applied input.
struct HeadVals {
    int32_t g0, i0, shift, warm;
    uint32_t s;
    uint32_t allow[kMaskWords];
    double theta0, t_now, v_prev;
    double u_prev[4];
    double x0[13];
};

// Steps the warm start is shifted by: none in an inner iteration of the same
// control step (the previous iteration ran at this time), else
// max(1, round(elapsed / dt)).
__device__ __forceinline__ int warm_shift(const KArgs &a, int warm, double t_now, double t_prev)
{
    if (a.inner && warm && t_prev == t_now) return 0;
    return solve_shift(warm, t_now, t_prev, a.dt);
}

// Rate model, contouring: the progress speed state at this solve's time, the
// previous solve's initial speed advanced over the shift by its averaged
// accelerations (clamped to [0, v_max] each step) and held beyond that
// solution's horizon; 0 at a cold start.
__device__ __forceinline__ double rate_speed0(const KArgs &a, const DevWarm *w, int warm, int shift)
{
    if (!warm) return 0.0;
    double v = w->vtheta;
    for (int j = 0; j < shift && j < a.N; ++j) v = clampT(v + a.dt * a.wV[j], 0.0, a.v_max);
    return v;
}

// Run by all threads of one block (any size up to 512); h is in LDS.  A
// kernel built for another objective than contouring passes CONTOUR = false
// and allocates no LDS for the projection.
template <bool CONTOUR = true> __device__ void compute_head(const KArgs &a, HeadVals &h)
{
    const int tid = threadIdx.x;
    const DevWarm *w = a.warm;
    const int warm = w->warm;

    double theta0 = 0.0;
    if (CONTOUR && a.objective == OBJ_CONTOUR) {
        __shared__ double s_d2[512];   // one entry per thread, up to 512 threads
        __shared__ double s_th[512];
        __shared__ int s_j[512];
        // the block size, read once (a read from the dispatch's implicit
        // arguments, which inside the barrier loop below would be repeated
        // at every barrier)
        const int nthr = (int)blockDim.x;
        const int P = a.P;
        const double L = a.path_len, ds = L / (double)P;
        const bool global = !warm;
        const int W = a.proj_window;
        int ic = 0;
        if (!global) {
            ic = (int)floor(wrap_len_d(w->theta0, L) / ds);
            if (ic >= P) ic = P - 1;
        }
        const int count = global ? P : 2 * W + 1;
        double best = INFINITY, best_th = 0.0;
        int best_j = 0x7fffffff;
        const double p0 = a.req[0], p1 = a.req[1], p2 = a.req[2];
        for (int j = tid; j < count; j += nthr) {
            const int i = global ? j : (((ic + (j - W)) % P) + P) % P;
            const int i1 = (i + 1) % P;
            const double *A = a.path_d + 6 * i, *B = a.path_d + 6 * i1;
            const double ab0 = B[0] - A[0], ab1 = B[1] - A[1], ab2 = B[2] - A[2];
            const double ap0 = p0 - A[0], ap1 = p1 - A[1], ap2 = p2 - A[2];
            const double l2 = ab0 * ab0 + ab1 * ab1 + ab2 * ab2;
            double t = l2 > 0.0 ? (ap0 * ab0 + ap1 * ab1 + ap2 * ab2) / l2 : 0.0;
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            const double d0 = ap0 - t * ab0, d1 = ap1 - t * ab1, d2 = ap2 - t * ab2;
            const double dd = d0 * d0 + d1 * d1 + d2 * d2;
            if (dd < best) { best = dd; best_th = ((double)i + t) * ds; best_j = j; }
        }
        s_d2[tid] = best; s_th[tid] = best_th; s_j[tid] = best_j;
        __syncthreads();
        // smallest distance, ties to the first candidate in search order
        for (int st = 256; st > 0; st >>= 1) {
            if (tid < st && tid + st < nthr) {
                const double d_o = s_d2[tid + st];
                const int j_o = s_j[tid + st];
                if (d_o < s_d2[tid] || (d_o == s_d2[tid] && j_o < s_j[tid])) {
                    s_d2[tid] = d_o; s_th[tid] = s_th[tid + st]; s_j[tid] = j_o;
                }
            }
            __syncthreads();
        }
        theta0 = wrap_len_d(s_th[0], L);
    }

    if (tid == 0) {
        const double t_now = a.req[13];
        int g0 = w->g0;
        uint32_t allow[kMaskWords];
        for (int j = 0; j < kMaskWords; ++j) allow[j] = warm ? w->allow[j] : 0xffffffffu;
        if (warm && a.objective == OBJ_GATE && g0 >= 0 && g0 < a.G &&
            gate_cross_d(w->x_prev, a.req, a.gates_d + 4 * a.G + 8 * g0, a.gate_half)) {
            g0 = (g0 + 1) % a.G;
            for (int j = 0; j < kMaskWords; ++j) allow[j] = 0xffffffffu;
        }
        int i0 = 0;
        if (a.objective == OBJ_TRACK) {
            double r = floor(t_now / a.ref_dt + 0.5);
            if (!(r >= 0.0)) r = 0.0;
            if (r > (double)(a.R - 1)) r = (double)(a.R - 1);
            i0 = (int)r;
        }
        h.g0 = g0;
        h.i0 = i0;
        h.shift = warm_shift(a, warm, t_now, w->t_prev);
        h.warm = warm;
        h.s = w->s;
        for (int j = 0; j < kMaskWords; ++j) h.allow[j] = allow[j];
        h.theta0 = theta0;
        h.t_now = t_now;
        // an inner iteration keeps the last applied input of the control step,
        // which the previous iteration published
        const bool same_step = a.inner && warm && w->t_prev == t_now;
        for (int i = 0; i < 4; ++i) h.u_prev[i] = same_step ? a.cur->u_prev[i] : (warm ? a.wU[i] : a.hover);
        h.v_prev = same_step ? a.cur->v_prev : (warm ? a.wV[0] : 0.0);
        // the rate model carries the progress speed state in v_prev
        if (a.input_model == INPUT_RATE) h.v_prev = rate_speed0(a, w, warm, h.shift);
        for (int i = 0; i < 13; ++i) h.x0[i] = a.req[i];
    }
    __syncthreads();
}

// Publish the head for the kernels that follow (thread 0 of one block).
__device__ void publish_head(const KArgs &a, const HeadVals &h)
{
    DevCur *c = a.cur;
    c->g0 = h.g0;
    c->i0 = h.i0;
    c->shift = h.shift;
    c->warm = h.warm;
    c->s = h.s;
    for (int j = 0; j < kMaskWords; ++j) c->allow[j] = h.allow[j];
    c->theta0 = h.theta0;
    c->t_now = h.t_now;
    for (int i = 0; i < 4; ++i) c->u_prev[i] = h.u_prev[i];
    c->v_prev = h.v_prev;
    for (int i = 0; i < 13; ++i) c->x0[i] = h.x0[i];
}

__device__ void solve_head(const KArgs &a)
{
    __shared__ HeadVals h;
    compute_head(a, h);
    if (threadIdx.x == 0) {
        publish_head(a, h);
        a.cur->J_nom = 0.0;
    }
}

// ---------------------------------------------------------------- sample

// One block of 256 samples over the steps [k0, k1); the block of the first
// samples and steps also runs the head.  The shifted warm start (R4 per step)
// is staged in LDS once, so each step is the noise and the clipped samples of
// 256 samples with one coalesced store.  Every sample and step is drawn from
// its own counters, so any split of the steps gives the same samples.
template <typename Real, bool HAS_V>
__device__ __forceinline__ void sample_body(const KArgs &a, int bx, int k0, int k1)
{
    typedef typename Vec4<Real>::T R4;
    __shared__ R4 s_us[kNMax];
    __shared__ Real s_vs[HAS_V ? kNMax : 1];
    if (bx == 0 && k0 == 0) solve_head(a);

    // nominal of this solve: the previous solution shifted, or hover (cold)
    const DevWarm *w = a.warm;
    const int warm = w->warm;
    const int shift = warm_shift(a, warm, a.req[13], w->t_prev);
    const uint32_t s = w->s;
    const int N = a.N, K = a.K;
    for (int k = k0 + (int)threadIdx.x; k < k1; k += blockDim.x) {
        int src = k + shift;
        if (src > N - 1) src = N - 1;
        R4 o;
        o.x = warm ? (Real)a.wU[4 * src + 0] : (Real)a.hover;
        o.y = warm ? (Real)a.wU[4 * src + 1] : (Real)a.hover;
        o.z = warm ? (Real)a.wU[4 * src + 2] : (Real)a.hover;
        o.w = warm ? (Real)a.wU[4 * src + 3] : (Real)a.hover;
        s_us[k] = o;
        if (HAS_V) s_vs[k] = warm ? (Real)a.wV[src] : Real(0);
    }
    __syncthreads();

    const int m = bx * 256 + threadIdx.x;
    const Real tmin = (Real)a.t_min, tmax = (Real)a.t_max;
    if (a.input_model == INPUT_RATE) {
        // the paper's input: thrust rates (and contouring's progress
        // acceleration) clipped to their bounds.  The clip to the range that
        // keeps each thrust within [t_min, t_max] (the speed within [0, v_max])
        // follows the sample's own thrust chain: the rollout applies it step
        // by step, where that chain is integrated, and writes the result back.
        if (m > K) return;
        const bool noisy = m < K;
        const Real rlo = (Real)a.rate_lim[0], rhi = (Real)a.rate_lim[1];
        const Real dlo = (Real)a.dv_lim[0], dhi = (Real)a.dv_lim[1];
        const Real sg[4] = {(Real)a.sigma[0], (Real)a.sigma[1], (Real)a.sigma[2], (Real)a.sigma[3]};
#pragma unroll 2
        for (int k = k0; k < k1; ++k) {
            const R4 us = s_us[k];
            const Real ust[4] = {us.x, us.y, us.z, us.w};
            Real z[4] = {Real(0), Real(0), Real(0), Real(0)};
            if (noisy) {
                const Normal4<Real> n4 = normals4<Real>((uint32_t)m, (uint32_t)k, s, 0u, a.seed_lo, a.seed_hi);
                z[0] = n4.z0; z[1] = n4.z1; z[2] = n4.z2; z[3] = n4.z3;
            }
            Real u[4];
            for (int i = 0; i < 4; ++i) u[i] = clampT(noisy ? ust[i] + sg[i] * z[i] : ust[i], rlo, rhi);
            R4 o;
            o.x = u[0]; o.y = u[1]; o.z = u[2]; o.w = u[3];
            if (noisy) ((R4 *)a.ctrl)[(size_t)k * (size_t)K + (size_t)m] = o;
            else ((R4 *)a.nomU)[k] = o;
            if (HAS_V) {
                Real zv = Real(0);
                if (noisy) zv = normal1<Real>((uint32_t)m, (uint32_t)k, s, 1u, a.seed_lo, a.seed_hi);
                const Real acc = clampT(noisy ? s_vs[k] + (Real)a.sigma_v * zv : s_vs[k], dlo, dhi);
                if (noisy) ((Real *)a.vctrl)[(size_t)k * (size_t)K + (size_t)m] = acc;
                else ((Real *)a.nomV)[k] = acc;
            }
        }
        return;
    }
    if (m == K) {  // the noise-free sample
        for (int k = k0; k < k1; ++k) {
            const R4 us = s_us[k];
            R4 o;
            o.x = clampT(us.x, tmin, tmax); o.y = clampT(us.y, tmin, tmax);
            o.z = clampT(us.z, tmin, tmax); o.w = clampT(us.w, tmin, tmax);
            ((R4 *)a.nomU)[k] = o;
            if (HAS_V) ((Real *)a.nomV)[k] = clampT(s_vs[k], Real(0), (Real)a.v_max);
        }
    } else if (m < K) {
        const Real sig0 = (Real)a.sigma[0], sig1 = (Real)a.sigma[1];
        const Real sig2 = (Real)a.sigma[2], sig3 = (Real)a.sigma[3];
#pragma unroll 2
        for (int k = k0; k < k1; ++k) {
            const R4 us = s_us[k];
            const Normal4<Real> z = normals4<Real>((uint32_t)m, (uint32_t)k, s, 0u, a.seed_lo, a.seed_hi);
            R4 o;
            o.x = clampT(us.x + sig0 * z.z0, tmin, tmax);
            o.y = clampT(us.y + sig1 * z.z1, tmin, tmax);
            o.z = clampT(us.z + sig2 * z.z2, tmin, tmax);
            o.w = clampT(us.w + sig3 * z.z3, tmin, tmax);
            const size_t idx = (size_t)k * (size_t)K + (size_t)m;
            ((R4 *)a.ctrl)[idx] = o;
            if (HAS_V) {
                const Real zv = normal1<Real>((uint32_t)m, (uint32_t)k, s, 1u, a.seed_lo, a.seed_hi);
                ((Real *)a.vctrl)[idx] = clampT(s_vs[k] + (Real)a.sigma_v * zv, Real(0), (Real)a.v_max);
            }
        }
    }
    __syncthreads();
}

// Steps per block of the sample kernel: the draws are independent, so the
// grid spreads them over (samples, steps) and every CU takes a share.
constexpr int kSampleSteps = 4;

template <typename Real, bool HAS_V> __global__ __launch_bounds__(256) void k_sample(KArgs a)
{
    const int k0 = (int)blockIdx.y * kSampleSteps;
    sample_body<Real, HAS_V>(a, blockIdx.x, k0, min(a.N, k0 + kSampleSteps));
}

// The head and the nominal's clipped inputs, for a rollout that draws its
// samples itself (one-wave layout): one block.
template <typename Real, bool HAS_V> __global__ __launch_bounds__(256) void k_head(KArgs a)
{
    typedef typename Vec4<Real>::T R4;
    __shared__ HeadVals h;
    compute_head(a, h);
    if (threadIdx.x == 0) {
        publish_head(a, h);
        a.cur->J_nom = 0.0;
    }
    const Real tmin = (Real)a.t_min, tmax = (Real)a.t_max;
    for (int k = threadIdx.x; k < a.N; k += blockDim.x) {
        int src = k + h.shift;
        if (src > a.N - 1) src = a.N - 1;
        R4 o;
        o.x = clampT(h.warm ? (Real)a.wU[4 * src + 0] : (Real)a.hover, tmin, tmax);
        o.y = clampT(h.warm ? (Real)a.wU[4 * src + 1] : (Real)a.hover, tmin, tmax);
        o.z = clampT(h.warm ? (Real)a.wU[4 * src + 2] : (Real)a.hover, tmin, tmax);
        o.w = clampT(h.warm ? (Real)a.wU[4 * src + 3] : (Real)a.hover, tmin, tmax);
        ((R4 *)a.nomU)[k] = o;
        if (HAS_V) ((Real *)a.nomV)[k] = clampT(h.warm ? (Real)a.wV[src] : Real(0), Real(0), (Real)a.v_max);
    }
}

// ---------------------------------------------------------------- rollout

// Minimum over the 64 lanes of a wave (all lanes active), returned to every
// lane.  Binary32 goes through DPP moves, each a few cycles instead of an
// LDS-crossbar round trip: two quad permutes ([1,0,3,2], [2,3,0,1]), row
// shifts by 4 and 8 (lane 15 of each row then holds the row's minimum), the
// broadcast of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3
// (lane 63 then holds the wave's minimum); a lane without a source keeps
// +inf.  Binary64 uses lane shuffles.  A minimum does not depend on the
// order of the comparisons, so either way every caller sees the same value.
template <int CTRL, int ROW_MASK = 0xf> __device__ __forceinline__ float dpp_or_inf(float v)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(INFINITY), __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

__device__ __forceinline__ float wave_min(float v)
{
    float o;
    o = dpp_or_inf<0xb1>(v);       v = o < v ? o : v;
    o = dpp_or_inf<0x4e>(v);       v = o < v ? o : v;
    o = dpp_or_inf<0x114>(v);      v = o < v ? o : v;
    o = dpp_or_inf<0x118>(v);      v = o < v ? o : v;
    o = dpp_or_inf<0x142, 0xa>(v); v = o < v ? o : v;
    o = dpp_or_inf<0x143, 0xc>(v); v = o < v ? o : v;
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// Smallest finite sample cost of a 64-sample tile (+inf when there is none),
// stored by lane 0 of the wave that holds the tile's costs.  The weighted
// average takes J_min as the minimum over tiles: no atomics, nothing to reset.
template <typename Real> __device__ __forceinline__ void store_tile_min(Real v, bool use, void *tmin, int tile)
{
    v = wave_min(use ? v : Real(INFINITY));
    if ((threadIdx.x & 63) == 0) ((Real *)tmin)[tile] = v;
}

template <typename Real> struct GateRegs {
    Real cx, cy, cz, nx, ny, hx, hy;
    __device__ __forceinline__ void load(const Real *tab, int g)
    {
        const Real *r = tab + 8 * g;
        cx = r[0]; cy = r[1]; cz = r[2]; nx = r[3]; ny = r[4]; hx = r[5]; hy = r[6];
    }
};

// One wave: samples 64*blk .. 64*blk+63 (sample K is the noise-free nominal).
// DRAW: the wave draws its samples itself (the noise, perturbation and clip
// of the sample kernel, same operations, one step ahead of the dynamics) and
// stores them for the weighted average with streaming stores; the shifted
// warm start is staged in LDS from the head that k_head published.
// Otherwise the wave reads the samples that the sample kernel stored.
template <int OBJ, typename Real, bool DRAW = false>
__device__ __forceinline__ void rollout1_body(const KArgs &a, int blk)
{
    typedef typename Vec4<Real>::T R4;
    constexpr bool HAS_V = OBJ == OBJ_CONTOUR;
    __shared__ R4 s_us[DRAW ? kNMax : 1];
    __shared__ Real s_vs[DRAW && HAS_V ? kNMax : 1];
    const int m = blk * 64 + (int)(threadIdx.x & 63);
    const int K = a.K, N = a.N;
    const bool active = m <= K;
    const bool nominal = m == K;
    const DevCur *cur = a.cur;
    Real Jfinal = Real(0);
    if (DRAW) {
        const int shift = cur->shift, warm = cur->warm;
        for (int k = (int)threadIdx.x; k < N; k += 64) {
            int src = k + shift;
            if (src > N - 1) src = N - 1;
            R4 o;
            o.x = warm ? (Real)a.wU[4 * src + 0] : (Real)a.hover;
            o.y = warm ? (Real)a.wU[4 * src + 1] : (Real)a.hover;
            o.z = warm ? (Real)a.wU[4 * src + 2] : (Real)a.hover;
            o.w = warm ? (Real)a.wU[4 * src + 3] : (Real)a.hover;
            s_us[k] = o;
            if (HAS_V) s_vs[k] = warm ? (Real)a.wV[src] : Real(0);
            // the weighted average draws the samples again from these rows
            if (a.regen && blk == (K >> 6)) {
                ((R4 *)a.nomU)[k] = o;
                if (HAS_V) ((Real *)a.nomV)[k] = s_vs[k];
            }
        }
        __syncthreads();
    }

    if (active) {
        const Model<Real> M(a);
        const Real dt = (Real)a.dt;
        const Real w_max = (Real)a.w_max, w_lim = (Real)a.w_lim;
        State<Real> st;
        load_state(st, cur->x0);
        KSum<Real> J;

        const R4 *urow = nominal ? (const R4 *)a.nomU : (const R4 *)a.ctrl + m;
        const size_t ustride = nominal ? 1 : (size_t)K;
        const Real *vrow = nullptr;
        if (OBJ == OBJ_CONTOUR) vrow = nominal ? (const Real *)a.nomV : (const Real *)a.vctrl + m;
        // the inputs (u, V) of step k: drawn (and stored, unless the weighted
        // average draws them again) or read.  Drawing, the nominal clips the
        // staged rows itself (the values the head kernel wrote to nomU / nomV,
        // which then hold the unclipped rows of the regenerating average).
        const bool keep = !a.regen;
        const uint32_t s_solve = cur->s;
        const Real tmin = (Real)a.t_min, tmax = (Real)a.t_max;
        const Real sig0 = (Real)a.sigma[0], sig1 = (Real)a.sigma[1];
        const Real sig2 = (Real)a.sigma[2], sig3 = (Real)a.sigma[3];
        auto input = [&](const int k, R4 &uo, Real &vo) {
            if (DRAW && nominal) {
                const R4 us = s_us[k];
                uo.x = clampT(us.x, tmin, tmax);
                uo.y = clampT(us.y, tmin, tmax);
                uo.z = clampT(us.z, tmin, tmax);
                uo.w = clampT(us.w, tmin, tmax);
                if (HAS_V) vo = clampT(s_vs[k], Real(0), (Real)a.v_max);
            } else if (DRAW) {
                const R4 us = s_us[k];
                const Normal4<Real> z = normals4<Real>((uint32_t)m, (uint32_t)k, s_solve, 0u, a.seed_lo, a.seed_hi);
                uo.x = clampT(us.x + sig0 * z.z0, tmin, tmax);
                uo.y = clampT(us.y + sig1 * z.z1, tmin, tmax);
                uo.z = clampT(us.z + sig2 * z.z2, tmin, tmax);
                uo.w = clampT(us.w + sig3 * z.z3, tmin, tmax);
                const size_t idx = (size_t)k * (size_t)K + (size_t)m;
                if (keep) store_nt(&((R4 *)a.ctrl)[idx], uo);
                if (HAS_V) {
                    const Real zv = normal1<Real>((uint32_t)m, (uint32_t)k, s_solve, 1u, a.seed_lo, a.seed_hi);
                    vo = clampT(s_vs[k] + (Real)a.sigma_v * zv, Real(0), (Real)a.v_max);
                    if (keep) store_nt(&((Real *)a.vctrl)[idx], vo);
                }
            } else {
                uo = urow[(size_t)k * ustride];
                if (HAS_V) vo = vrow[(size_t)k * ustride];
            }
        };

        // gate objective state
        const Real *gtab = (const Real *)a.gates_r;
        GateRegs<Real> gt, g0r;
        int g = 0, passes = 0;
        Real q_near = 0, r_near2 = 0, half = 0;
        if (OBJ == OBJ_GATE) {
            g = cur->g0;
            gt.load(gtab, g);
            g0r = gt;
            q_near = (Real)a.q_near;
            r_near2 = (Real)(a.r_near * a.r_near);
            half = (Real)a.gate_half;
        }
        // tracking / contouring state
        Real up[4];
        for (int i = 0; i < 4; ++i) up[i] = (Real)cur->u_prev[i];
        Real vp = (Real)cur->v_prev;
        Real rdt[4];
        for (int i = 0; i < 4; ++i) rdt[i] = (Real)(a.R_dT[i] / (a.dt * a.dt));
        const int i0 = cur->i0;
        const Real *xref = (const Real *)a.xref_r;
        const Real *path = (const Real *)a.path_r;
        // arc length theta = th_hi + th_lo (th_lo stays 0 in binary64)
        Real th_hi = 0, th_lo = 0;
        Real ds = 0, inv_ds = 0, L = 0;
        if (OBJ == OBJ_CONTOUR) {
            th_hi = (Real)cur->theta0;
            if (sizeof(Real) == 4) th_lo = (Real)(cur->theta0 - (double)th_hi);
            L = (Real)a.path_len;
            ds = (Real)(a.path_len / (double)a.P);
            inv_ds = (Real)((double)a.P / a.path_len);
        }

        // rate model: the thrust states and the progress speed state, carried
        // in binary64 in every precision (integrators: in binary32 their
        // rounding over the horizon reaches the attitude through the small
        // inertia and the position through the attitude)
        const bool rate = a.input_model == INPUT_RATE;
        double T[4];
        for (int i = 0; i < 4; ++i) T[i] = rate ? a.req[kReqThrust + i] : 0.0;
        double vs = rate ? cur->v_prev : 0.0;

        // the rate input's range clips (multiplied by 1/dt: the bound can
        // differ from the quotient in the last binary64 place)
        const double inv_dt = 1.0 / a.dt;
        R4 u;
        Real v = Real(0);
        input(0, u, v);
        for (int k = 0; k < N; ++k) {
            R4 un = u;
            Real vn = v;
            if (k + 1 < N) input(k + 1, un, vn);
            if (rate) {
                // clip the drawn rates to the range that keeps each thrust of
                // this sample's chain within [t_min, t_max] over the step (the
                // progress acceleration: the speed within [0, v_max]); the
                // clipped inputs replace the drawn ones for the average
                u.x = (Real)clampT((double)u.x, (a.t_min - T[0]) * inv_dt, (a.t_max - T[0]) * inv_dt);
                u.y = (Real)clampT((double)u.y, (a.t_min - T[1]) * inv_dt, (a.t_max - T[1]) * inv_dt);
                u.z = (Real)clampT((double)u.z, (a.t_min - T[2]) * inv_dt, (a.t_max - T[2]) * inv_dt);
                u.w = (Real)clampT((double)u.w, (a.t_min - T[3]) * inv_dt, (a.t_max - T[3]) * inv_dt);
                if (HAS_V) v = (Real)clampT((double)v, (0.0 - vs) * inv_dt, (a.v_max - vs) * inv_dt);
                if (nominal) {
                    ((R4 *)a.nomU)[k] = u;
                    if (HAS_V) ((Real *)a.nomV)[k] = v;
                } else {
                    ((R4 *)a.ctrl)[(size_t)k * (size_t)K + (size_t)m] = u;
                    if (HAS_V) ((Real *)a.vctrl)[(size_t)k * (size_t)K + (size_t)m] = v;
                }
            }
            Real term = Real(0);

            // ---- stage terms at state k
            Real ax = 0, ay = 0, az = 0;  // p_k - c_g (gate)
            if (OBJ == OBJ_GATE) {
                ax = st.x[0] - gt.cx;
                ay = st.x[1] - gt.cy;
                az = st.x[2] - gt.cz;
                const Real bx = st.x[0] - g0r.cx;
                const Real by = st.x[1] - g0r.cy;
                const Real bz = st.x[2] - g0r.cz;
                const Real d2 = bx * bx + by * by + bz * bz;
                if (d2 < r_near2) term += q_near * d2;  // Eq. (7), current gate
                if (nominal) a.front8[k] = (bx * g0r.nx + by * g0r.ny) < Real(0);
            } else if (OBJ == OBJ_TRACK) {
                int r = i0 + k;
                if (r > a.R - 1) r = a.R - 1;
                const Real *xr = xref + 16 * r;
#pragma unroll
                for (int i = 0; i < 13; ++i) {
                    const Real e = st.x[i] - xr[i];
                    term += (Real)a.Q[i] * e * e;
                }
                if (rate) {  // Eq. (8)'s u_k is the sampled thrust rate
                    term += (Real)a.R_dT[0] * u.x * u.x + (Real)a.R_dT[1] * u.y * u.y + (Real)a.R_dT[2] * u.z * u.z +
                            (Real)a.R_dT[3] * u.w * u.w;
                } else {
                    const Real d0 = u.x - up[0], d1 = u.y - up[1], d2 = u.z - up[2], d3 = u.w - up[3];
                    term += rdt[0] * d0 * d0 + rdt[1] * d1 * d1 + rdt[2] * d2 * d2 + rdt[3] * d3 * d3;
                }
            } else {  // contouring
                const Real fl = floor(th_hi * inv_ds);
                const Real f = ((th_hi - fl * ds) + th_lo) * inv_ds;
                // table row of theta, always inside [0, P)
                int i = (fl >= Real(0) && fl < Real(1 << 30)) ? ((int)fl % a.P) : 0;
                const int i1 = (i + 1 == a.P) ? 0 : i + 1;
                const Real *A = path + 8 * i, *B = path + 8 * i1;
                const Real g1 = Real(1) - f;
                const Real px = g1 * A[0] + f * B[0], py = g1 * A[1] + f * B[1], pz = g1 * A[2] + f * B[2];
                Real tx = g1 * A[3] + f * B[3], ty = g1 * A[4] + f * B[4], tz = g1 * A[5] + f * B[5];
                const Real tn = inv_sqrt(tx * tx + ty * ty + tz * tz);
                tx *= tn; ty *= tn; tz *= tn;
                const Real ex = st.x[0] - px;
                const Real ey = st.x[1] - py;
                const Real ez = st.x[2] - pz;
                const Real et = ex * tx + ey * ty + ez * tz;
                const Real lx = et * tx, ly = et * ty, lz = et * tz;
                const Real cxe = ex - lx, cye = ey - ly, cze = ez - lz;
                term += (Real)a.q_l * (lx * lx + ly * ly + lz * lz);
                term += (Real)a.q_c * (cxe * cxe + cye * cye + cze * cze);
                term += (Real)a.Q_w[0] * st.x[10] * st.x[10] + (Real)a.Q_w[1] * st.x[11] * st.x[11] +
                        (Real)a.Q_w[2] * st.x[12] * st.x[12];
                const Real vk = v;
                Real adv;  // arc length advanced over the step
                if (rate) {
                    // Eq. (9) with the progress acceleration as the input and
                    // the speed as a state, which moves linearly over the step
                    term += (Real)a.r_dv * vk * vk;
                    term += (Real)a.R_dT[0] * u.x * u.x + (Real)a.R_dT[1] * u.y * u.y + (Real)a.R_dT[2] * u.z * u.z +
                            (Real)a.R_dT[3] * u.w * u.w;
                    term -= (Real)a.mu * (Real)vs;
                    const double vsn = vs + a.dt * (double)vk;
                    adv = (Real)(0.5 * a.dt * (vs + vsn));
                    vs = vsn;
                } else {
                    const Real dv = vk - vp;
                    term += (Real)(a.r_dv / (a.dt * a.dt)) * dv * dv;
                    const Real d0 = u.x - up[0], d1 = u.y - up[1], d2 = u.z - up[2], d3 = u.w - up[3];
                    term += rdt[0] * d0 * d0 + rdt[1] * d1 * d1 + rdt[2] * d2 * d2 + rdt[3] * d3 * d3;
                    term -= (Real)a.mu * vk;
                    adv = vk * dt;
                }
                vp = vk;
                {   // theta_{k+1} = theta_k + advance (mod L), compensated in binary32
                    const Real y = adv + th_lo;
                    const Real t = th_hi + y;
                    th_lo = (sizeof(Real) == 4) ? y - (t - th_hi) : Real(0);
                    th_hi = t;
                    if (th_hi >= L) th_hi -= L;
                }
            }

            // ---- dynamics
            Real dx[13];
            if (rate) {
                // the thrusts move linearly over the step: RK4 of the 17-state
                // system sees them at the start, middle and end of the step
                const double h = 0.5 * a.dt, ur[4] = {(double)u.x, (double)u.y, (double)u.z, (double)u.w};
                const StepInput<Real> in1 = step_input(M, (Real)T[0], (Real)T[1], (Real)T[2], (Real)T[3]);
                const StepInput<Real> in2 = step_input(M, (Real)(T[0] + h * ur[0]), (Real)(T[1] + h * ur[1]),
                                                       (Real)(T[2] + h * ur[2]), (Real)(T[3] + h * ur[3]));
                const StepInput<Real> in4 = step_input(M, (Real)(T[0] + a.dt * ur[0]), (Real)(T[1] + a.dt * ur[1]),
                                                       (Real)(T[2] + a.dt * ur[2]), (Real)(T[3] + a.dt * ur[3]));
                rk4_increment_stages(M, in1, in2, in4, st.x, dt, dx);
                for (int i = 0; i < 4; ++i) T[i] += a.dt * ur[i];
            } else {
                const StepInput<Real> in = step_input(M, u.x, u.y, u.z, u.w);
                rk4_increment(M, in, st.x, dt, dx);
            }
            commit(st, dx);

            // ---- progress and switching (gate)
            if (OBJ == OBJ_GATE) {
                // |p_{k+1} - c|^2 - |p_k - c|^2 = dp . (2 (p_k - c) + dp)
                term += dx[0] * (Real(2) * ax + dx[0]) + dx[1] * (Real(2) * ay + dx[1]) +
                        dx[2] * (Real(2) * az + dx[2]);
                const Real sa = ax * gt.nx + ay * gt.ny;
                const Real sb = (ax + dx[0]) * gt.nx + (ay + dx[1]) * gt.ny;
                if (sa < Real(0) && sb >= Real(0)) {
                    const Real t = sa / (sa - sb);
                    const Real yx = ax + t * dx[0], yy = ay + t * dx[1], yz = az + t * dx[2];
                    const Real lat = yx * gt.hx + yy * gt.hy;
                    const bool inside = fabs(lat) <= half && fabs(yz) <= half;
                    const int j = k + 1;
                    const bool allowed = passes > 0 || ((cur->allow[j >> 5] >> (j & 31)) & 1u);
                    if (inside && allowed) {
                        g = (g + 1 == a.G) ? 0 : g + 1;
                        ++passes;
                        gt.load(gtab, g);
                    }
                }
            }
            // ---- body-rate penalty on the new state
#pragma unroll
            for (int i = 10; i < 13; ++i) {
                const Real e = fmax(fabs(st.x[i]) - w_max, Real(0));
                term += w_lim * e * e;
            }
            J.add(term);
            up[0] = u.x; up[1] = u.y; up[2] = u.z; up[3] = u.w;
            u = un;
            v = vn;
        }
        if (OBJ == OBJ_TRACK) {
            int r = i0 + N;
            if (r > a.R - 1) r = a.R - 1;
            const Real *xr = xref + 16 * r;
            Real term = 0;
#pragma unroll
            for (int i = 0; i < 13; ++i) {
                const Real e = st.x[i] - xr[i];
                term += (Real)a.QN[i] * e * e;
            }
            J.add(term);
        }
        if (OBJ == OBJ_GATE && nominal) {
            const Real bx = st.x[0] - g0r.cx;
            const Real by = st.x[1] - g0r.cy;
            a.front8[N] = (bx * g0r.nx + by * g0r.ny) < Real(0);
        }
        Jfinal = J.value();
        if (nominal) a.cur->J_nom = (double)Jfinal;
        else ((Real *)a.J)[m] = Jfinal;
    }
    // smallest finite sample cost of the tile
    store_tile_min(Jfinal, active && !nominal && isfinite(Jfinal), a.tmin, blk);
}

template <int OBJ, typename Real, bool DRAW> __global__ __launch_bounds__(64) void k_rollout(KArgs a)
{
    rollout1_body<OBJ, Real, DRAW>(a, blockIdx.x);
}

// ---------------------------------------------------------------- rollout, two waves

// The rotational subsystem (q, omega) of Eq. (2) does not depend on position
// or velocity, so one sample's rollout splits over two waves of a workgroup:
// wave 0 integrates (q, omega) and hands the four RK4 stage quaternions of
// every step to wave 1 through an LDS ring of B steps; wave 1 integrates
// (p, v) from them and evaluates the position-dependent cost terms.  Each
// wave accumulates the cost terms of its own state components; the two
// partial costs are added at the end.  The arithmetic of every component is
// the same as in the one-wave rollout; only the two halves run concurrently
// on two SIMDs, which halves the critical path of a step.
template <typename Real> struct SplitRing;
template <> struct SplitRing<float> { static constexpr int B = 8; };
template <> struct SplitRing<double> { static constexpr int B = 4; };

template <int OBJ, typename Real> __device__ __forceinline__ void rollout2_body(const KArgs &a, int blk)
{
    typedef typename Vec4<Real>::T R4;
    constexpr int B = SplitRing<Real>::B;
    __shared__ R4 s_q[2][B][4][64];
    __shared__ Real s_jr[64];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = blk * 64 + lane;
    const int K = a.K, N = a.N;
    const bool active = m <= K;
    const bool nominal = m == K;
    const DevCur *cur = a.cur;
    const Model<Real> M(a);
    const Real dt = (Real)a.dt;
    const Real h2 = Real(0.5) * dt;
    const Real dt6 = dt / Real(6);
    const Real h4 = Real(0.5) * h2, dt12 = Real(0.5) * dt6;
    const Real w_max = (Real)a.w_max, w_lim = (Real)a.w_lim;
    const bool use_nom = m >= K;  // lanes past K read the nominal row, results unused
    const R4 *urow = use_nom ? (const R4 *)a.nomU : (const R4 *)a.ctrl + m;
    const size_t ustride = use_nom ? 1 : (size_t)K;
    const Real *xref = (const Real *)a.xref_r;
    const int i0 = cur->i0;
    Real rdt[4];
    for (int i = 0; i < 4; ++i) rdt[i] = (Real)(a.R_dT[i] / (a.dt * a.dt));

    KSum<Real> J;
    // ---- wave 0: attitude and body rates
    Real q[4], w[3], up[4];
    // ---- wave 1: position and velocity
    Real p[3], v[3];
    GateRegs<Real> gt, g0r;
    int g = 0, passes = 0;
    Real vp = 0, th_hi = 0, th_lo = 0, ds = 0, inv_ds = 0, L = 0;
    const Real *vrow = nullptr;
    const Real *gtab = (const Real *)a.gates_r;
    const Real *path = (const Real *)a.path_r;
    {
        const double *x0 = cur->x0;
        for (int i = 0; i < 4; ++i) {
            q[i] = (Real)x0[6 + i];
        }
        for (int i = 0; i < 3; ++i) {
            w[i] = (Real)x0[10 + i];
            p[i] = (Real)x0[i];
            v[i] = (Real)x0[3 + i];
        }
        for (int i = 0; i < 4; ++i) up[i] = (Real)cur->u_prev[i];
    }
    if (wave == 1) {
        if (OBJ == OBJ_GATE) {
            g = cur->g0;
            gt.load(gtab, g);
            g0r = gt;
        }
        if (OBJ == OBJ_CONTOUR) {
            vrow = use_nom ? (const Real *)a.nomV : (const Real *)a.vctrl + m;
            vp = (Real)cur->v_prev;
            th_hi = (Real)cur->theta0;
            if (sizeof(Real) == 4) th_lo = (Real)(cur->theta0 - (double)th_hi);
            L = (Real)a.path_len;
            ds = (Real)(a.path_len / (double)a.P);
            inv_ds = (Real)((double)a.P / a.path_len);
        }
    }
    const Real q_near = (Real)a.q_near, r_near2 = (Real)(a.r_near * a.r_near), half = (Real)a.gate_half;

    const int nch = (N + B - 1) / B;
    // the control of the next step is always in flight while a step computes
    R4 u_next = urow[0];
    Real v_next = Real(0);
    if (OBJ == OBJ_CONTOUR && wave == 1) v_next = vrow[0];
    for (int c = 0; c <= nch; ++c) {
        if (wave == 0 && c < nch) {
            const int kb = c * B, ke = min(N, kb + B);
            for (int k = kb; k < ke; ++k) {
                R4 (*slot)[64] = s_q[c & 1][k - kb];
                const R4 u = u_next;
                if (k + 1 < N) u_next = urow[(size_t)(k + 1) * ustride];
                Real term = Real(0);
                if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const Real e = q[i] - xr[6 + i];
                        term += (Real)a.Q[6 + i] * e * e;
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = w[i] - xr[10 + i];
                        term += (Real)a.Q[10 + i] * e * e;
                    }
                }
                if (OBJ == OBJ_CONTOUR)
                    term += (Real)a.Q_w[0] * w[0] * w[0] + (Real)a.Q_w[1] * w[1] * w[1] +
                            (Real)a.Q_w[2] * w[2] * w[2];
                if (OBJ != OBJ_GATE) {
                    const Real d0 = u.x - up[0], d1 = u.y - up[1], d2 = u.z - up[2], d3 = u.w - up[3];
                    term += rdt[0] * d0 * d0 + rdt[1] * d1 * d1 + rdt[2] * d2 * d2 + rdt[3] * d3 * d3;
                }
                const StepInput<Real> in = step_input(M, u.x, u.y, u.z, u.w);
                // RK4 on (q, omega)
                Real ws[3], qs[4], kw[3], kq[4], dw[3], dq[4];
#pragma unroll
                for (int i = 0; i < 3; ++i) ws[i] = w[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) qs[i] = q[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    R4 o;
                    o.x = qs[0]; o.y = qs[1]; o.z = qs[2]; o.w = qs[3];
                    slot[st][lane] = o;
                    kw[0] = in.tx - M.gx * ws[1] * ws[2];
                    kw[1] = in.ty - M.gy * ws[2] * ws[0];
                    kw[2] = in.tz - M.gz * ws[0] * ws[1];
                    // kq is twice the quaternion rate; the factor 1/2 is
                    // carried by the step sizes (exact: a power of two)
                    kq[0] = -qs[1] * ws[0] - qs[2] * ws[1] - qs[3] * ws[2];
                    kq[1] = qs[0] * ws[0] + qs[2] * ws[2] - qs[3] * ws[1];
                    kq[2] = qs[0] * ws[1] - qs[1] * ws[2] + qs[3] * ws[0];
                    kq[3] = qs[0] * ws[2] + qs[1] * ws[1] - qs[2] * ws[0];
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] = kw[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = kq[i];
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] += Real(2) * kw[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] += Real(2) * kq[i];
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] = dt6 * (dw[i] + kw[i]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = dt12 * (dq[i] + kq[i]);
                    }
                    if (st < 3) {
                        const Real hh = st < 2 ? h2 : dt;
                        const Real hq = st < 2 ? h4 : h2;
#pragma unroll
                        for (int i = 0; i < 3; ++i) ws[i] = w[i] + hh * kw[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) qs[i] = q[i] + hq * kq[i];
                    }
                }
                // commit the step, unit quaternion
#pragma unroll
                for (int i = 0; i < 3; ++i) w[i] += dw[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) q[i] += dq[i];
                renormalize(q);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const Real e = fmax(fabs(w[i]) - w_max, Real(0));
                    term += w_lim * e * e;
                }
                J.add(term);
                up[0] = u.x; up[1] = u.y; up[2] = u.z; up[3] = u.w;
            }
        } else if (wave == 1 && c >= 1) {
            const int kb = (c - 1) * B, ke = min(N, kb + B);
            for (int k = kb; k < ke; ++k) {
                R4 (*slot)[64] = s_q[(c - 1) & 1][k - kb];
                const R4 u = u_next;
                if (k + 1 < N) u_next = urow[(size_t)(k + 1) * ustride];
                R4 qstage[4];
#pragma unroll
                for (int st = 0; st < 4; ++st) qstage[st] = slot[st][lane];
                const Real fm = ((u.x + u.y) + (u.z + u.w)) * M.inv_m;
                Real term = Real(0);
                Real ax = 0, ay = 0, az = 0;
                if (OBJ == OBJ_GATE) {
                    ax = p[0] - gt.cx;
                    ay = p[1] - gt.cy;
                    az = p[2] - gt.cz;
                    const Real bx = p[0] - g0r.cx;
                    const Real by = p[1] - g0r.cy;
                    const Real bz = p[2] - g0r.cz;
                    const Real d2 = bx * bx + by * by + bz * bz;
                    if (d2 < r_near2) term += q_near * d2;
                    if (nominal) a.front8[k] = (bx * g0r.nx + by * g0r.ny) < Real(0);
                } else if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = p[i] - xr[i];
                        term += (Real)a.Q[i] * e * e;
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = v[i] - xr[3 + i];
                        term += (Real)a.Q[3 + i] * e * e;
                    }
                } else {
                    const Real fl = floor(th_hi * inv_ds);
                    const Real f = ((th_hi - fl * ds) + th_lo) * inv_ds;
                    const int i = (fl >= Real(0) && fl < Real(1 << 30)) ? ((int)fl % a.P) : 0;
                    const int i1 = (i + 1 == a.P) ? 0 : i + 1;
                    const Real *A = path + 8 * i, *Bp = path + 8 * i1;
                    const Real g1 = Real(1) - f;
                    const Real px = g1 * A[0] + f * Bp[0], py = g1 * A[1] + f * Bp[1], pz = g1 * A[2] + f * Bp[2];
                    Real tx = g1 * A[3] + f * Bp[3], ty = g1 * A[4] + f * Bp[4], tz = g1 * A[5] + f * Bp[5];
                    const Real tn = inv_sqrt(tx * tx + ty * ty + tz * tz);
                    tx *= tn; ty *= tn; tz *= tn;
                    const Real ex = p[0] - px;
                    const Real ey = p[1] - py;
                    const Real ez = p[2] - pz;
                    const Real et = ex * tx + ey * ty + ez * tz;
                    const Real lx = et * tx, ly = et * ty, lz = et * tz;
                    const Real cxe = ex - lx, cye = ey - ly, cze = ez - lz;
                    term += (Real)a.q_l * (lx * lx + ly * ly + lz * lz);
                    term += (Real)a.q_c * (cxe * cxe + cye * cye + cze * cze);
                    const Real vk = v_next;
                    if (k + 1 < N) v_next = vrow[(size_t)(k + 1) * ustride];
                    const Real dv = vk - vp;
                    term += (Real)(a.r_dv / (a.dt * a.dt)) * dv * dv;
                    term -= (Real)a.mu * vk;
                    vp = vk;
                    const Real y = vk * dt + th_lo;
                    const Real t = th_hi + y;
                    th_lo = (sizeof(Real) == 4) ? y - (t - th_hi) : Real(0);
                    th_hi = t;
                    if (th_hi >= L) th_hi -= L;
                }
                // RK4 on (p, v) with the stage quaternions of wave 0
                Real vs[3], kv[3], dpv[3], dvv[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) vs[i] = v[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const R4 qq = qstage[st];
                    const Real r3x = Real(2) * (qq.y * qq.w + qq.x * qq.z);
                    const Real r3y = Real(2) * (qq.z * qq.w - qq.x * qq.y);
                    const Real r3z = Real(1) - Real(2) * (qq.y * qq.y + qq.z * qq.z);
                    kv[0] = fm * r3x;
                    kv[1] = fm * r3y;
                    kv[2] = fm * r3z - M.g;
                    if (M.drag) {
                        const Real qw = qq.x, qx = qq.y, qy = qq.z, qz = qq.w;
                        const Real r11 = Real(1) - Real(2) * (qy * qy + qz * qz), r12 = Real(2) * (qx * qy - qw * qz);
                        const Real r21 = Real(2) * (qx * qy + qw * qz), r22 = Real(1) - Real(2) * (qx * qx + qz * qz);
                        const Real r31 = Real(2) * (qx * qz - qw * qy), r32 = Real(2) * (qy * qz + qw * qx);
                        const Real b0 = M.d0 * (r11 * vs[0] + r21 * vs[1] + r31 * vs[2]);
                        const Real b1 = M.d1 * (r12 * vs[0] + r22 * vs[1] + r32 * vs[2]);
                        const Real b2 = M.d2 * (r3x * vs[0] + r3y * vs[1] + r3z * vs[2]);
                        kv[0] -= r11 * b0 + r12 * b1 + r3x * b2;
                        kv[1] -= r21 * b0 + r22 * b1 + r3y * b2;
                        kv[2] -= r31 * b0 + r32 * b1 + r3z * b2;
                    }
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] = vs[i]; dvv[i] = kv[i]; }
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] += Real(2) * vs[i]; dvv[i] += Real(2) * kv[i]; }
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] = dt6 * (dpv[i] + vs[i]); dvv[i] = dt6 * (dvv[i] + kv[i]); }
                    }
                    if (st < 3) {
                        const Real hh = st < 2 ? h2 : dt;
#pragma unroll
                        for (int i = 0; i < 3; ++i) vs[i] = v[i] + hh * kv[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    p[i] += dpv[i];
                    v[i] += dvv[i];
                }
                if (OBJ == OBJ_GATE) {
                    term += dpv[0] * (Real(2) * ax + dpv[0]) + dpv[1] * (Real(2) * ay + dpv[1]) +
                            dpv[2] * (Real(2) * az + dpv[2]);
                    const Real sa = ax * gt.nx + ay * gt.ny;
                    const Real sb = (ax + dpv[0]) * gt.nx + (ay + dpv[1]) * gt.ny;
                    if (sa < Real(0) && sb >= Real(0)) {
                        const Real t = sa / (sa - sb);
                        const Real yx = ax + t * dpv[0], yy = ay + t * dpv[1], yz = az + t * dpv[2];
                        const Real lat = yx * gt.hx + yy * gt.hy;
                        const bool inside = fabs(lat) <= half && fabs(yz) <= half;
                        const int j = k + 1;
                        const bool allowed = passes > 0 || ((cur->allow[j >> 5] >> (j & 31)) & 1u);
                        if (inside && allowed) {
                            g = (g + 1 == a.G) ? 0 : g + 1;
                            ++passes;
                            gt.load(gtab, g);
                        }
                    }
                }
                J.add(term);
            }
        }
        __syncthreads();
    }

    // terminal terms, then the two partial costs are added
    if (OBJ == OBJ_TRACK) {
        int r = i0 + N;
        if (r > a.R - 1) r = a.R - 1;
        const Real *xr = xref + 16 * r;
        Real term = 0;
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const Real e = q[i] - xr[6 + i];
                term += (Real)a.QN[6 + i] * e * e;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const Real e = w[i] - xr[10 + i];
                term += (Real)a.QN[10 + i] * e * e;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const Real e = p[i] - xr[i];
                term += (Real)a.QN[i] * e * e;
                const Real f = v[i] - xr[3 + i];
                term += (Real)a.QN[3 + i] * f * f;
            }
        }
        J.add(term);
    }
    if (wave == 0) s_jr[lane] = J.value();
    __syncthreads();
    if (wave == 1) {
        Real Jfinal = Real(0);
        if (active) {
            Jfinal = J.value() + s_jr[lane];
            if (OBJ == OBJ_GATE && nominal) {
                const Real bx = p[0] - g0r.cx;
                const Real by = p[1] - g0r.cy;
                a.front8[N] = (bx * g0r.nx + by * g0r.ny) < Real(0);
            }
            if (nominal) a.cur->J_nom = (double)Jfinal;
            else ((Real *)a.J)[m] = Jfinal;
        }
        store_tile_min(Jfinal, active && !nominal && isfinite(Jfinal), a.tmin, blk);
    }
}

template <int OBJ, typename Real> __global__ __launch_bounds__(128) void k_rollout_split(KArgs a)
{
    rollout2_body<OBJ, Real>(a, blockIdx.x);
}

// ---------------------------------------------------------------- rollout, three waves

// Sampling joins the rollout: per 64-sample tile, wave 0 draws the noise and
// the clipped controls of every step (Eq. (3)), stores them in the sample
// tensor for the weighted average and hands the step's collective thrust over
// mass and torques over inertia to the other waves through an LDS ring;
// wave 1 integrates (q, omega) and hands on the RK4 stage quaternions; wave 2
// integrates (p, v) and evaluates the position costs.  Each wave accumulates
// the cost terms of what it computes (wave 0: control-rate and progress-speed
// terms; wave 1: attitude and body-rate terms; wave 2: position terms); the
// three partial costs are added at the end.  Every workgroup derives the
// per-solve head itself; workgroup 0 publishes it for the tail.
template <typename Real> struct Ring3;
template <> struct Ring3<float> { static constexpr int B = 8; };
template <> struct Ring3<double> { static constexpr int B = 4; };

template <int OBJ, typename Real>
__device__ __forceinline__ void rollout3_body(const KArgs &a, int blk, const HeadVals &h)
{
    typedef typename Vec4<Real>::T R4;
    constexpr int B = Ring3<Real>::B;
    constexpr bool HAS_V = OBJ == OBJ_CONTOUR;
    __shared__ R4 s_in[3][B][64];                  // (F/m, tau_x/J_x, tau_y/J_y, tau_z/J_z)
    __shared__ Real s_v[HAS_V ? 3 : 1][B][64];     // progress speed
    __shared__ R4 s_q[2][B][4][64];                // stage quaternions
    __shared__ Real s_jp[2][64];                   // partial costs of waves 0 and 1
    __shared__ R4 s_us[kNMax];                     // shifted warm-start thrusts per step
    __shared__ Real s_vs[HAS_V ? kNMax : 1];       // shifted warm-start progress speed
    __shared__ Real s_gtab[OBJ == OBJ_GATE ? 8 * kGMax : 1];   // the gate table, staged once
    __shared__ uint8_t s_f8[OBJ == OBJ_GATE ? kNMax : 1];      // front flags of the nominal, steps 0..N-1

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = blk * 64 + lane;
    const int K = a.K, N = a.N;
    const bool active = m <= K;
    const bool nominal = m == K;
    const bool sampled = m < K;
    const Model<Real> M(a);
    const Real dt = (Real)a.dt;
    const Real h2 = Real(0.5) * dt;
    const Real dt6 = dt / Real(6);
    const Real h4 = Real(0.5) * h2, dt12 = Real(0.5) * dt6;
    const Real w_max = (Real)a.w_max, w_lim = (Real)a.w_lim;
    const Real *xref = (const Real *)a.xref_r;
    const int i0 = h.i0;
    Real rdt[4];
    for (int i = 0; i < 4; ++i) rdt[i] = (Real)(a.R_dT[i] / (a.dt * a.dt));
    const Real r_dv = (Real)(a.r_dv / (a.dt * a.dt));

    KSum<Real> J;
    // wave 0: sampling
    Real up[4], vp = (Real)h.v_prev;
    for (int i = 0; i < 4; ++i) up[i] = (Real)h.u_prev[i];
    // wave 1: attitude and body rates; wave 2: position and velocity
    Real q[4], w[3], p[3], v[3];
    for (int i = 0; i < 4; ++i) {
        q[i] = (Real)h.x0[6 + i];
    }
    for (int i = 0; i < 3; ++i) {
        w[i] = (Real)h.x0[10 + i];
        p[i] = (Real)h.x0[i];
        v[i] = (Real)h.x0[3 + i];
    }
    GateRegs<Real> gt, g0r;
    int g = 0, passes = 0;
    const Real *gtab = (const Real *)a.gates_r;
    const Real *path = (const Real *)a.path_r;
    Real th_hi = 0, th_lo = 0, ds = 0, inv_ds = 0, L = 0;
    if (OBJ == OBJ_GATE) g = h.g0;
    if (OBJ == OBJ_CONTOUR) {
        th_hi = (Real)h.theta0;
        if (sizeof(Real) == 4) th_lo = (Real)(h.theta0 - (double)th_hi);
        L = (Real)a.path_len;
        ds = (Real)(a.path_len / (double)a.P);
        inv_ds = (Real)((double)a.P / a.path_len);
    }
    const Real q_near = (Real)a.q_near, r_near2 = (Real)(a.r_near * a.r_near), half = (Real)a.gate_half;
    const Real tmin = (Real)a.t_min, tmax = (Real)a.t_max, vmax = (Real)a.v_max;
    const Real sig0 = (Real)a.sigma[0], sig1 = (Real)a.sigma[1], sig2 = (Real)a.sigma[2], sig3 = (Real)a.sigma[3];
    const Real sigv = (Real)a.sigma_v, hover = (Real)a.hover;
    typedef typename Vec4<Real>::T R4g;
    R4g *ctrl = (R4g *)a.ctrl;
    Real *vctrl = (Real *)a.vctrl;

    // the gate table in LDS: a gate switch inside the pipeline then waits on
    // no global load (which would also wait on the wave's sample stores)
    if (OBJ == OBJ_GATE)
        for (int i = threadIdx.x; i < 8 * a.G; i += blockDim.x) s_gtab[i] = gtab[i];
    // the shifted warm start (Alg. 1, warm start) of every step, staged once
    // so that the sampling wave reads it from LDS instead of waiting on a
    // dependent global load per step
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        int src = k + h.shift;
        if (src > N - 1) src = N - 1;
        R4 o;
        o.x = h.warm ? (Real)a.wU[4 * src + 0] : hover;
        o.y = h.warm ? (Real)a.wU[4 * src + 1] : hover;
        o.z = h.warm ? (Real)a.wU[4 * src + 2] : hover;
        o.w = h.warm ? (Real)a.wU[4 * src + 3] : hover;
        s_us[k] = o;
        if (HAS_V) s_vs[k] = h.warm ? (Real)a.wV[src] : Real(0);
        // the weighted average regenerates the samples from these rows
        if (a.regen && blk == (K >> 6)) {
            ((R4 *)a.nomU)[k] = o;
            if (HAS_V) ((Real *)a.nomV)[k] = s_vs[k];
        }
    }
    __syncthreads();
    if (OBJ == OBJ_GATE) {
        gt.load(s_gtab, g);
        g0r = gt;
    }

    const int nch = (N + B - 1) / B;
    for (int c = 0; c <= nch + 1; ++c) {
        if (wave == 0 && c < nch) {
            const int kb = c * B, ke = min(N, kb + B);
            auto noise_step = [&](const int k, const int j) {
                const R4 w4 = s_us[k];
                const Real us[4] = {w4.x, w4.y, w4.z, w4.w};
                const Real vs = HAS_V ? s_vs[k] : Real(0);
                R4 u;
                Real V = Real(0);
                if (sampled) {
                    const Normal4<Real> z = normals4<Real>((uint32_t)m, (uint32_t)k, h.s, 0u, a.seed_lo, a.seed_hi);
                    u.x = clampT(us[0] + sig0 * z.z0, tmin, tmax);
                    u.y = clampT(us[1] + sig1 * z.z1, tmin, tmax);
                    u.z = clampT(us[2] + sig2 * z.z2, tmin, tmax);
                    u.w = clampT(us[3] + sig3 * z.z3, tmin, tmax);
                    const size_t idx = (size_t)k * (size_t)K + (size_t)m;
                    if (!a.regen) store_nt(&ctrl[idx], u);
                    if (HAS_V) {
                        const Real zv = normal1<Real>((uint32_t)m, (uint32_t)k, h.s, 1u, a.seed_lo, a.seed_hi);
                        V = clampT(vs + sigv * zv, Real(0), vmax);
                        if (!a.regen) store_nt(&vctrl[idx], V);
                    }
                } else {  // the noise-free nominal (and idle lanes past it)
                    u.x = clampT(us[0], tmin, tmax);
                    u.y = clampT(us[1], tmin, tmax);
                    u.z = clampT(us[2], tmin, tmax);
                    u.w = clampT(us[3], tmin, tmax);
                    if (HAS_V) V = clampT(vs, Real(0), vmax);
                }
                if (HAS_V) s_v[c % 3][j][lane] = V;
                if (OBJ != OBJ_GATE) {
                    const Real d0 = u.x - up[0], d1 = u.y - up[1], d2 = u.z - up[2], d3 = u.w - up[3];
                    Real term = rdt[0] * d0 * d0 + rdt[1] * d1 * d1 + rdt[2] * d2 * d2 + rdt[3] * d3 * d3;
                    if (HAS_V) {
                        const Real dv = V - vp;
                        term += r_dv * dv * dv;
                        term -= (Real)a.mu * V;
                        vp = V;
                    }
                    J.add(term);
                    up[0] = u.x; up[1] = u.y; up[2] = u.z; up[3] = u.w;
                }
                const StepInput<Real> in = step_input(M, u.x, u.y, u.z, u.w);
                R4 o;
                o.x = in.fm; o.y = in.tx; o.z = in.ty; o.w = in.tz;
                s_in[c % 3][j][lane] = o;
            };
            if (ke - kb == B) {
#pragma unroll
                for (int j = 0; j < B; ++j) noise_step(kb + j, j);
            } else {
                for (int k = kb; k < ke; ++k) noise_step(k, k - kb);
            }
        } else if (wave == 1 && c >= 1 && c <= nch) {
            const int kb = (c - 1) * B, ke = min(N, kb + B);
            auto rot_step = [&](const int k, const int j) {
                const R4 in = s_in[(c - 1) % 3][j][lane];
                R4 (*slot)[64] = s_q[(c - 1) & 1][j];
                Real term = Real(0);
                if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const Real e = q[i] - xr[6 + i];
                        term += (Real)a.Q[6 + i] * e * e;
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = w[i] - xr[10 + i];
                        term += (Real)a.Q[10 + i] * e * e;
                    }
                }
                if (OBJ == OBJ_CONTOUR)
                    term += (Real)a.Q_w[0] * w[0] * w[0] + (Real)a.Q_w[1] * w[1] * w[1] +
                            (Real)a.Q_w[2] * w[2] * w[2];
                Real ws[3], qs[4], kw[3], kq[4], dw[3], dq[4];
#pragma unroll
                for (int i = 0; i < 3; ++i) ws[i] = w[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) qs[i] = q[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    R4 o;
                    o.x = qs[0]; o.y = qs[1]; o.z = qs[2]; o.w = qs[3];
                    slot[st][lane] = o;
                    kw[0] = in.y - M.gx * ws[1] * ws[2];
                    kw[1] = in.z - M.gy * ws[2] * ws[0];
                    kw[2] = in.w - M.gz * ws[0] * ws[1];
                    // kq is twice the quaternion rate; the factor 1/2 is
                    // carried by the step sizes (exact: a power of two)
                    kq[0] = -qs[1] * ws[0] - qs[2] * ws[1] - qs[3] * ws[2];
                    kq[1] = qs[0] * ws[0] + qs[2] * ws[2] - qs[3] * ws[1];
                    kq[2] = qs[0] * ws[1] - qs[1] * ws[2] + qs[3] * ws[0];
                    kq[3] = qs[0] * ws[2] + qs[1] * ws[1] - qs[2] * ws[0];
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] = kw[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = kq[i];
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] += Real(2) * kw[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] += Real(2) * kq[i];
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] = dt6 * (dw[i] + kw[i]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = dt12 * (dq[i] + kq[i]);
                    }
                    if (st < 3) {
                        const Real hh = st < 2 ? h2 : dt;
                        const Real hq = st < 2 ? h4 : h2;
#pragma unroll
                        for (int i = 0; i < 3; ++i) ws[i] = w[i] + hh * kw[i];
#pragma unroll
                        for (int i = 0; i < 4; ++i) qs[i] = q[i] + hq * kq[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) w[i] += dw[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) q[i] += dq[i];
                renormalize(q);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const Real e = fmax(fabs(w[i]) - w_max, Real(0));
                    term += w_lim * e * e;
                }
                J.add(term);
            };
            if (ke - kb == B) {
#pragma unroll
                for (int j = 0; j < B; ++j) rot_step(kb + j, j);
            } else {
                for (int k = kb; k < ke; ++k) rot_step(k, k - kb);
            }
        } else if (wave == 2 && c >= 2) {
            const int kb = (c - 2) * B, ke = min(N, kb + B);
            auto trans_step = [&](const int k, const int j) {
                const R4 in = s_in[(c - 2) % 3][j][lane];
                R4 qstage[4];
#pragma unroll
                for (int st = 0; st < 4; ++st) qstage[st] = s_q[(c - 2) & 1][j][st][lane];
                const Real fm = in.x;
                Real term = Real(0);
                Real ax = 0, ay = 0, az = 0;
                if (OBJ == OBJ_GATE) {
                    ax = p[0] - gt.cx;
                    ay = p[1] - gt.cy;
                    az = p[2] - gt.cz;
                    const Real bx = p[0] - g0r.cx;
                    const Real by = p[1] - g0r.cy;
                    const Real bz = p[2] - g0r.cz;
                    const Real d2 = bx * bx + by * by + bz * bz;
                    if (d2 < r_near2) term += q_near * d2;
                    if (nominal) s_f8[k] = (bx * g0r.nx + by * g0r.ny) < Real(0);
                } else if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = p[i] - xr[i];
                        term += (Real)a.Q[i] * e * e;
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = v[i] - xr[3 + i];
                        term += (Real)a.Q[3 + i] * e * e;
                    }
                } else {
                    const Real vk = s_v[(c - 2) % 3][j][lane];
                    const Real fl = floor(th_hi * inv_ds);
                    const Real f = ((th_hi - fl * ds) + th_lo) * inv_ds;
                    const int i = (fl >= Real(0) && fl < Real(1 << 30)) ? ((int)fl % a.P) : 0;
                    const int i1 = (i + 1 == a.P) ? 0 : i + 1;
                    const Real *A = path + 8 * i, *Bp = path + 8 * i1;
                    const Real g1 = Real(1) - f;
                    const Real px = g1 * A[0] + f * Bp[0], py = g1 * A[1] + f * Bp[1], pz = g1 * A[2] + f * Bp[2];
                    Real tx = g1 * A[3] + f * Bp[3], ty = g1 * A[4] + f * Bp[4], tz = g1 * A[5] + f * Bp[5];
                    const Real tn = inv_sqrt(tx * tx + ty * ty + tz * tz);
                    tx *= tn; ty *= tn; tz *= tn;
                    const Real ex = p[0] - px;
                    const Real ey = p[1] - py;
                    const Real ez = p[2] - pz;
                    const Real et = ex * tx + ey * ty + ez * tz;
                    const Real lx = et * tx, ly = et * ty, lz = et * tz;
                    const Real cxe = ex - lx, cye = ey - ly, cze = ez - lz;
                    term += (Real)a.q_l * (lx * lx + ly * ly + lz * lz);
                    term += (Real)a.q_c * (cxe * cxe + cye * cye + cze * cze);
                    const Real y = vk * dt + th_lo;
                    const Real t = th_hi + y;
                    th_lo = (sizeof(Real) == 4) ? y - (t - th_hi) : Real(0);
                    th_hi = t;
                    if (th_hi >= L) th_hi -= L;
                }
                Real vs[3], kv[3], dpv[3], dvv[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) vs[i] = v[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const R4 qq = qstage[st];
                    const Real r3x = Real(2) * (qq.y * qq.w + qq.x * qq.z);
                    const Real r3y = Real(2) * (qq.z * qq.w - qq.x * qq.y);
                    const Real r3z = Real(1) - Real(2) * (qq.y * qq.y + qq.z * qq.z);
                    kv[0] = fm * r3x;
                    kv[1] = fm * r3y;
                    kv[2] = fm * r3z - M.g;
                    if (M.drag) {
                        const Real qw = qq.x, qx = qq.y, qy = qq.z, qz = qq.w;
                        const Real r11 = Real(1) - Real(2) * (qy * qy + qz * qz), r12 = Real(2) * (qx * qy - qw * qz);
                        const Real r21 = Real(2) * (qx * qy + qw * qz), r22 = Real(1) - Real(2) * (qx * qx + qz * qz);
                        const Real r31 = Real(2) * (qx * qz - qw * qy), r32 = Real(2) * (qy * qz + qw * qx);
                        const Real b0 = M.d0 * (r11 * vs[0] + r21 * vs[1] + r31 * vs[2]);
                        const Real b1 = M.d1 * (r12 * vs[0] + r22 * vs[1] + r32 * vs[2]);
                        const Real b2 = M.d2 * (r3x * vs[0] + r3y * vs[1] + r3z * vs[2]);
                        kv[0] -= r11 * b0 + r12 * b1 + r3x * b2;
                        kv[1] -= r21 * b0 + r22 * b1 + r3y * b2;
                        kv[2] -= r31 * b0 + r32 * b1 + r3z * b2;
                    }
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] = vs[i]; dvv[i] = kv[i]; }
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] += Real(2) * vs[i]; dvv[i] += Real(2) * kv[i]; }
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] = dt6 * (dpv[i] + vs[i]); dvv[i] = dt6 * (dvv[i] + kv[i]); }
                    }
                    if (st < 3) {
                        const Real hh = st < 2 ? h2 : dt;
#pragma unroll
                        for (int i = 0; i < 3; ++i) vs[i] = v[i] + hh * kv[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    p[i] += dpv[i];
                    v[i] += dvv[i];
                }
                if (OBJ == OBJ_GATE) {
                    term += dpv[0] * (Real(2) * ax + dpv[0]) + dpv[1] * (Real(2) * ay + dpv[1]) +
                            dpv[2] * (Real(2) * az + dpv[2]);
                    const Real sa = ax * gt.nx + ay * gt.ny;
                    const Real sb = (ax + dpv[0]) * gt.nx + (ay + dpv[1]) * gt.ny;
                    if (sa < Real(0) && sb >= Real(0)) {
                        const Real t = sa / (sa - sb);
                        const Real yx = ax + t * dpv[0], yy = ay + t * dpv[1], yz = az + t * dpv[2];
                        const Real lat = yx * gt.hx + yy * gt.hy;
                        const bool inside = fabs(lat) <= half && fabs(yz) <= half;
                        const int jj = k + 1;
                        const bool allowed = passes > 0 || ((h.allow[jj >> 5] >> (jj & 31)) & 1u);
                        if (inside && allowed) {
                            g = (g + 1 == a.G) ? 0 : g + 1;
                            ++passes;
                            gt.load(s_gtab, g);
                        }
                    }
                }
                J.add(term);
            };
            if (ke - kb == B) {
#pragma unroll
                for (int j = 0; j < B; ++j) trans_step(kb + j, j);
            } else {
                for (int k = kb; k < ke; ++k) trans_step(k, k - kb);
            }
        }
        __syncthreads();
    }

    if (OBJ == OBJ_TRACK && wave > 0) {
        int r = i0 + N;
        if (r > a.R - 1) r = a.R - 1;
        const Real *xr = xref + 16 * r;
        Real term = 0;
        if (wave == 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const Real e = q[i] - xr[6 + i];
                term += (Real)a.QN[6 + i] * e * e;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const Real e = w[i] - xr[10 + i];
                term += (Real)a.QN[10 + i] * e * e;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const Real e = p[i] - xr[i];
                term += (Real)a.QN[i] * e * e;
                const Real f = v[i] - xr[3 + i];
                term += (Real)a.QN[3 + i] * f * f;
            }
        }
        J.add(term);
    }
    if (wave < 2) s_jp[wave][lane] = J.value();
    __syncthreads();
    if (wave == 2) {
        Real Jfinal = Real(0);
        if (active) {
            Jfinal = (s_jp[0][lane] + s_jp[1][lane]) + J.value();
            if (OBJ == OBJ_GATE && nominal) {
                const Real bx = p[0] - g0r.cx;
                const Real by = p[1] - g0r.cy;
                a.front8[N] = (bx * g0r.nx + by * g0r.ny) < Real(0);
            }
            if (nominal) a.cur->J_nom = (double)Jfinal;
            else ((Real *)a.J)[m] = Jfinal;
        }
        // the tile of the nominal writes its front flags of steps 0..N-1
        if (OBJ == OBJ_GATE && blk == (K >> 6))
            for (int i = lane; i < N; i += 64) a.front8[i] = s_f8[i];
        store_tile_min(Jfinal, active && !nominal && isfinite(Jfinal), a.tmin, blk);
    }
    __syncthreads();
}

// ---------------------------------------------------------------- rollout, four-wave pipeline

// The step of Eq. (2) split into four pipeline stages over four waves (one
// per SIMD), a 64-sample tile per workgroup, chunks of B steps between
// workgroup barriers.  At chunk iteration c:
//   wave 0  draws the noise of the even steps of chunk c (Eq. (3)) and
//           integrates the body rates over chunk c-1 (they depend on the
//           torques only), with the rate-limit and body-rate cost terms;
//   wave 3  draws the noise of the odd steps of chunk c and adds the
//           position cost terms of chunk c-4 (gate progress, near-gate
//           term, crossing and switch; contouring) and the input-rate terms;
//   wave 1  integrates the attitude over chunk c-2 from the stage body rates;
//   wave 2  integrates position and velocity over chunk c-3 from the stage
//           attitudes, with the tracking terms of position and velocity.
// Each stage hands its stage values on through LDS rings; every quantity is
// computed with the same operations as in the three-wave layout, whatever the
// chunk size B: the chunking only moves the barriers.  B = 4 for binary32
// with one workgroup per CU; B = 2 halves the rings so that two workgroups
// share a CU (binary32 with more tiles than CUs; always for binary64, whose
// rings are twice as large).
template <int OBJ, typename Real, int B>
__device__ __forceinline__ void rollout4_body(const KArgs &a, int blk, const HeadVals &h)
{
    typedef typename Vec4<Real>::T R4;
    constexpr bool HAS_V = OBJ == OBJ_CONTOUR;
    constexpr bool RATE = OBJ != OBJ_GATE;
    constexpr bool POS = OBJ != OBJ_TRACK;        // position costs in wave 3
    __shared__ R4 s_in[4][B][64];                  // (F/m, tau_x/J_x, tau_y/J_y, tau_z/J_z), chunk c at c % 4
    __shared__ R4 s_w[2][B][4][64];                // stage body rates, chunk c at c % 2
    __shared__ R4 s_q[2][B][4][64];                // stage quaternions, chunk c at c % 2
    __shared__ R4 s_p[POS ? 2 : 1][B][2][64];      // p_k and its increment; chunk c at c % 2
    __shared__ R4 s_u[RATE ? 5 : 1][B][64];        // clipped inputs, chunk c at c % 5
    __shared__ Real s_v[HAS_V ? 5 : 1][B][64];     // progress speed, chunk c at c % 5
    __shared__ R4 s_us[kNMax];                     // shifted warm-start thrusts per step
    __shared__ Real s_vs[HAS_V ? kNMax : 1];       // shifted warm-start progress speed
    __shared__ Real s_jp[3][64];                   // partial costs of waves 0, 1, 2
    __shared__ R4 s_pN[64];                        // p_N (front flag of the nominal)
    __shared__ Real s_gtab[OBJ == OBJ_GATE ? 8 * kGMax : 1];   // the gate table, staged once
    __shared__ uint8_t s_f8[OBJ == OBJ_GATE ? kNMax : 1];      // front flags of the nominal, steps 0..N-1

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = blk * 64 + lane;
    const int K = a.K, N = a.N;
    const bool active = m <= K;
    const bool nominal = m == K;
    const bool sampled = m < K;
    const Model<Real> M(a);
    const Real dt = (Real)a.dt;
    const Real h2 = Real(0.5) * dt;
    const Real dt6 = dt / Real(6);
    const Real h4 = Real(0.5) * h2, dt12 = Real(0.5) * dt6;
    const Real w_max = (Real)a.w_max, w_lim = (Real)a.w_lim;
    const Real *xref = (const Real *)a.xref_r;
    const int i0 = h.i0;
    Real rdt[4];
    for (int i = 0; i < 4; ++i) rdt[i] = (Real)(a.R_dT[i] / (a.dt * a.dt));
    const Real r_dv = (Real)(a.r_dv / (a.dt * a.dt));

    KSum<Real> J;
    Real up[4], vp = (Real)h.v_prev;
    for (int i = 0; i < 4; ++i) up[i] = (Real)h.u_prev[i];
    Real q[4], w[3], p[3], v[3];
    for (int i = 0; i < 4; ++i) {
        q[i] = (Real)h.x0[6 + i];
    }
    for (int i = 0; i < 3; ++i) {
        w[i] = (Real)h.x0[10 + i];
        p[i] = (Real)h.x0[i];
        v[i] = (Real)h.x0[3 + i];
    }
    GateRegs<Real> gt, g0r;
    int g = 0, passes = 0;
    const Real *gtab = (const Real *)a.gates_r;
    const Real *path = (const Real *)a.path_r;
    Real th_hi = 0, th_lo = 0, ds = 0, inv_ds = 0, L = 0;
    if (OBJ == OBJ_GATE) g = h.g0;
    if (OBJ == OBJ_CONTOUR) {
        th_hi = (Real)h.theta0;
        if (sizeof(Real) == 4) th_lo = (Real)(h.theta0 - (double)th_hi);
        L = (Real)a.path_len;
        ds = (Real)(a.path_len / (double)a.P);
        inv_ds = (Real)((double)a.P / a.path_len);
    }
    const Real q_near = (Real)a.q_near, r_near2 = (Real)(a.r_near * a.r_near), half = (Real)a.gate_half;
    const Real tmin = (Real)a.t_min, tmax = (Real)a.t_max, vmax = (Real)a.v_max;
    const Real sig0 = (Real)a.sigma[0], sig1 = (Real)a.sigma[1], sig2 = (Real)a.sigma[2], sig3 = (Real)a.sigma[3];
    const Real sigv = (Real)a.sigma_v, hover = (Real)a.hover;
    typedef typename Vec4<Real>::T R4g;
    R4g *ctrl = (R4g *)a.ctrl;
    Real *vctrl = (Real *)a.vctrl;

    // the gate table in LDS: a gate switch inside the pipeline then waits on
    // no global load (which would also wait on the wave's sample stores)
    if (OBJ == OBJ_GATE)
        for (int i = threadIdx.x; i < 8 * a.G; i += blockDim.x) s_gtab[i] = gtab[i];
    // the shifted warm start of every step, staged once
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        int src = k + h.shift;
        if (src > N - 1) src = N - 1;
        R4 o;
        o.x = h.warm ? (Real)a.wU[4 * src + 0] : hover;
        o.y = h.warm ? (Real)a.wU[4 * src + 1] : hover;
        o.z = h.warm ? (Real)a.wU[4 * src + 2] : hover;
        o.w = h.warm ? (Real)a.wU[4 * src + 3] : hover;
        s_us[k] = o;
        if (HAS_V) s_vs[k] = h.warm ? (Real)a.wV[src] : Real(0);
        // the weighted average regenerates the samples from these rows
        if (a.regen && blk == (K >> 6)) {
            ((R4 *)a.nomU)[k] = o;
            if (HAS_V) ((Real *)a.nomV)[k] = s_vs[k];
        }
    }
    __syncthreads();
    if (OBJ == OBJ_GATE) {
        gt.load(s_gtab, g);
        g0r = gt;
    }

    const int nch = (N + B - 1) / B;
    for (int c = 0; c <= nch + 3; ++c) {
        // The draws.  With eight waves (one workgroup per CU), waves 4-7 draw
        // one step of each chunk each and share the SIMDs with the four
        // integration waves: the Philox products and the Box-Muller
        // transcendentals run at a quarter of the vector rate and fill issue
        // slots the latency-bound integration leaves free.  With four waves,
        // waves 0 and 3 draw every second step.
        const bool eight = blockDim.x == 8 * 64;
        constexpr int ND8 = B >= 4 ? 4 : 2;
        const int ND = eight ? ND8 : 2;
        const int dslot = eight ? (wave >= 4 && wave - 4 < ND8 ? wave - 4 : -1)
                                : (wave == 3 ? 1 : (wave == 0 ? 0 : -1));
        if (dslot >= 0 && c < nch) {
            // noise, clipped inputs and the per-step thrust and torques
            const int kb = c * B, ke = min(N, kb + B);
            const int k_first = dslot;
            // a step's draw: the clipped inputs (u, V) of sample m at step k;
            // every lane draws (no branch around the arithmetic, so the steps
            // of a chunk interleave), the noise-free nominal and the idle
            // lanes past it with zero noise
            auto draw = [&](const int k, R4 &u, Real &V) {
                const R4 w4 = s_us[k];
                const Real us[4] = {w4.x, w4.y, w4.z, w4.w};
                const Normal4<Real> z = normals4<Real>((uint32_t)m, (uint32_t)k, h.s, 0u, a.seed_lo, a.seed_hi);
                const Real p0 = us[0] + sig0 * z.z0, p1 = us[1] + sig1 * z.z1;
                const Real p2 = us[2] + sig2 * z.z2, p3 = us[3] + sig3 * z.z3;
                u.x = clamp_finite(sampled ? p0 : us[0], tmin, tmax);
                u.y = clamp_finite(sampled ? p1 : us[1], tmin, tmax);
                u.z = clamp_finite(sampled ? p2 : us[2], tmin, tmax);
                u.w = clamp_finite(sampled ? p3 : us[3], tmin, tmax);
                V = Real(0);
                if (HAS_V) {
                    const Real vs = s_vs[k];
                    const Real zv = normal1<Real>((uint32_t)m, (uint32_t)k, h.s, 1u, a.seed_lo, a.seed_hi);
                    const Real pv = vs + sigv * zv;
                    V = clamp_finite(sampled ? pv : vs, Real(0), vmax);
                }
            };
            // store the samples, hand the inputs on
            auto put = [&](const int k, const int j, const R4 u, const Real V) {
                if (sampled && !a.regen) {
                    const size_t idx = (size_t)k * (size_t)K + (size_t)m;
                    store_nt(&ctrl[idx], u);
                    if (HAS_V) store_nt(&vctrl[idx], V);
                }
                if (HAS_V) s_v[c % 5][j][lane] = V;
                if (RATE) s_u[c % 5][j][lane] = u;
                const StepInput<Real> in = step_input(M, u.x, u.y, u.z, u.w);
                R4 o;
                o.x = in.fm; o.y = in.tx; o.z = in.ty; o.w = in.tz;
                s_in[c % 4][j][lane] = o;
            };
            if (ke - kb == B && !eight) {
                static_assert(B % 2 == 0, "each of two drawing waves takes B / 2 steps of a chunk");
                constexpr int NS = B / 2;
                R4 uu[NS];
                Real vv[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) draw(kb + k_first + 2 * i, uu[i], vv[i]);
#pragma unroll
                for (int i = 0; i < NS; ++i) put(kb + k_first + 2 * i, k_first + 2 * i, uu[i], vv[i]);
            } else if (ke - kb == B) {
                static_assert(B % ND8 == 0, "each drawing wave takes B / ND8 steps of a chunk");
                constexpr int NS = B / ND8;
                R4 uu[NS];
                Real vv[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) draw(kb + k_first + ND8 * i, uu[i], vv[i]);
#pragma unroll
                for (int i = 0; i < NS; ++i) put(kb + k_first + ND8 * i, k_first + ND8 * i, uu[i], vv[i]);
            } else {
                for (int k = kb + k_first; k < ke; k += ND) {
                    R4 u1;
                    Real v1;
                    draw(k, u1, v1);
                    put(k, k - kb, u1, v1);
                }
            }
        }
        if (wave == 0 && c >= 1 && c <= nch) {
            // body rates over chunk c - 1
            const int kb = (c - 1) * B, ke = min(N, kb + B);
            auto omega_step = [&](const int k, const int j, const R4 in) {
                R4 (*slot)[64] = s_w[(c - 1) & 1][j];
                Real term = Real(0);
                if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = w[i] - xr[10 + i];
                        term += (Real)a.Q[10 + i] * e * e;
                    }
                }
                if (OBJ == OBJ_CONTOUR)
                    term += (Real)a.Q_w[0] * w[0] * w[0] + (Real)a.Q_w[1] * w[1] * w[1] +
                            (Real)a.Q_w[2] * w[2] * w[2];
                Real ws[3], kw[3], dw[3];
                R4 stv[4];   // stage body rates, stored once the step is done
#pragma unroll
                for (int i = 0; i < 3; ++i) ws[i] = w[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    stv[st].x = ws[0]; stv[st].y = ws[1]; stv[st].z = ws[2];
                    kw[0] = in.y - M.gx * ws[1] * ws[2];
                    kw[1] = in.z - M.gy * ws[2] * ws[0];
                    kw[2] = in.w - M.gz * ws[0] * ws[1];
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] = kw[i];
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] += Real(2) * kw[i];
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) dw[i] = dt6 * (dw[i] + kw[i]);
                    }
                    if (st < 3) {
                        const Real hh = st < 2 ? h2 : dt;
#pragma unroll
                        for (int i = 0; i < 3; ++i) ws[i] = w[i] + hh * kw[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) w[i] += dw[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    stv[st].w = Real(0);
                    slot[st][lane] = stv[st];
                }
                if (OBJ != OBJ_GATE) J.add(term);
                // rate limit on the body rates after the step (here rather than
                // on the attitude wave, whose recurrence sets the pipeline's pace)
                Real rl = Real(0);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const Real e = fmax(fabs(w[i]) - w_max, Real(0));
                    rl += w_lim * e * e;
                }
                J.add(rl);
            };
            // the chunk's LDS inputs are loaded before the first step uses them
            if (ke - kb == B) {
                R4 inp[B];
#pragma unroll
                for (int j = 0; j < B; ++j) inp[j] = s_in[(c - 1) % 4][j][lane];
#pragma unroll
                for (int j = 0; j < B; ++j) omega_step(kb + j, j, inp[j]);
            } else {
                for (int k = kb; k < ke; ++k) omega_step(k, k - kb, s_in[(c - 1) % 4][k - kb][lane]);
            }
        } else if (wave == 1 && c >= 2 && c <= nch + 1) {
            // attitude over chunk c - 2
            const int kb = (c - 2) * B, ke = min(N, kb + B);
            auto quat_step = [&](const int k, const int j, const R4 *wst) {
                R4 (*slot)[64] = s_q[(c - 2) & 1][j];
                if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
                    Real term = Real(0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const Real e = q[i] - xr[6 + i];
                        term += (Real)a.Q[6 + i] * e * e;
                    }
                    J.add(term);
                }
                Real qs[4], kq[4], dq[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) qs[i] = q[i];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const R4 ws = wst[st];
                    R4 o;
                    o.x = qs[0]; o.y = qs[1]; o.z = qs[2]; o.w = qs[3];
                    slot[st][lane] = o;
                    // kq is twice the quaternion rate; the factor 1/2 is
                    // carried by the step sizes (exact: a power of two)
                    kq[0] = -qs[1] * ws.x - qs[2] * ws.y - qs[3] * ws.z;
                    kq[1] = qs[0] * ws.x + qs[2] * ws.z - qs[3] * ws.y;
                    kq[2] = qs[0] * ws.y - qs[1] * ws.z + qs[3] * ws.x;
                    kq[3] = qs[0] * ws.z + qs[1] * ws.y - qs[2] * ws.x;
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = kq[i];
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] += Real(2) * kq[i];
                    } else {
                        // the last stage closes the step in one multiply-add
                        // per component (this wave's recurrence sets the pace)
#pragma unroll
                        for (int i = 0; i < 4; ++i) q[i] = q[i] + dt12 * (dq[i] + kq[i]);
                    }
                    if (st < 3) {
                        const Real hq = st < 2 ? h4 : h2;
#pragma unroll
                        for (int i = 0; i < 4; ++i) qs[i] = q[i] + hq * kq[i];
                    }
                }
                renormalize(q);
            };
            if (ke - kb == B) {
                R4 wpre[B][4];
#pragma unroll
                for (int j = 0; j < B; ++j)
#pragma unroll
                    for (int st = 0; st < 4; ++st) wpre[j][st] = s_w[(c - 2) & 1][j][st][lane];
#pragma unroll
                for (int j = 0; j < B; ++j) quat_step(kb + j, j, wpre[j]);
            } else {
                for (int k = kb; k < ke; ++k) {
                    R4 wst[4];
#pragma unroll
                    for (int st = 0; st < 4; ++st) wst[st] = s_w[(c - 2) & 1][k - kb][st][lane];
                    quat_step(k, k - kb, wst);
                }
            }
        } else if (wave == 2 && c >= 3 && c <= nch + 2) {
            // position and velocity over chunk c - 3
            const int kb = (c - 3) * B, ke = min(N, kb + B);
            // drag is a launch constant: the branch sits outside the step, so the
            // stages of a step (independent without drag) schedule together
            auto trans_step = [&](const int k, const int j, const Real fm, const R4 *qstage, auto drag_tag) {
                constexpr bool DRAG = decltype(drag_tag)::value;
                if (OBJ == OBJ_TRACK) {
                    int r = i0 + k;
                    if (r > a.R - 1) r = a.R - 1;
                    const Real *xr = xref + 16 * r;
                    Real term = Real(0);
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = p[i] - xr[i];
                        term += (Real)a.Q[i] * e * e;
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const Real e = v[i] - xr[3 + i];
                        term += (Real)a.Q[3 + i] * e * e;
                    }
                    J.add(term);
                }
                Real vs[3], kv[3], dpv[3], dvv[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) vs[i] = v[i];
                // F/m times the thrust direction; the factor 2 of its first
                // two components rides on F/m (exact: a power of two)
                const Real fm2 = Real(2) * fm;
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const R4 qq = qstage[st];
                    const Real r3x = Real(2) * (qq.y * qq.w + qq.x * qq.z);
                    const Real r3y = Real(2) * (qq.z * qq.w - qq.x * qq.y);
                    const Real r3z = Real(1) - Real(2) * (qq.y * qq.y + qq.z * qq.z);
                    kv[0] = fm2 * (qq.y * qq.w + qq.x * qq.z);
                    kv[1] = fm2 * (qq.z * qq.w - qq.x * qq.y);
                    kv[2] = fm * r3z - M.g;
                    if (DRAG) {
                        const Real qw = qq.x, qx = qq.y, qy = qq.z, qz = qq.w;
                        const Real r11 = Real(1) - Real(2) * (qy * qy + qz * qz), r12 = Real(2) * (qx * qy - qw * qz);
                        const Real r21 = Real(2) * (qx * qy + qw * qz), r22 = Real(1) - Real(2) * (qx * qx + qz * qz);
                        const Real r31 = Real(2) * (qx * qz - qw * qy), r32 = Real(2) * (qy * qz + qw * qx);
                        const Real b0 = M.d0 * (r11 * vs[0] + r21 * vs[1] + r31 * vs[2]);
                        const Real b1 = M.d1 * (r12 * vs[0] + r22 * vs[1] + r32 * vs[2]);
                        const Real b2 = M.d2 * (r3x * vs[0] + r3y * vs[1] + r3z * vs[2]);
                        kv[0] -= r11 * b0 + r12 * b1 + r3x * b2;
                        kv[1] -= r21 * b0 + r22 * b1 + r3y * b2;
                        kv[2] -= r31 * b0 + r32 * b1 + r3z * b2;
                    }
                    if (st == 0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] = vs[i]; dvv[i] = kv[i]; }
                    } else if (st < 3) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] += Real(2) * vs[i]; dvv[i] += Real(2) * kv[i]; }
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) { dpv[i] = dt6 * (dpv[i] + vs[i]); dvv[i] = dt6 * (dvv[i] + kv[i]); }
                    }
                    if (st < 3) {
                        const Real hh = st < 2 ? h2 : dt;
#pragma unroll
                        for (int i = 0; i < 3; ++i) vs[i] = v[i] + hh * kv[i];
                    }
                }
                if (POS) {
                    R4 (*ps)[64] = s_p[(c - 3) & 1][j];
                    R4 o;
                    o.x = p[0]; o.y = p[1]; o.z = p[2]; o.w = Real(0);
                    ps[0][lane] = o;
                    o.x = dpv[0]; o.y = dpv[1]; o.z = dpv[2];
                    ps[1][lane] = o;
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    p[i] += dpv[i];
                    v[i] += dvv[i];
                }
            };
            if (ke - kb == B) {
                Real fpre[B];
                R4 qpre[B][4];
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    fpre[j] = s_in[(c - 3) % 4][j][lane].x;
#pragma unroll
                    for (int st = 0; st < 4; ++st) qpre[j][st] = s_q[(c - 3) & 1][j][st][lane];
                }
                if (M.drag) {
#pragma unroll
                    for (int j = 0; j < B; ++j) trans_step(kb + j, j, fpre[j], qpre[j], std::true_type{});
                } else {
#pragma unroll
                    for (int j = 0; j < B; ++j) trans_step(kb + j, j, fpre[j], qpre[j], std::false_type{});
                }
            } else {
                for (int k = kb; k < ke; ++k) {
                    R4 qst[4];
#pragma unroll
                    for (int st = 0; st < 4; ++st) qst[st] = s_q[(c - 3) & 1][k - kb][st][lane];
                    if (M.drag) trans_step(k, k - kb, s_in[(c - 3) % 4][k - kb][lane].x, qst, std::true_type{});
                    else trans_step(k, k - kb, s_in[(c - 3) % 4][k - kb][lane].x, qst, std::false_type{});
                }
            }
            if (POS && c == nch + 2) {
                R4 o;
                o.x = p[0]; o.y = p[1]; o.z = p[2]; o.w = Real(0);
                s_pN[lane] = o;
            }
        }
        if (wave == 3 && c >= 4) {
            // position costs and input-rate terms of chunk c - 4
            const int kb = (c - 4) * B, ke = min(N, kb + B);
            auto cost_step = [&](const int k, const int j, const R4 *pr) {
                Real term = Real(0);
                if (RATE) {
                    const R4 u = s_u[(c - 4) % 5][j][lane];
                    const Real d0 = u.x - up[0], d1 = u.y - up[1], d2 = u.z - up[2], d3 = u.w - up[3];
                    term += rdt[0] * d0 * d0 + rdt[1] * d1 * d1 + rdt[2] * d2 * d2 + rdt[3] * d3 * d3;
                    up[0] = u.x; up[1] = u.y; up[2] = u.z; up[3] = u.w;
                }
                if (HAS_V) {
                    const Real V = s_v[(c - 4) % 5][j][lane];
                    const Real dv = V - vp;
                    term += r_dv * dv * dv;
                    term -= (Real)a.mu * V;
                    vp = V;
                }
                if (POS) {
                    const R4 ph = pr[0];
                    const Real pk[3] = {ph.x, ph.y, ph.z};
                    if (OBJ == OBJ_GATE) {
                        const R4 dp4 = pr[1];
                        const Real dpv[3] = {dp4.x, dp4.y, dp4.z};
                        const Real ax = pk[0] - gt.cx;
                        const Real ay = pk[1] - gt.cy;
                        const Real az = pk[2] - gt.cz;
                        const Real bx = pk[0] - g0r.cx;
                        const Real by = pk[1] - g0r.cy;
                        const Real bz = pk[2] - g0r.cz;
                        const Real d2 = bx * bx + by * by + bz * bz;
                        if (d2 < r_near2) term += q_near * d2;
                        if (nominal) s_f8[k] = (bx * g0r.nx + by * g0r.ny) < Real(0);
                        term += dpv[0] * (Real(2) * ax + dpv[0]) + dpv[1] * (Real(2) * ay + dpv[1]) +
                                dpv[2] * (Real(2) * az + dpv[2]);
                        const Real sa = ax * gt.nx + ay * gt.ny;
                        const Real sb = (ax + dpv[0]) * gt.nx + (ay + dpv[1]) * gt.ny;
                        if (sa < Real(0) && sb >= Real(0)) {
                            const Real t = sa / (sa - sb);
                            const Real yx = ax + t * dpv[0], yy = ay + t * dpv[1], yz = az + t * dpv[2];
                            const Real lat = yx * gt.hx + yy * gt.hy;
                            const bool inside = fabs(lat) <= half && fabs(yz) <= half;
                            const int jj = k + 1;
                            const bool allowed = passes > 0 || ((h.allow[jj >> 5] >> (jj & 31)) & 1u);
                            if (inside && allowed) {
                                g = (g + 1 == a.G) ? 0 : g + 1;
                                ++passes;
                                gt.load(s_gtab, g);
                            }
                        }
                    } else {
                        const Real fl = floor(th_hi * inv_ds);
                        const Real f = ((th_hi - fl * ds) + th_lo) * inv_ds;
                        const int i = (fl >= Real(0) && fl < Real(1 << 30)) ? ((int)fl % a.P) : 0;
                        const int i1 = (i + 1 == a.P) ? 0 : i + 1;
                        const Real *A = path + 8 * i, *Bp = path + 8 * i1;
                        const Real g1 = Real(1) - f;
                        const Real px = g1 * A[0] + f * Bp[0], py = g1 * A[1] + f * Bp[1], pz = g1 * A[2] + f * Bp[2];
                        Real tx = g1 * A[3] + f * Bp[3], ty = g1 * A[4] + f * Bp[4], tz = g1 * A[5] + f * Bp[5];
                        const Real tn = inv_sqrt(tx * tx + ty * ty + tz * tz);
                        tx *= tn; ty *= tn; tz *= tn;
                        const Real ex = pk[0] - px;
                        const Real ey = pk[1] - py;
                        const Real ez = pk[2] - pz;
                        const Real et = ex * tx + ey * ty + ez * tz;
                        const Real lx = et * tx, ly = et * ty, lz = et * tz;
                        const Real cxe = ex - lx, cye = ey - ly, cze = ez - lz;
                        term += (Real)a.q_l * (lx * lx + ly * ly + lz * lz);
                        term += (Real)a.q_c * (cxe * cxe + cye * cye + cze * cze);
                        const Real vk = s_v[(c - 4) % 5][j][lane];
                        const Real y = vk * dt + th_lo;
                        const Real t = th_hi + y;
                        th_lo = (sizeof(Real) == 4) ? y - (t - th_hi) : Real(0);
                        th_hi = t;
                        if (th_hi >= L) th_hi -= L;
                    }
                }
                J.add(term);
            };
            if (ke - kb == B) {
                R4 ppre[B][2];
#pragma unroll
                for (int j = 0; j < B; ++j)
#pragma unroll
                    for (int i = 0; i < 2; ++i) ppre[j][i] = POS ? s_p[(c - 4) & 1][j][i][lane] : R4{};
#pragma unroll
                for (int j = 0; j < B; ++j) cost_step(kb + j, j, ppre[j]);
            } else {
                for (int k = kb; k < ke; ++k) {
                    R4 pr[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) pr[i] = POS ? s_p[(c - 4) & 1][k - kb][i][lane] : R4{};
                    cost_step(k, k - kb, pr);
                }
            }
        }
        __syncthreads();
    }

    // terminal tracking terms, on the wave that holds each part of x_N
    if (OBJ == OBJ_TRACK && wave < 3) {
        int r = i0 + N;
        if (r > a.R - 1) r = a.R - 1;
        const Real *xr = xref + 16 * r;
        Real term = 0;
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const Real e = w[i] - xr[10 + i];
                term += (Real)a.QN[10 + i] * e * e;
            }
        } else if (wave == 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const Real e = q[i] - xr[6 + i];
                term += (Real)a.QN[6 + i] * e * e;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const Real e = p[i] - xr[i];
                term += (Real)a.QN[i] * e * e;
                const Real f = v[i] - xr[3 + i];
                term += (Real)a.QN[3 + i] * f * f;
            }
        }
        J.add(term);
    }
    if (wave < 3) s_jp[wave][lane] = J.value();
    __syncthreads();
    if (wave == 3) {
        Real Jfinal = Real(0);
        if (active) {
            Jfinal = ((s_jp[0][lane] + s_jp[1][lane]) + s_jp[2][lane]) + J.value();
            if (OBJ == OBJ_GATE && nominal) {
                const R4 ph = s_pN[lane];
                const Real bx = ph.x - g0r.cx;
                const Real by = ph.y - g0r.cy;
                a.front8[N] = (bx * g0r.nx + by * g0r.ny) < Real(0);
            }
            if (nominal) a.cur->J_nom = (double)Jfinal;
            else ((Real *)a.J)[m] = Jfinal;
        }
        // the tile of the nominal writes its front flags of steps 0..N-1
        if (OBJ == OBJ_GATE && blk == (K >> 6))
            for (int i = lane; i < N; i += 64) a.front8[i] = s_f8[i];
        store_tile_min(Jfinal, active && !nominal && isfinite(Jfinal), a.tmin, blk);
    }
    __syncthreads();
}

template <int OBJ, typename Real, int B> __global__ __launch_bounds__(512) void k_rollout4(KArgs a)
{
    __shared__ HeadVals h;
    compute_head<OBJ == OBJ_CONTOUR>(a, h);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_head(a, h);
    rollout4_body<OBJ, Real, B>(a, blockIdx.x, h);
}

template <int OBJ, typename Real> __global__ __launch_bounds__(192) void k_rollout3(KArgs a)
{
    __shared__ HeadVals h;
    compute_head<OBJ == OBJ_CONTOUR>(a, h);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_head(a, h);
    rollout3_body<OBJ, Real>(a, blockIdx.x, h);
}

// ---------------------------------------------------------------- control cost

// The control-cost term of information-theoretic MPPI added to every sample's
// cost: gamma * sum_k sum_i U*_k,i (U^m_k,i - U*_k,i) / sigma_i^2 over the
// channels with sigma_i > 0 (thrusts, then the contouring speed), U* the
// shifted warm start of the solve and U^m the stored clipped sample, summed in
// step order.  One wave per 64-sample tile reads its samples step by step
// (64 consecutive records per step) and rewrites the tile's smallest finite
// cost.
template <typename Real, bool HAS_V> __device__ __forceinline__ void ctrl_cost_body(const KArgs &a, int tile)
{
    typedef typename Vec4<Real>::T R4;
    const int m = tile * 64 + (int)threadIdx.x;
    const int K = a.K, N = a.N;
    const DevCur *cur = a.cur;
    const int shift = cur->shift;
    const bool warm = cur->warm != 0;
    const Real gam = (Real)a.ctrl_cost, hover = (Real)a.hover;
    const Real is0 = (Real)a.inv_sig2[0], is1 = (Real)a.inv_sig2[1], is2 = (Real)a.inv_sig2[2];
    const Real is3 = (Real)a.inv_sig2[3], isv = (Real)a.inv_sig2[4];
    Real Jm = Real(INFINITY);
    if (m < K) {
        const R4 *ctrl = (const R4 *)a.ctrl;
        const Real *vctrl = (const Real *)a.vctrl;
        Real C = Real(0);
        for (int k = 0; k < N; ++k) {
            const int src = k + shift < N ? k + shift : N - 1;
            const Real u0 = warm ? (Real)a.wU[4 * src + 0] : hover, u1 = warm ? (Real)a.wU[4 * src + 1] : hover;
            const Real u2 = warm ? (Real)a.wU[4 * src + 2] : hover, u3 = warm ? (Real)a.wU[4 * src + 3] : hover;
            const R4 u = ctrl[(size_t)k * (size_t)K + (size_t)m];
            C += gam * u0 * (u.x - u0) * is0;
            C += gam * u1 * (u.y - u1) * is1;
            C += gam * u2 * (u.z - u2) * is2;
            C += gam * u3 * (u.w - u3) * is3;
            if (HAS_V) {
                const Real vs = warm ? (Real)a.wV[src] : Real(0);
                C += gam * vs * (vctrl[(size_t)k * (size_t)K + (size_t)m] - vs) * isv;
            }
        }
        Jm = ((Real *)a.J)[m] + C;
        ((Real *)a.J)[m] = Jm;
    }
    store_tile_min(Jm, m < K && isfinite(Jm), a.tmin, tile);
}

template <typename Real, bool HAS_V> __global__ __launch_bounds__(64) void k_ctrl_cost(KArgs a)
{
    ctrl_cost_body<Real, HAS_V>(a, blockIdx.x);
}

// ---------------------------------------------------------------- weighted average

// Sum over the 64 lanes of a wave (all lanes active) by a fixed tree,
// returned to every lane: binary32 through the DPP moves of wave_min (a lane
// without a source adds 0; lane 63 ends with the sum), binary64 through lane
// shuffles.
template <int CTRL, int ROW_MASK = 0xf> __device__ __forceinline__ float dpp_or_zero(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_or_zero<0xb1>(v);
    v += dpp_or_zero<0x4e>(v);
    v += dpp_or_zero<0x114>(v);
    v += dpp_or_zero<0x118>(v);
    v += dpp_or_zero<0x142, 0xa>(v);
    v += dpp_or_zero<0x143, 0xc>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Eq. (4)-(5) for step k in one block of kFinalThreads threads:
//   J_min = min over the tile minima (each wave reduces them all),  w~_m = exp(-(J_m - J_min)/lambda)
//   (0 for non-finite J_m),  S = sum_m w~_m,  U_k = sum_m w~_m U^m_k / S.
// Thread t adds the samples t, t + kFinalThreads, ... in that order.  The
// thread sums go to LDS; lane l of wave i then adds value i of threads l,
// l + 64, ..., l + kFinalThreads - 64 in that order and the lanes are added
// by the fixed tree of wave_sum, one value per wave, all values at once.  S
// and sum_m w~_m^2 come out of the same loop in every block, bit for bit, so
// no block waits for another.  The block of step 0 also writes the first
// input, the report, the nominal's pass mask for the next solve and the
// warm-start hand-over.  The samples are loaded first, then the tile minima,
// so that one wait covers all of them.
//
// REGEN: the samples are not read from the sample tensor (which the rollout
// then does not write) but drawn again from the counter-based noise of this
// solve and the shifted warm start of step k that the rollout left in nomU /
// nomV, with the same operations as the rollout's draw, so the weighted sums
// are the same bit for bit: Philox and Box-Muller arithmetic in place of
// 16 B (20 B contouring) of HBM traffic per sample and step.
template <typename Real, typename Acc, bool HAS_V, bool REGEN, int UR = 4>
__device__ __forceinline__ void final_body(const KArgs &a, int k)
{
    constexpr int C = HAS_V ? 5 : 4;
    constexpr int NV = C + 2;
    constexpr int NT = kFinalThreads, NWV = NT / 64;
    typedef typename Vec4<Real>::T R4;
    static_assert(NV <= NWV, "one wave per reduced value");
    __shared__ Acc s_part[NV][NT];
    __shared__ Acc s_tot[NV];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int K = a.K, N = a.N;
    const Real *J = (const Real *)a.J;
    const R4 *ctrl = (const R4 *)a.ctrl + (size_t)k * (size_t)K;
    const Real *vctrl = HAS_V ? (const Real *)a.vctrl + (size_t)k * (size_t)K : nullptr;
    const Real inv_lambda = (Real)(1.0 / a.lambda);
    DevCur *cur = a.cur;
    DevWarm *w = a.warm;
    const bool head = k == 0;
    const bool gate = a.objective == OBJ_GATE;
    // regenerated draws: the shifted warm start of step k and the noise key
    R4 us{};
    Real vs = Real(0);
    uint32_t s_solve = 0;
    if (REGEN) {
        us = ((const R4 *)a.nomU)[k];
        if (HAS_V) vs = ((const Real *)a.nomV)[k];
        s_solve = cur->s;
    }
    const Real tmin = (Real)a.t_min, tmax = (Real)a.t_max, vmax = (Real)a.v_max;
    const Real sig0 = (Real)a.sigma[0], sig1 = (Real)a.sigma[1], sig2 = (Real)a.sigma[2], sig3 = (Real)a.sigma[3];
    const Real sigv = (Real)a.sigma_v;
    auto redraw = [&](const int m, R4 &u, Real &V) {
        const Normal4<Real> z = normals4<Real>((uint32_t)m, (uint32_t)k, s_solve, 0u, a.seed_lo, a.seed_hi);
        u.x = clamp_finite(us.x + sig0 * z.z0, tmin, tmax);
        u.y = clamp_finite(us.y + sig1 * z.z1, tmin, tmax);
        u.z = clamp_finite(us.z + sig2 * z.z2, tmin, tmax);
        u.w = clamp_finite(us.w + sig3 * z.z3, tmin, tmax);
        if (HAS_V) {
            const Real zv = normal1<Real>((uint32_t)m, (uint32_t)k, s_solve, 1u, a.seed_lo, a.seed_hi);
            V = clamp_finite(vs + sigv * zv, Real(0), vmax);
        }
    };

    // loads: the first UR samples of this thread, then the tile minima (every
    // wave reads all of them), four per lane before the first comparison, so
    // that one round trip to memory covers all of them
    Real Jm[UR], vm[UR];
    R4 u[UR];
#pragma unroll
    for (int i = 0; i < UR; ++i) {
        const int m = tid + NT * i;
        if (m < K) {
            Jm[i] = J[m];
            if (!REGEN) {
                u[i] = ctrl[m];
                if (HAS_V) vm[i] = vctrl[m];
            }
        }
    }
    Real mn = Real(INFINITY);
    for (int t0 = lane; t0 < a.n_tiles; t0 += 4 * 64) {
        Real tv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = t0 + 64 * j;
            tv[j] = t < a.n_tiles ? ((const Real *)a.tmin)[t] : Real(INFINITY);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) mn = tv[j] < mn ? tv[j] : mn;
    }
    // head values for the report and the hand-over (block of step 0)
    const bool fr = head && gate && tid <= N && tid < 256 && a.front8[tid] != 0;
    const bool fr_last = head && gate && tid == 0 && N >= 256 && a.front8[256] != 0;
    // (spread over the lanes of wave 0: lane 5 the report's head fields,
    // lane 6 the warm-start fields, lanes 7..19 one state component each)
    double rep_Jnom = 0.0, rep_theta0 = 0.0, rep_t = 0.0, rep_x = 0.0, rep_v = 0.0;
    int32_t rep_g0 = 0, rep_i0 = 0, rep_shift = 0;
    uint32_t rep_s = 0;
    if (head && (tid == 5 || tid == 6)) {
        rep_Jnom = cur->J_nom;
        rep_theta0 = cur->theta0;
        rep_t = cur->t_now;
        rep_g0 = cur->g0;
        rep_i0 = cur->i0;
        rep_shift = cur->shift;
        rep_s = cur->s;
        rep_v = cur->v_prev;
    }
    if (head && tid >= 7 && tid < 20) rep_x = cur->x0[tid - 7];
    // J_min within each wave (a minimum does not depend on the grouping, so
    // every wave of every block finds the same value without a block barrier)
    const Real jmin = wave_min(mn);

    // weighted sums, UR samples per round in sample order; the next round's
    // loads are issued before this round's arithmetic
    Acc v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = Acc(0);
    for (int m0 = tid; m0 < K; m0 += NT * UR) {
        Real Jn[UR], vn[UR];
        R4 un[UR];
        const int m1 = m0 + NT * UR;
        if (m1 < K) {
#pragma unroll
            for (int i = 0; i < UR; ++i) {
                const int m = m1 + NT * i;
                if (m < K) {
                    Jn[i] = J[m];
                    if (!REGEN) {
                        un[i] = ctrl[m];
                        if (HAS_V) vn[i] = vctrl[m];
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < UR; ++i) {
            if (m0 + NT * i < K) {
                if (REGEN) redraw(m0 + NT * i, u[i], vm[i]);
                const Real wr = isfinite(Jm[i]) ? exp(-(Jm[i] - jmin) * inv_lambda) : Real(0);
                const Acc wa = (Acc)wr;
                v[0] += wa * (Acc)u[i].x;
                v[1] += wa * (Acc)u[i].y;
                v[2] += wa * (Acc)u[i].z;
                v[3] += wa * (Acc)u[i].w;
                if (HAS_V) v[4] += wa * (Acc)vm[i];
                v[C] += wa;
                v[C + 1] += wa * wa;
            }
        }
        if (m1 < K) {
#pragma unroll
            for (int i = 0; i < UR; ++i) {
                Jm[i] = Jn[i];
                if (!REGEN) {
                    u[i] = un[i];
                    if (HAS_V) vm[i] = vn[i];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) s_part[i][tid] = v[i];
    __syncthreads();
    if (wv < NV) {
        Acc t = s_part[wv][lane];
#pragma unroll
        for (int j = 1; j < NWV; ++j) t += s_part[wv][64 * j + lane];
        t = wave_sum(t);
        if (lane == 0) s_tot[wv] = t;
    }
    __syncthreads();
    const Acc den = s_tot[C], den2 = s_tot[C + 1];
    const bool ok = isfinite(jmin) && den > Acc(0);
    if (ok && tid < C) {
        const double uk = (double)(s_tot[tid] / den);
        if (tid < 4) a.wU[4 * k + tid] = uk;
        else a.wV[k] = uk;
    }
    if (!HAS_V && ok && tid == 0) a.wV[k] = 0.0;
    if (!head) return;

    // pass mask of the next solve: bit j = front flag of the nominal at step j
    if (gate) {
        if (tid < 256) {
            const unsigned long long bal = __ballot(fr);
            if ((tid & 63) == 0 && ok) {
                w->allow[tid >> 5] = (uint32_t)bal;
                w->allow[(tid >> 5) + 1] = (uint32_t)(bal >> 32);
            }
        }
        if (tid == 0 && ok) w->allow[8] = fr_last ? 1u : 0u;
    } else if (tid < kMaskWords && ok) {
        w->allow[tid] = 0xffffffffu;
    }
    // the report and the warm-start hand-over, one group of fields per lane
    DevResult *r = a.res;
    if (tid < 4) {
        const double u0 = ok ? (double)(s_tot[tid] / den) : (double)NAN;
        r->u0[tid] = u0;
        if (a.u0_out) a.u0_out[tid] = u0;
    } else if (tid == 4) {
        r->J_min = (double)jmin;
        r->S = (double)den;
        r->S2 = (double)den2;
        r->ess = ok ? (double)den * (double)den / (double)den2 : 0.0;
    } else if (tid == 5) {
        r->J_nom = rep_Jnom;
        r->theta0 = rep_theta0;
        r->status = ok ? ST_OK : ST_NONFINITE;
        r->g0 = rep_g0;
        r->i0 = rep_i0;
        r->shift = rep_shift;
        r->s = rep_s;
    } else if (tid == 6 && ok) {
        w->warm = 1;
        w->g0 = rep_g0;
        w->s = rep_s + 1u;
        w->N = N;
        w->t_prev = rep_t;
        w->theta0 = rep_theta0;
        // rate model: the progress speed state of this solve
        w->vtheta = a.input_model == INPUT_RATE ? rep_v : 0.0;
    } else if (tid >= 7 && tid < 20 && ok) {
        w->x_prev[tid - 7] = rep_x;
    }
}

template <typename Real, typename Acc, bool HAS_V, bool REGEN, int UR>
__global__ __launch_bounds__(kFinalThreads) void k_final(KArgs a)
{
    final_body<Real, Acc, HAS_V, REGEN, UR>(a, blockIdx.x);
}

// ---------------------------------------------------------------- batched (persistent)

// The item of unit u: the largest i in [0, n) with prefix[i] <= u (prefix[0]
// = 0, prefix[n] = total).  Every persistent kernel takes its units in
// increasing order, so the item only moves forward from the block's previous
// one: usually one load per unit instead of a binary search.
__device__ __forceinline__ int advance_item(const int32_t *prefix, int n, int u, int item)
{
    while (item + 1 < n && prefix[item + 1] <= u) ++item;
    return item;
}

// Stage the kernel arguments of an item's context in LDS, with the item's
// request and output pointers.
__device__ __forceinline__ void stage_args(KArgs &s_a, int &s_ctx, const BArgs &b, int item)
{
    const BatchItem it = b.items[item];
    if (it.ctx != s_ctx) {
        const uint32_t *src = (const uint32_t *)(b.table + it.ctx);
        uint32_t *dst = (uint32_t *)&s_a;
        for (int t = threadIdx.x; t < (int)(sizeof(KArgs) / 4); t += blockDim.x) dst[t] = src[t];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_a.req = it.req;
        s_a.u0_out = it.u0_out;
        if (it.ws) {
            const WsLayout l = ws_layout(s_a.K, s_a.N, s_a.C, s_a.real_bytes);
            s_a.ctrl = it.ws + l.ctrl;
            s_a.vctrl = s_a.C == 5 ? it.ws + l.vctrl : nullptr;
            s_a.nomU = it.ws + l.nomU;
            s_a.nomV = it.ws + l.nomV;
            s_a.J = it.ws + l.J;
            s_a.tmin = it.ws + l.tmin;
            s_a.front8 = (uint8_t *)(it.ws + l.front8);
        }
        // a workspace is bound per item: restage the next item in any case
        s_ctx = it.ws ? -1 : it.ctx;
    }
    __syncthreads();
}

// One unit per (item, block of 256 samples), all steps of the item; units
// are taken from a device queue in order (longest horizons first).
template <typename Real, bool HAS_V> __global__ __launch_bounds__(256) void kb_sample(BArgs b)
{
    __shared__ KArgs s_a;
    __shared__ int s_ctx, s_unit;
    if (threadIdx.x == 0) s_ctx = -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) b.desc->queue = 0u;
    const int n = b.desc->n, total = b.desc->n_sample_units;
    int item = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(&b.desc->sample_queue, 1u);
        __syncthreads();
        const int u = s_unit;
        if (u >= total) break;
        item = advance_item(b.sample_prefix, n, u, item);
        stage_args(s_a, s_ctx, b, item);
        sample_body<Real, HAS_V>(s_a, u - b.sample_prefix[item], 0, s_a.N);
    }
}

template <int OBJ, typename Real, int WAVES> __global__ __launch_bounds__(64 * WAVES) void kb_rollout(BArgs b)
{
    __shared__ KArgs s_a;
    __shared__ int s_ctx, s_unit;
    if (threadIdx.x == 0) s_ctx = -1;
    const int n = b.desc->n, total = b.desc->n_tiles;
    int item = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(&b.desc->queue, 1u);
        __syncthreads();
        const int u = s_unit;
        if (u >= total) break;
        item = advance_item(b.tile_prefix, n, u, item);
        stage_args(s_a, s_ctx, b, item);
        const int blk = u - b.tile_prefix[item];
        if (WAVES == 2) rollout2_body<OBJ, Real>(s_a, blk);
        else rollout1_body<OBJ, Real>(s_a, blk);
    }
}

template <int OBJ, typename Real> __global__ __launch_bounds__(192) void kb_rollout3(BArgs b)
{
    __shared__ KArgs s_a;
    __shared__ HeadVals h;
    __shared__ int s_ctx, s_unit;
    if (threadIdx.x == 0) s_ctx = -1;
    const int n = b.desc->n, total = b.desc->n_tiles;
    int item = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(&b.desc->queue, 1u);
        __syncthreads();
        const int u = s_unit;
        if (u >= total) break;
        item = advance_item(b.tile_prefix, n, u, item);
        stage_args(s_a, s_ctx, b, item);
        const int blk = u - b.tile_prefix[item];
        compute_head<OBJ == OBJ_CONTOUR>(s_a, h);
        if (blk == 0 && threadIdx.x == 0) publish_head(s_a, h);
        rollout3_body<OBJ, Real>(s_a, blk, h);
    }
}

template <int OBJ, typename Real, int B> __global__ __launch_bounds__(256) void kb_rollout4(BArgs b)
{
    __shared__ KArgs s_a;
    __shared__ HeadVals h;
    __shared__ int s_ctx, s_unit;
    if (threadIdx.x == 0) s_ctx = -1;
    const int n = b.desc->n, total = b.desc->n_tiles;
    int item = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(&b.desc->queue, 1u);
        __syncthreads();
        const int u = s_unit;
        if (u >= total) break;
        item = advance_item(b.tile_prefix, n, u, item);
        stage_args(s_a, s_ctx, b, item);
        const int blk = u - b.tile_prefix[item];
        compute_head<OBJ == OBJ_CONTOUR>(s_a, h);
        if (blk == 0 && threadIdx.x == 0) publish_head(s_a, h);
        rollout4_body<OBJ, Real, B>(s_a, blk, h);
    }
}

// One unit per (item, 64-sample tile) of the control-cost term; items
// without the term are skipped.
template <typename Real, bool HAS_V> __global__ __launch_bounds__(64) void kb_ctrl_cost(BArgs b)
{
    __shared__ KArgs s_a;
    __shared__ int s_ctx;
    if (threadIdx.x == 0) s_ctx = -1;
    __syncthreads();
    const int n = b.desc->n, total = b.desc->n_tiles;
    int item = 0;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        item = advance_item(b.tile_prefix, n, u, item);
        stage_args(s_a, s_ctx, b, item);
        if (s_a.ctrl_cost != 0.0) ctrl_cost_body<Real, HAS_V>(s_a, u - b.tile_prefix[item]);
        __syncthreads();
    }
}

// One unit per (item, step) of the weighted average.  The sample and rollout
// kernels of this step have finished, so their work queues are reset here
// for the next iteration of the step.
template <typename Real, typename Acc, bool HAS_V> __global__ __launch_bounds__(kFinalThreads) void kb_final(BArgs b)
{
    __shared__ KArgs s_a;
    __shared__ int s_ctx;
    if (threadIdx.x == 0) s_ctx = -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.desc->queue = 0u;
        b.desc->sample_queue = 0u;
    }
    // every thread reads s_ctx in stage_args before its first barrier
    __syncthreads();
    const int n = b.desc->n, total = b.desc->n_steps;
    int item = 0;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        item = advance_item(b.step_prefix, n, u, item);
        stage_args(s_a, s_ctx, b, item);
        // a context whose rollout left no sample tensor: draw the samples again
        if (s_a.regen) final_body<Real, Acc, HAS_V, true>(s_a, u - b.step_prefix[item]);
        else final_body<Real, Acc, HAS_V, false>(s_a, u - b.step_prefix[item]);
        __syncthreads();
    }
}

template <typename Real, int OBJ>
static hipError_t launch_batch_t(const BArgs &b, const BatchLaunch &L, hipStream_t st)
{
    constexpr bool HAS_V = OBJ == OBJ_CONTOUR;
    if (L.rollout_waves < 3)
        hipLaunchKernelGGL((kb_sample<Real, HAS_V>), dim3(L.sample_groups), dim3(256), 0, st, b);
    if (L.rollout_waves == 4) {
        if constexpr (sizeof(Real) == 4) {
            if (L.ring4_b == 4)
                hipLaunchKernelGGL((kb_rollout4<OBJ, Real, 4>), dim3(L.rollout_groups), dim3(256), 0, st, b);
            else
                hipLaunchKernelGGL((kb_rollout4<OBJ, Real, 2>), dim3(L.rollout_groups), dim3(256), 0, st, b);
        } else {
            hipLaunchKernelGGL((kb_rollout4<OBJ, Real, 2>), dim3(L.rollout_groups), dim3(256), 0, st, b);
        }
    } else if (L.rollout_waves == 3)
        hipLaunchKernelGGL((kb_rollout3<OBJ, Real>), dim3(L.rollout_groups), dim3(192), 0, st, b);
    else if (L.rollout_waves == 2)
        hipLaunchKernelGGL((kb_rollout<OBJ, Real, 2>), dim3(L.rollout_groups), dim3(128), 0, st, b);
    else
        hipLaunchKernelGGL((kb_rollout<OBJ, Real, 1>), dim3(L.rollout_groups), dim3(64), 0, st, b);
    if (L.ctrl_groups > 0)
        hipLaunchKernelGGL((kb_ctrl_cost<Real, HAS_V>), dim3(L.ctrl_groups), dim3(64), 0, st, b);
    if (L.acc64 || sizeof(Real) == 8)
        hipLaunchKernelGGL((kb_final<Real, double, HAS_V>), dim3(L.final_groups), dim3(kFinalThreads), 0, st, b);
    else
        hipLaunchKernelGGL((kb_final<Real, float, HAS_V>), dim3(L.final_groups), dim3(kFinalThreads), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_batch(const BArgs &b, const BatchLaunch &L, hipStream_t st)
{
    if (L.fp64) {
        switch (L.objective) {
        case OBJ_CONTOUR: return launch_batch_t<double, OBJ_CONTOUR>(b, L, st);
        case OBJ_TRACK: return launch_batch_t<double, OBJ_TRACK>(b, L, st);
        default: return launch_batch_t<double, OBJ_GATE>(b, L, st);
        }
    }
    switch (L.objective) {
    case OBJ_CONTOUR: return launch_batch_t<float, OBJ_CONTOUR>(b, L, st);
    case OBJ_TRACK: return launch_batch_t<float, OBJ_TRACK>(b, L, st);
    default: return launch_batch_t<float, OBJ_GATE>(b, L, st);
    }
}

// ---------------------------------------------------------------- launches

template <typename Real> static hipError_t launch_setup_t(const KArgs &a, hipStream_t st)
{
    int n = a.G > a.P ? a.G : a.P;
    if (a.R > n) n = a.R;
    if (n < 1) n = 1;
    hipLaunchKernelGGL(k_setup<Real>, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_setup(const KArgs &a, bool fp64, hipStream_t st)
{
    return fp64 ? launch_setup_t<double>(a, st) : launch_setup_t<float>(a, st);
}

template <typename Real, typename Acc, bool HAS_V>
static hipError_t launch_average_t(const KArgs &a, hipStream_t st)
{
    // binary32: all of a thread's samples in one round of loads when they are
    // at most eight, else (and in binary64, whose registers hold half as
    // many) rounds of four with the next round's loads in flight; the
    // accumulation order, and so the result, is the same either way
    const bool one_round = sizeof(Real) == 4 && a.K <= 8 * kFinalThreads;
    if (a.regen) {
        if (one_round)
            hipLaunchKernelGGL((k_final<Real, Acc, HAS_V, true, 8>), dim3(a.N), dim3(kFinalThreads), 0, st, a);
        else
            hipLaunchKernelGGL((k_final<Real, Acc, HAS_V, true, 4>), dim3(a.N), dim3(kFinalThreads), 0, st, a);
    } else {
        if (one_round)
            hipLaunchKernelGGL((k_final<Real, Acc, HAS_V, false, 8>), dim3(a.N), dim3(kFinalThreads), 0, st, a);
        else
            hipLaunchKernelGGL((k_final<Real, Acc, HAS_V, false, 4>), dim3(a.N), dim3(kFinalThreads), 0, st, a);
    }
    return hipGetLastError();
}

template <typename Real, int OBJ>
static hipError_t launch_solve_t(const KArgs &a, bool acc64, hipStream_t st, hipEvent_t *ev)
{
    constexpr bool HAS_V = OBJ == OBJ_CONTOUR;
    const dim3 gs((a.K + 1 + 255) / 256, (a.N + kSampleSteps - 1) / kSampleSteps);
    if (ev) (void)hipEventRecord(ev[0], st);
    // a one-wave rollout that draws its samples (binary32) needs only the head first
    const bool draw = sizeof(Real) == 4 && a.rollout_draw;
    if (draw) {
        if constexpr (sizeof(Real) == 4) hipLaunchKernelGGL((k_head<Real, HAS_V>), dim3(1), dim3(256), 0, st, a);
    } else if (a.rollout_waves < 3) {
        hipLaunchKernelGGL((k_sample<Real, HAS_V>), gs, dim3(256), 0, st, a);
    }
    if (ev) (void)hipEventRecord(ev[1], st);
    const dim3 gt((a.K + 1 + 63) / 64);
    if (a.rollout_waves == 4) {
        if constexpr (sizeof(Real) == 4) {
            if (a.ring4_b == 4)
                hipLaunchKernelGGL((k_rollout4<OBJ, Real, 4>), gt, dim3(512), 0, st, a);
            else
                hipLaunchKernelGGL((k_rollout4<OBJ, Real, 2>), gt, dim3(256), 0, st, a);
        } else {
            hipLaunchKernelGGL((k_rollout4<OBJ, Real, 2>), gt, dim3(256), 0, st, a);
        }
    } else if (a.rollout_waves == 3) {
        hipLaunchKernelGGL((k_rollout3<OBJ, Real>), gt, dim3(192), 0, st, a);
    } else if (a.rollout_waves == 2) {
        hipLaunchKernelGGL((k_rollout_split<OBJ, Real>), gt, dim3(128), 0, st, a);
    } else if (draw) {
        if constexpr (sizeof(Real) == 4) hipLaunchKernelGGL((k_rollout<OBJ, Real, true>), gt, dim3(64), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_rollout<OBJ, Real, false>), gt, dim3(64), 0, st, a);
    }
    if (a.ctrl_cost != 0.0)
        hipLaunchKernelGGL((k_ctrl_cost<Real, HAS_V>), dim3(a.n_tiles), dim3(64), 0, st, a);
    if (ev) (void)hipEventRecord(ev[2], st);
    hipError_t e = (acc64 || sizeof(Real) == 8) ? launch_average_t<Real, double, HAS_V>(a, st)
                                                : launch_average_t<Real, float, HAS_V>(a, st);
    if (ev) (void)hipEventRecord(ev[3], st);
    return e;
}

hipError_t launch_solve(const KArgs &a, bool fp64, bool acc64, hipStream_t st, hipEvent_t *ev)
{
    if (fp64) {
        switch (a.objective) {
        case OBJ_CONTOUR: return launch_solve_t<double, OBJ_CONTOUR>(a, true, st, ev);
        case OBJ_TRACK: return launch_solve_t<double, OBJ_TRACK>(a, true, st, ev);
        default: return launch_solve_t<double, OBJ_GATE>(a, true, st, ev);
        }
    }
    switch (a.objective) {
    case OBJ_CONTOUR: return launch_solve_t<float, OBJ_CONTOUR>(a, acc64, st, ev);
    case OBJ_TRACK: return launch_solve_t<float, OBJ_TRACK>(a, acc64, st, ev);
    default: return launch_solve_t<float, OBJ_GATE>(a, acc64, st, ev);
    }
}

// ------------------------------------------------------- fixed workspace

// Workspace of the allocation-free solve: one array per GPU, held by the
// library's code object until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// it resolves the device address per device and passes that.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_lock;
void *g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t scratch_address(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace mppi
