// Host runtime behind the C ABI declared in include/mppi.h: argument
// validation, device memory of a context, the launch sequence of one solve,
// result transfer, warm-start export/import, and the host plant step.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/mppi.h"
#include "device.hpp"
#include "kernels.hpp"

using namespace mppi;

static_assert(MPPI_MASK_WORDS == kMaskWords, "mask width");
static_assert(MPPI_N_MAX == kNMax, "horizon bound");
static_assert(MPPI_REQ_DOUBLES == kReqDoubles, "request record");

struct mppi_ctx {
    mppi_params prm;
    mppi_quad quad;
    int K = 0, N = 0, G = 0, P = 0, R = 0, objective = 0, C = 4;
    bool fp64 = false, acc64 = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mppi_allocator alloc{};
    bool have_alloc = false;
    std::vector<void *> dev_blocks;
    KArgs args{};
    DevWarm *warm = nullptr;
    DevResult *res = nullptr;
    double *req = nullptr;      // device request record of mppi_solve
    double *h_req = nullptr;    // pinned staging
    DevResult *h_res = nullptr; // pinned staging
    double *h_U = nullptr;      // pinned staging, N x 4
    // per-kernel timing
    bool profiling = false;
    std::vector<hipEvent_t> events;  // kProfSlots x 4
    int prof_count = 0;
    std::string err;
};

static constexpr int kProfSlots = 4096;

// Events of the next solve when profiling, else null.
static hipEvent_t *next_events(mppi_ctx *c)
{
    if (!c->profiling || c->events.empty()) return nullptr;
    if (c->prof_count >= kProfSlots) return nullptr;
    return &c->events[4 * (size_t)(c->prof_count++)];
}

static thread_local std::string g_create_err;

static mppi_status fail(mppi_ctx *c, mppi_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
static mppi_status fail(mppi_ctx *c, mppi_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_err = buf;
    return s;
}

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), MPPI_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

static void *dev_alloc(mppi_ctx *c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->have_alloc) {
        p = c->alloc.alloc(bytes, c->alloc.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->dev_blocks.push_back(p);
    return p;
}

static void release(mppi_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *p : c->dev_blocks) {
        if (c->have_alloc) c->alloc.free(p, c->alloc.user);
        else (void)hipFree(p);
    }
    c->dev_blocks.clear();
    if (c->h_req) (void)hipHostFree(c->h_req);
    if (c->h_res) (void)hipHostFree(c->h_res);
    if (c->h_U) (void)hipHostFree(c->h_U);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    c->events.clear();
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

static bool finite_all(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

static mppi_status validate(const mppi_params *p, const mppi_quad *q, const mppi_problem *pb)
{
    if (!p || !q || !pb) return fail(nullptr, MPPI_E_INVAL, "params, quad and problem are required");
    if (p->K < 1 || p->K > MPPI_K_MAX) return fail(nullptr, MPPI_E_INVAL, "K=%d outside [1, %d]", p->K, MPPI_K_MAX);
    if (p->N < 1 || p->N > MPPI_N_MAX) return fail(nullptr, MPPI_E_INVAL, "N=%d outside [1, %d]", p->N, MPPI_N_MAX);
    if (p->objective < MPPI_OBJ_GATE || p->objective > MPPI_OBJ_TRACK)
        return fail(nullptr, MPPI_E_INVAL, "unknown objective %d", p->objective);
    if (p->precision != MPPI_FP32 && p->precision != MPPI_FP64)
        return fail(nullptr, MPPI_E_INVAL, "unknown precision %d", p->precision);
    if (!(p->dt > 0.0) || !isfinite(p->dt)) return fail(nullptr, MPPI_E_INVAL, "dt must be > 0");
    if (!(p->lambda > 0.0) || !isfinite(p->lambda)) return fail(nullptr, MPPI_E_INVAL, "lambda must be > 0");
    for (int i = 0; i < 4; ++i)
        if (!(p->sigma[i] >= 0.0) || !isfinite(p->sigma[i]))
            return fail(nullptr, MPPI_E_INVAL, "sigma[%d] must be finite and >= 0", i);
    if (!(p->sigma_v >= 0.0) || !isfinite(p->sigma_v)) return fail(nullptr, MPPI_E_INVAL, "sigma_v must be >= 0");
    const double sc[] = {p->w_lim, p->q_near, p->r_near, p->q_l, p->q_c, p->r_dv, p->mu, p->v_max};
    if (!finite_all(sc, 8) || !finite_all(p->Q, 13) || !finite_all(p->QN, 13) || !finite_all(p->R_dT, 4) ||
        !finite_all(p->Q_w, 3))
        return fail(nullptr, MPPI_E_INVAL, "cost weights must be finite");
    if (!(q->mass > 0.0) || !isfinite(q->mass)) return fail(nullptr, MPPI_E_INVAL, "mass must be > 0");
    for (int i = 0; i < 3; ++i)
        if (!(q->inertia[i] > 0.0) || !isfinite(q->inertia[i]))
            return fail(nullptr, MPPI_E_INVAL, "inertia[%d] must be > 0", i);
    const double qs[] = {q->arm, q->c_tau, q->gravity, q->t_min, q->t_max, q->w_max};
    if (!finite_all(qs, 6) || !finite_all(q->drag, 3)) return fail(nullptr, MPPI_E_INVAL, "quad fields must be finite");
    if (!(q->t_max >= q->t_min)) return fail(nullptr, MPPI_E_INVAL, "t_max < t_min");
    if (p->objective == MPPI_OBJ_GATE) {
        if (!pb->gates || pb->n_gates < 1) return fail(nullptr, MPPI_E_INVAL, "gate objective needs >= 1 gate");
        if (!finite_all(pb->gates, 4 * pb->n_gates)) return fail(nullptr, MPPI_E_INVAL, "gate data must be finite");
        if (!(pb->gate_size > 0.0) || !isfinite(pb->gate_size)) return fail(nullptr, MPPI_E_INVAL, "gate_size must be > 0");
    }
    if (p->objective == MPPI_OBJ_CONTOUR) {
        if (!pb->path || pb->n_path < 2) return fail(nullptr, MPPI_E_INVAL, "contouring needs >= 2 path points");
        if (!(pb->path_len > 0.0) || !isfinite(pb->path_len)) return fail(nullptr, MPPI_E_INVAL, "path_len must be > 0");
        if (!finite_all(pb->path, 6 * pb->n_path)) return fail(nullptr, MPPI_E_INVAL, "path data must be finite");
        if (p->proj_window < 0) return fail(nullptr, MPPI_E_INVAL, "proj_window must be >= 0");
        if (!(p->v_max >= 0.0)) return fail(nullptr, MPPI_E_INVAL, "v_max must be >= 0");
        if (!(p->v_max * p->dt < pb->path_len))
            return fail(nullptr, MPPI_E_INVAL, "v_max * dt must be below the path length");
    }
    if (p->objective == MPPI_OBJ_TRACK) {
        if (!pb->xref || pb->n_ref < 1) return fail(nullptr, MPPI_E_INVAL, "tracking needs >= 1 reference row");
        if (!(pb->ref_dt > 0.0) || !isfinite(pb->ref_dt)) return fail(nullptr, MPPI_E_INVAL, "ref_dt must be > 0");
        if (!finite_all(pb->xref, 13 * pb->n_ref)) return fail(nullptr, MPPI_E_INVAL, "reference must be finite");
    }
    return MPPI_OK;
}

// Reduction tiling: one step per block, sample tiles of a multiple of 256
// samples, about two thousand blocks in all and at most 32 tiles per step.
static void plan_average(mppi_ctx *c)
{
    KArgs &a = c->args;
    const int K = c->K, N = c->N;
    int n_mt = (2048 + N - 1) / N;
    if (n_mt > 32) n_mt = 32;
    const int max_mt = (K + 255) / 256;
    if (n_mt > max_mt) n_mt = max_mt;
    if (n_mt < 1) n_mt = 1;
    int mt = (K + n_mt - 1) / n_mt;
    mt = (mt + 255) / 256 * 256;
    a.mt_size = mt;
    a.n_mt = (K + mt - 1) / mt;
    // Rollout layout: with fewer waves than SIMDs (1024 on MI355X) the chip
    // is latency bound and the two-wave split shortens each step; with more,
    // one wave per 64 samples issues fewer instructions in total.  The
    // environment variable MPPI_ROLLOUT_WAVES (1 or 2) overrides the choice.
    const int waves = (K + 1 + 63) / 64;
    a.rollout_waves = waves < 1024 ? 2 : 1;
    if (const char *e = getenv("MPPI_ROLLOUT_WAVES")) {
        if (e[0] == '1') a.rollout_waves = 1;
        if (e[0] == '2') a.rollout_waves = 2;
    }
}

extern "C" {

const char *mppi_status_string(mppi_status s)
{
    switch (s) {
    case MPPI_OK: return "MPPI_OK";
    case MPPI_E_INVAL: return "MPPI_E_INVAL";
    case MPPI_E_NOMEM: return "MPPI_E_NOMEM";
    case MPPI_E_DEVICE: return "MPPI_E_DEVICE";
    case MPPI_E_NONFINITE: return "MPPI_E_NONFINITE";
    }
    return "MPPI_E_UNKNOWN";
}

const char *mppi_last_error(const mppi_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

mppi_status mppi_create(const mppi_params *params, const mppi_quad *quad, const mppi_problem *problem,
                        void *stream, const mppi_allocator *allocator, mppi_ctx **out)
{
    if (!out) return fail(nullptr, MPPI_E_INVAL, "out is NULL");
    *out = nullptr;
    g_create_err.clear();
    mppi_status st = validate(params, quad, problem);
    if (st != MPPI_OK) return st;
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(nullptr, MPPI_E_INVAL, "allocator needs both alloc and free");

    mppi_ctx *c = new (std::nothrow) mppi_ctx();
    if (!c) return fail(nullptr, MPPI_E_NOMEM, "host allocation failed");
    c->prm = *params;
    c->quad = *quad;
    c->K = params->K;
    c->N = params->N;
    c->objective = params->objective;
    c->C = params->objective == MPPI_OBJ_CONTOUR ? 5 : 4;
    c->fp64 = params->precision == MPPI_FP64;
    c->acc64 = c->fp64 || params->K >= 65536;
    if (allocator) { c->alloc = *allocator; c->have_alloc = true; }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            release(c);
            return fail(nullptr, MPPI_E_DEVICE, "hipStreamCreateWithFlags failed");
        }
        c->own_stream = true;
    }
    c->G = params->objective == MPPI_OBJ_GATE ? problem->n_gates : 0;
    c->P = params->objective == MPPI_OBJ_CONTOUR ? problem->n_path : 0;
    c->R = params->objective == MPPI_OBJ_TRACK ? problem->n_ref : 0;

    KArgs &a = c->args;
    const mppi_params &p = *params;
    const mppi_quad &q = *quad;
    a.K = c->K; a.N = c->N; a.G = c->G; a.P = c->P; a.R = c->R; a.objective = c->objective;
    a.proj_window = p.proj_window;
    a.has_drag = (q.drag[0] != 0.0 || q.drag[1] != 0.0 || q.drag[2] != 0.0) ? 1 : 0;
    a.seed_lo = (uint32_t)(p.seed & 0xffffffffu);
    a.seed_hi = (uint32_t)(p.seed >> 32);
    a.inv_mass = 1.0 / q.mass;
    a.gravity = q.gravity;
    a.arm_s = q.arm / sqrt(2.0);
    a.c_tau = q.c_tau;
    for (int i = 0; i < 3; ++i) { a.inv_J[i] = 1.0 / q.inertia[i]; a.drag[i] = q.drag[i]; }
    a.gyro[0] = (q.inertia[2] - q.inertia[1]) / q.inertia[0];
    a.gyro[1] = (q.inertia[0] - q.inertia[2]) / q.inertia[1];
    a.gyro[2] = (q.inertia[1] - q.inertia[0]) / q.inertia[2];
    a.t_min = q.t_min; a.t_max = q.t_max; a.w_max = q.w_max;
    a.hover = q.mass * q.gravity / 4.0;
    a.dt = p.dt; a.lambda = p.lambda;
    for (int i = 0; i < 4; ++i) { a.sigma[i] = p.sigma[i]; a.R_dT[i] = p.R_dT[i]; }
    a.sigma_v = p.sigma_v;
    a.w_lim = p.w_lim; a.q_near = p.q_near; a.r_near = p.r_near;
    a.gate_half = 0.5 * problem->gate_size;
    for (int i = 0; i < 13; ++i) { a.Q[i] = p.Q[i]; a.QN[i] = p.QN[i]; }
    a.q_l = p.q_l; a.q_c = p.q_c;
    for (int i = 0; i < 3; ++i) a.Q_w[i] = p.Q_w[i];
    a.r_dv = p.r_dv; a.mu = p.mu; a.v_max = p.v_max;
    a.path_len = problem->path_len;
    a.ref_dt = problem->ref_dt;
    plan_average(c);

    const size_t rs = c->fp64 ? sizeof(double) : sizeof(float);
    const size_t as = c->acc64 ? sizeof(double) : sizeof(float);
    const size_t K = (size_t)c->K, N = (size_t)c->N;
    struct Want { void **dst; size_t bytes; };
    void *gates_d = nullptr, *gates_r = nullptr, *path_d = nullptr, *path_r = nullptr, *xref_r = nullptr;
    void *warm = nullptr, *wU = nullptr, *wV = nullptr, *cur = nullptr, *res = nullptr, *req = nullptr;
    void *ctrl = nullptr, *vctrl = nullptr, *nomU = nullptr, *nomV = nullptr, *J = nullptr, *part = nullptr;
    void *front8 = nullptr, *tickets = nullptr;
    Want wants[] = {
        {&warm, sizeof(DevWarm)}, {&wU, sizeof(double) * kNMax * 4}, {&wV, sizeof(double) * kNMax},
        {&cur, sizeof(DevCur)}, {&res, sizeof(DevResult)}, {&req, sizeof(double) * kReqDoubles},
        {&ctrl, rs * 4 * K * N}, {&nomU, rs * 4 * N}, {&nomV, rs * N}, {&J, rs * K},
        {&part, as * ((size_t)a.n_mt * N * (size_t)c->C + 2 * (size_t)a.n_mt + N * (size_t)c->C + 2)},
        {&tickets, sizeof(uint32_t) * (kNMax + 1)}, {&front8, N + 1},
    };
    for (auto &w : wants) {
        *w.dst = dev_alloc(c, w.bytes);
        if (!*w.dst) {
            release(c);
            return fail(nullptr, MPPI_E_NOMEM, "device allocation of %zu bytes failed", w.bytes);
        }
    }
    if (c->objective == MPPI_OBJ_CONTOUR) {
        vctrl = dev_alloc(c, rs * K * N);
        path_d = dev_alloc(c, sizeof(double) * 6 * (size_t)c->P);
        path_r = dev_alloc(c, rs * 8 * (size_t)c->P);
        if (!vctrl || !path_d || !path_r) { release(c); return fail(nullptr, MPPI_E_NOMEM, "device allocation failed"); }
    }
    if (c->objective == MPPI_OBJ_GATE) {
        gates_d = dev_alloc(c, sizeof(double) * 4 * (size_t)c->G);
        gates_r = dev_alloc(c, rs * 8 * (size_t)c->G);
        if (!gates_d || !gates_r) { release(c); return fail(nullptr, MPPI_E_NOMEM, "device allocation failed"); }
    }
    if (c->objective == MPPI_OBJ_TRACK) {
        xref_r = dev_alloc(c, rs * 16 * (size_t)c->R + sizeof(double) * 13 * (size_t)c->R);
        if (!xref_r) { release(c); return fail(nullptr, MPPI_E_NOMEM, "device allocation failed"); }
    }
    if (hipHostMalloc((void **)&c->h_req, sizeof(double) * kReqDoubles, 0) != hipSuccess ||
        hipHostMalloc((void **)&c->h_res, sizeof(DevResult), 0) != hipSuccess ||
        hipHostMalloc((void **)&c->h_U, sizeof(double) * 4 * kNMax, 0) != hipSuccess) {
        release(c);
        return fail(nullptr, MPPI_E_NOMEM, "pinned host allocation failed");
    }
    a.gates_d = (const double *)gates_d; a.gates_r = gates_r;
    a.path_d = (const double *)path_d; a.path_r = path_r; a.xref_r = xref_r;
    a.warm = (DevWarm *)warm; a.wU = (double *)wU; a.wV = (double *)wV;
    a.cur = (DevCur *)cur; a.res = (DevResult *)res;
    a.ctrl = ctrl; a.vctrl = vctrl; a.nomU = nomU; a.nomV = nomV; a.J = J; a.part = part;
    a.front8 = (uint8_t *)front8;
    a.tickets = (uint32_t *)tickets;
    c->warm = (DevWarm *)warm; c->res = (DevResult *)res; c->req = (double *)req;

    // problem data, initial (cold) warm state
    hipError_t e = hipSuccess;
    if (gates_d) e = hipMemcpyAsync(gates_d, problem->gates, sizeof(double) * 4 * c->G, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && path_d)
        e = hipMemcpyAsync(path_d, problem->path, sizeof(double) * 6 * c->P, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && xref_r)
        e = hipMemcpyAsync((char *)xref_r + rs * 16 * (size_t)c->R, problem->xref, sizeof(double) * 13 * c->R,
                           hipMemcpyHostToDevice, c->stream);
    DevWarm w0;
    memset(&w0, 0, sizeof w0);
    w0.N = c->N;
    if (e == hipSuccess) e = hipMemcpyAsync(warm, &w0, sizeof w0, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(wU, 0, sizeof(double) * kNMax * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(wV, 0, sizeof(double) * kNMax, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(res, 0, sizeof(DevResult), c->stream);
    if (e == hipSuccess) e = launch_setup(a, c->fp64, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        release(c);
        return fail(nullptr, MPPI_E_DEVICE, "context set-up failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return MPPI_OK;
}

void mppi_destroy(mppi_ctx *ctx) { release(ctx); }

mppi_status mppi_solve_device(mppi_ctx *ctx, const double *d_req, double *d_u0)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    if (!d_req) return fail(ctx, MPPI_E_INVAL, "d_req is NULL");
    ctx->err.clear();
    KArgs a = ctx->args;
    a.req = d_req;
    a.u0_out = d_u0;
    HIP_TRY(ctx, launch_solve(a, ctx->fp64, ctx->acc64, ctx->stream, next_events(ctx)));
    return MPPI_OK;
}

mppi_status mppi_set_profiling(mppi_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    if (enable && ctx->events.empty()) {
        ctx->events.resize(4 * (size_t)kProfSlots, nullptr);
        for (auto &e : ctx->events) HIP_TRY(ctx, hipEventCreate(&e));
    }
    ctx->profiling = enable != 0;
    ctx->prof_count = 0;
    return MPPI_OK;
}

mppi_status mppi_read_profile(mppi_ctx *ctx, double mean_ms[3], int32_t *n_solves)
{
    if (!ctx || !mean_ms) return fail(ctx, MPPI_E_INVAL, "ctx and mean_ms are required");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < ctx->prof_count; ++i) {
        for (int j = 0; j < 3; ++j) {
            float ms = 0.0f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->events[4 * (size_t)i + j], ctx->events[4 * (size_t)i + j + 1]));
            acc[j] += ms;
        }
    }
    for (int j = 0; j < 3; ++j) mean_ms[j] = ctx->prof_count ? acc[j] / ctx->prof_count : 0.0;
    if (n_solves) *n_solves = ctx->prof_count;
    ctx->prof_count = 0;
    return MPPI_OK;
}

static mppi_status copy_info(mppi_ctx *ctx, const DevResult &r, mppi_info *info)
{
    if (info) {
        info->J_min = r.J_min;
        info->S = r.S;
        info->ess = r.ess;
        info->J_nom = r.J_nom;
        info->theta0 = r.theta0;
        info->status = r.status;
        info->g0 = r.g0;
        info->i0 = r.i0;
        info->shift = r.shift;
        info->solve_index = r.s;
        info->pad_ = 0;
    }
    if (r.status == ST_NONFINITE)
        return fail(ctx, MPPI_E_NONFINITE, "every sample cost was non-finite; warm state kept");
    return (mppi_status)r.status;
}

mppi_status mppi_solve(mppi_ctx *ctx, const double x0[13], double t_now, double u0_out[4], double *U_out,
                       mppi_info *info)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    if (!x0 || !u0_out) return fail(ctx, MPPI_E_INVAL, "x0 and u0_out are required");
    if (!finite_all(x0, 13) || !isfinite(t_now)) return fail(ctx, MPPI_E_INVAL, "x0 and t_now must be finite");
    const double qn = x0[6] * x0[6] + x0[7] * x0[7] + x0[8] * x0[8] + x0[9] * x0[9];
    if (!(qn > 0.0)) return fail(ctx, MPPI_E_INVAL, "quaternion of x0 has zero norm");
    ctx->err.clear();
    for (int i = 0; i < 13; ++i) ctx->h_req[i] = x0[i];
    ctx->h_req[13] = t_now;
    ctx->h_req[14] = ctx->h_req[15] = 0.0;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->req, ctx->h_req, sizeof(double) * kReqDoubles, hipMemcpyHostToDevice,
                                ctx->stream));
    KArgs a = ctx->args;
    a.req = ctx->req;
    a.u0_out = nullptr;
    HIP_TRY(ctx, launch_solve(a, ctx->fp64, ctx->acc64, ctx->stream, next_events(ctx)));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_res, ctx->res, sizeof(DevResult), hipMemcpyDeviceToHost, ctx->stream));
    if (U_out)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->h_U, ctx->args.wU, sizeof(double) * 4 * ctx->N, hipMemcpyDeviceToHost,
                                    ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const DevResult r = *ctx->h_res;
    mppi_status s = copy_info(ctx, r, info);
    if (s != MPPI_OK) return s;
    for (int i = 0; i < 4; ++i) u0_out[i] = r.u0[i];
    if (U_out) memcpy(U_out, ctx->h_U, sizeof(double) * 4 * ctx->N);
    return MPPI_OK;
}

mppi_status mppi_read_info(mppi_ctx *ctx, mppi_info *info)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_res, ctx->res, sizeof(DevResult), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return copy_info(ctx, *ctx->h_res, info);
}

mppi_status mppi_read_samples(mppi_ctx *ctx, double *J, double *U_samples)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const size_t K = (size_t)ctx->K, N = (size_t)ctx->N;
    if (J) {
        if (ctx->fp64) {
            HIP_TRY(ctx, hipMemcpy(J, ctx->args.J, sizeof(double) * K, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(K);
            HIP_TRY(ctx, hipMemcpy(tmp.data(), ctx->args.J, sizeof(float) * K, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < K; ++i) J[i] = tmp[i];
        }
    }
    if (U_samples) {
        if (ctx->fp64) {
            HIP_TRY(ctx, hipMemcpy(U_samples, ctx->args.ctrl, sizeof(double) * 4 * K * N, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(4 * K * N);
            HIP_TRY(ctx, hipMemcpy(tmp.data(), ctx->args.ctrl, sizeof(float) * 4 * K * N, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < 4 * K * N; ++i) U_samples[i] = tmp[i];
        }
    }
    return MPPI_OK;
}

mppi_status mppi_get_warm(mppi_ctx *ctx, mppi_warm *out)
{
    if (!ctx || !out) return fail(ctx, MPPI_E_INVAL, "ctx and out are required");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    DevWarm w;
    HIP_TRY(ctx, hipMemcpy(&w, ctx->warm, sizeof w, hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    HIP_TRY(ctx, hipMemcpy(out->U, ctx->args.wU, sizeof(double) * 4 * kNMax, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(out->V, ctx->args.wV, sizeof(double) * kNMax, hipMemcpyDeviceToHost));
    out->warm = w.warm;
    out->g0 = w.g0;
    out->solve_index = w.s;
    out->N = ctx->N;
    memcpy(out->allow, w.allow, sizeof w.allow);
    out->t_prev = w.t_prev;
    memcpy(out->x_prev, w.x_prev, sizeof w.x_prev);
    out->theta0 = w.theta0;
    return MPPI_OK;
}

mppi_status mppi_set_warm(mppi_ctx *ctx, const mppi_warm *in)
{
    if (!ctx || !in) return fail(ctx, MPPI_E_INVAL, "ctx and in are required");
    if (in->N != ctx->N) return fail(ctx, MPPI_E_INVAL, "warm state has N=%d, context N=%d", in->N, ctx->N);
    if (ctx->objective == MPPI_OBJ_GATE && (in->g0 < 0 || in->g0 >= ctx->G))
        return fail(ctx, MPPI_E_INVAL, "g0=%d outside [0, %d)", in->g0, ctx->G);
    if (!finite_all(in->U, 4 * ctx->N) || !finite_all(in->V, ctx->N) || !finite_all(in->x_prev, 13) ||
        !isfinite(in->t_prev) || !isfinite(in->theta0))
        return fail(ctx, MPPI_E_INVAL, "warm state must be finite");
    DevWarm w;
    memset(&w, 0, sizeof w);
    w.warm = in->warm ? 1 : 0;
    w.g0 = in->g0;
    w.s = in->solve_index;
    w.N = ctx->N;
    memcpy(w.allow, in->allow, sizeof w.allow);
    w.t_prev = in->t_prev;
    memcpy(w.x_prev, in->x_prev, sizeof w.x_prev);
    w.theta0 = in->theta0;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipMemcpy(ctx->warm, &w, sizeof w, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(ctx->args.wU, in->U, sizeof(double) * 4 * kNMax, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(ctx->args.wV, in->V, sizeof(double) * kNMax, hipMemcpyHostToDevice));
    return MPPI_OK;
}

// Host plant: the same rigid-body model, integrated in binary64.
static void plant_deriv(const mppi_quad *q, const double *x, const double *u, double *d)
{
    const double qw = x[6], qx = x[7], qy = x[8], qz = x[9];
    const double wx = x[10], wy = x[11], wz = x[12];
    const double F = u[0] + u[1] + u[2] + u[3];
    const double as = q->arm / sqrt(2.0);
    const double tx = as * (u[0] + u[1] - u[2] - u[3]);
    const double ty = as * (-u[0] + u[1] + u[2] - u[3]);
    const double tz = q->c_tau * (u[0] - u[1] + u[2] - u[3]);
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                         2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                         2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double b[3];
    for (int i = 0; i < 3; ++i) b[i] = q->drag[i] * (R[i] * x[3] + R[3 + i] * x[4] + R[6 + i] * x[5]);
    for (int i = 0; i < 3; ++i) d[i] = x[3 + i];
    for (int i = 0; i < 3; ++i)
        d[3 + i] = R[3 * i + 2] * F / q->mass - (R[3 * i] * b[0] + R[3 * i + 1] * b[1] + R[3 * i + 2] * b[2]);
    d[5] -= q->gravity;
    d[6] = 0.5 * (-qx * wx - qy * wy - qz * wz);
    d[7] = 0.5 * (qw * wx + qy * wz - qz * wy);
    d[8] = 0.5 * (qw * wy - qx * wz + qz * wx);
    d[9] = 0.5 * (qw * wz + qx * wy - qy * wx);
    const double *J = q->inertia;
    d[10] = (tx - (J[2] - J[1]) * wy * wz) / J[0];
    d[11] = (ty - (J[0] - J[2]) * wz * wx) / J[1];
    d[12] = (tz - (J[1] - J[0]) * wx * wy) / J[2];
}

mppi_status mppi_plant_step(const mppi_quad *quad, const double x[13], const double u[4], double dt,
                            int32_t substeps, double x_out[13])
{
    if (!quad || !x || !u || !x_out || substeps < 1 || !(dt > 0.0))
        return fail(nullptr, MPPI_E_INVAL, "invalid plant step arguments");
    double s[13], k1[13], k2[13], k3[13], k4[13], t[13];
    memcpy(s, x, sizeof s);
    const double h = dt / substeps;
    for (int n = 0; n < substeps; ++n) {
        plant_deriv(quad, s, u, k1);
        for (int i = 0; i < 13; ++i) t[i] = s[i] + 0.5 * h * k1[i];
        plant_deriv(quad, t, u, k2);
        for (int i = 0; i < 13; ++i) t[i] = s[i] + 0.5 * h * k2[i];
        plant_deriv(quad, t, u, k3);
        for (int i = 0; i < 13; ++i) t[i] = s[i] + h * k3[i];
        plant_deriv(quad, t, u, k4);
        for (int i = 0; i < 13; ++i) s[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        const double nq = sqrt(s[6] * s[6] + s[7] * s[7] + s[8] * s[8] + s[9] * s[9]);
        for (int i = 6; i < 10; ++i) s[i] /= nq;
    }
    memcpy(x_out, s, sizeof s);
    return MPPI_OK;
}

}  // extern "C"
