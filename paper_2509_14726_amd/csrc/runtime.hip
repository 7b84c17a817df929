// Host runtime behind the C ABI declared in include/mppi.h: argument
// validation, device memory of a context, the launch sequence of one solve,
// result transfer, warm-start export/import, and the host plant step.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mppi.h"
#include "device.hpp"
#include "kernels.hpp"

using namespace mppi;

static_assert(MPPI_MASK_WORDS == kMaskWords, "mask width");
static_assert(MPPI_N_MAX == kNMax, "horizon bound");
static_assert(MPPI_G_MAX == kGMax, "gate bound");
static_assert(MPPI_REQ_DOUBLES == kReqDoubles, "request record");
static_assert(MPPI_SCRATCH_BYTES == kScratchBytes, "fixed workspace size");

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
    bool external_ws = false;   // per-solve scratch is lent by a server
    size_t ws_bytes = 0;        // size of that scratch
    int device = 0;             // device current at creation
    int n_iter = 1;             // MPPI iterations per solve
    bool no_tensor = false;     // the last solve's average drew the samples again
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

// ------------------------------------------------------------ autotuner cache
//
// A JSON object in one file, one entry per line:
//   "<key>": {"rollout_waves": W, "rollout_groups": R, "sample_groups": S, "regen_average": G, "ms": T},
// rewritten whole through a temporary file and a rename.
namespace tune {

struct Entry {
    int waves = 0, groups = 0, sgroups = 0, regen = 0;
    double ms = 0.0;
};

// The gfx architecture of a device, without its feature suffixes.
static std::string arch_of(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string s = prop.gcnArchName;
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

static int bucket(double x) { return x >= 1.0 ? (int)floor(log2(x)) : 0; }

static const char *prec_name(bool fp64) { return fp64 ? "fp64" : "fp32"; }

static bool field(const std::string &line, const char *name, double &out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t i = line.find(pat);
    if (i == std::string::npos) return false;
    char *end = nullptr;
    const char *p = line.c_str() + i + pat.size();
    out = strtod(p, &end);
    return end != p;
}

// Every entry of the file as (key, line); an unreadable file is empty.
static std::vector<std::pair<std::string, std::string>> read_all(const char *path)
{
    std::vector<std::pair<std::string, std::string>> out;
    FILE *f = fopen(path, "r");
    if (!f) return out;
    char buf[1024];
    while (fgets(buf, sizeof buf, f)) {
        std::string line(buf);
        while (!line.empty() && (line.back() == '\n' || line.back() == '\r' || line.back() == ',')) line.pop_back();
        if (line.size() < 2 || line[0] != '"') continue;
        const size_t q = line.find('"', 1);
        if (q == std::string::npos) continue;
        out.emplace_back(line.substr(1, q - 1), line);
    }
    fclose(f);
    return out;
}

static bool load(const char *path, const std::string &key, Entry &e)
{
    if (!path) return false;
    for (const auto &kv : read_all(path)) {
        if (kv.first != key) continue;
        double w = 0, g = 0, sg = 0, r = 0, ms = 0;
        if (!field(kv.second, "rollout_waves", w) || !field(kv.second, "rollout_groups", g) ||
            !field(kv.second, "sample_groups", sg) || !field(kv.second, "regen_average", r) ||
            !field(kv.second, "ms", ms))
            return false;
        e.waves = (int)w; e.groups = (int)g; e.sgroups = (int)sg; e.regen = (int)r; e.ms = ms;
        return true;
    }
    return false;
}

// Adds or replaces the entry of key; false when the file cannot be written.
static bool store(const char *path, const std::string &key, const Entry &e)
{
    if (!path) return true;
    auto all = read_all(path);
    char buf[512];
    snprintf(buf, sizeof buf,
             "\"%s\": {\"rollout_waves\": %d, \"rollout_groups\": %d, \"sample_groups\": %d, "
             "\"regen_average\": %d, \"ms\": %.6f}",
             key.c_str(), e.waves, e.groups, e.sgroups, e.regen, e.ms);
    bool found = false;
    for (auto &kv : all)
        if (kv.first == key) { kv.second = buf; found = true; }
    if (!found) all.emplace_back(key, buf);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fputs("{\n", f);
    for (size_t i = 0; i < all.size(); ++i) fprintf(f, "%s%s\n", all[i].second.c_str(), i + 1 < all.size() ? "," : "");
    fputs("}\n", f);
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace tune

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
    if (p->n_iter < 0 || p->n_iter > 64) return fail(nullptr, MPPI_E_INVAL, "n_iter=%d outside [0, 64]", p->n_iter);
    if (!(p->ctrl_cost >= 0.0) || !isfinite(p->ctrl_cost))
        return fail(nullptr, MPPI_E_INVAL, "ctrl_cost must be finite and >= 0");
    if (p->input_model != MPPI_INPUT_THRUST && p->input_model != MPPI_INPUT_RATE)
        return fail(nullptr, MPPI_E_INVAL, "unknown input model %d", p->input_model);
    if (p->input_model == MPPI_INPUT_RATE &&
        (!finite_all(p->rate_lim, 2) || !finite_all(p->dv_lim, 2) || !(p->rate_lim[0] <= 0.0) ||
         !(p->rate_lim[1] >= 0.0) || !(p->dv_lim[0] <= 0.0) || !(p->dv_lim[1] >= 0.0)))
        return fail(nullptr, MPPI_E_INVAL, "rate model bounds must be finite with lower <= 0 <= upper");
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
        if (pb->n_gates > kGMax) return fail(nullptr, MPPI_E_INVAL, "at most %d gates", kGMax);
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

// Rollout tiles of 64 samples (the nominal is sample K) and the layout.
static void plan_layout(mppi_ctx *c)
{
    KArgs &a = c->args;
    const int K = c->K;
    a.n_tiles = (K + 1 + 63) / 64;
    // Rollout layout: with few 64-sample tiles the chip is latency bound and
    // splitting each tile's step over four pipelined waves (sampling with body
    // rates, attitude, translation, sampling with position costs), one per
    // SIMD, shortens each step.  With chunks of 4 steps its LDS rings hold one
    // such workgroup per CU; with chunks of 2 (binary32) two share a CU, which
    // takes up to two tiles per CU in one round.  Beyond that one wave per 64
    // samples, which issues the fewest instructions, keeps the whole chip
    // busy.  Binary64 rings (chunks of 2) fit one workgroup per CU, so from
    // one to two tiles per CU the two-wave split (attitude | translation, two
    // workgroups per CU) takes over there.  Measured on 256 CUs for N = 50,
    // 100 and 200 at 129 to 1016 tiles.  The environment variable
    // MPPI_ROLLOUT_WAVES (1..4) overrides the layout.
    int n_cu = 0, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    c->device = dev;
    if (n_cu < 1) n_cu = 256;
    if (a.n_tiles <= n_cu) a.rollout_waves = 4;
    else if (a.n_tiles <= 2 * n_cu) a.rollout_waves = c->fp64 ? 2 : 4;
    else a.rollout_waves = 1;
    if (const char *e = getenv("MPPI_ROLLOUT_WAVES")) {
        if (e[0] >= '1' && e[0] <= '4') a.rollout_waves = e[0] - '0';
    }
    a.ring4_b = (!c->fp64 && a.n_tiles <= n_cu) ? 4 : 2;
    // The one-wave rollout draws its samples itself (binary32) when the
    // sample tensor exceeds the 256 MiB last-level cache: the separate
    // sample pass then costs more than the draw adds to the rollout.  Below
    // that the average reads a cached tensor, and the separate pass is as
    // fast or faster (measured at K = 32768 and 65000, N = 100 and 200).
    // MPPI_ROLLOUT_DRAW (0 or 1) overrides the rule.
    const double tensor_bytes = 16.0 * (double)c->K * (double)c->N;
    a.rollout_draw = (!c->fp64 && a.rollout_waves == 1 && tensor_bytes > 256.0 * 1048576.0) ? 1 : 0;
    if (const char *e = getenv("MPPI_ROLLOUT_DRAW")) {
        if (e[0] == '0' || e[0] == '1') a.rollout_draw = (!c->fp64 && a.rollout_waves == 1) ? e[0] - '0' : 0;
    }
}

// The average can draw the samples again only where the rollout draws them
// (three- and four-wave layouts, the drawing one-wave layout), with thrust as
// the input (a rate sample follows its thrust chain), and not when the
// control-cost term reads the sample tensor.
static bool can_regen(const KArgs &a)
{
    const bool draws = a.rollout_waves >= 3 || (a.rollout_waves == 1 && a.rollout_draw == 1);
    return draws && a.input_model == INPUT_THRUST && a.ctrl_cost == 0.0;
}

// Point the per-solve buffers of a at a workspace of ws_layout's size.
static void bind_workspace(KArgs &a, char *w)
{
    const WsLayout wl = ws_layout(a.K, a.N, a.C, a.real_bytes);
    a.ctrl = w + wl.ctrl;
    a.vctrl = a.C == 5 ? w + wl.vctrl : nullptr;
    a.nomU = w + wl.nomU;
    a.nomV = w + wl.nomV;
    a.J = w + wl.J;
    a.tmin = w + wl.tmin;
    a.front8 = (uint8_t *)(w + wl.front8);
}

// The launch sequence of one solve: n_iter MPPI iterations, the later ones
// marked inner (no shift, the first iteration's last applied input).
static mppi_status launch_iterations(mppi_ctx *ctx, KArgs a)
{
    ctx->no_tensor = a.regen != 0;
    for (int it = 0; it < ctx->n_iter; ++it) {
        a.inner = it > 0 ? 1 : 0;
        HIP_TRY(ctx, launch_solve(a, ctx->fp64, ctx->acc64, ctx->stream, next_events(ctx)));
    }
    return MPPI_OK;
}

extern "C" {

const char *mppi_status_string(int32_t s)
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
    // cold-start nominal: hover thrust for the thrust input; for the rate
    // input the zero sequence of Alg. 1, which holds the measured thrusts
    a.hover = p.input_model == MPPI_INPUT_RATE ? 0.0 : q.mass * q.gravity / 4.0;
    a.dt = p.dt; a.lambda = p.lambda;
    for (int i = 0; i < 4; ++i) { a.sigma[i] = p.sigma[i]; a.R_dT[i] = p.R_dT[i]; }
    a.sigma_v = p.sigma_v;
    a.ctrl_cost = p.ctrl_cost;
    a.input_model = p.input_model;
    for (int i = 0; i < 2; ++i) { a.rate_lim[i] = p.rate_lim[i]; a.dv_lim[i] = p.dv_lim[i]; }
    for (int i = 0; i < 4; ++i) a.inv_sig2[i] = p.sigma[i] > 0.0 ? 1.0 / (p.sigma[i] * p.sigma[i]) : 0.0;
    a.inv_sig2[4] = p.sigma_v > 0.0 ? 1.0 / (p.sigma_v * p.sigma_v) : 0.0;
    c->n_iter = p.n_iter > 1 ? p.n_iter : 1;
    a.w_lim = p.w_lim; a.q_near = p.q_near; a.r_near = p.r_near;
    a.gate_half = 0.5 * problem->gate_size;
    for (int i = 0; i < 13; ++i) { a.Q[i] = p.Q[i]; a.QN[i] = p.QN[i]; }
    a.q_l = p.q_l; a.q_c = p.q_c;
    for (int i = 0; i < 3; ++i) a.Q_w[i] = p.Q_w[i];
    a.r_dv = p.r_dv; a.mu = p.mu; a.v_max = p.v_max;
    a.path_len = problem->path_len;
    a.ref_dt = problem->ref_dt;
    plan_layout(c);
    if (p.input_model == MPPI_INPUT_RATE) {
        // a rate sample follows its thrust chain along the horizon, which the
        // sampling kernel walks per sample: the one-wave rollout reads it
        a.rollout_waves = 1;
        a.rollout_draw = 0;
    }

    const size_t rs = c->fp64 ? sizeof(double) : sizeof(float);
    a.C = c->C;
    a.real_bytes = (int32_t)rs;
    c->external_ws = (params->flags & MPPI_FLAG_EXTERNAL_WORKSPACE) != 0;
    a.regen = ((params->flags & MPPI_FLAG_REGEN_AVERAGE) != 0 && can_regen(a)) ? 1 : 0;
    struct Want { void **dst; size_t bytes; };
    void *gates_d = nullptr, *gates_r = nullptr, *path_d = nullptr, *path_r = nullptr, *xref_r = nullptr;
    void *warm = nullptr, *wU = nullptr, *wV = nullptr, *cur = nullptr, *res = nullptr, *req = nullptr;
    void *ws = nullptr;
    const WsLayout wl = ws_layout(c->K, c->N, c->C, (int)rs);
    c->ws_bytes = wl.total;
    Want wants[] = {
        {&warm, sizeof(DevWarm)}, {&wU, sizeof(double) * kNMax * 4}, {&wV, sizeof(double) * kNMax},
        {&cur, sizeof(DevCur)}, {&res, sizeof(DevResult)}, {&req, sizeof(double) * kReqDoubles},
        {&ws, c->external_ws ? 0 : wl.total},
    };
    for (auto &w : wants) {
        if (w.dst == &ws && c->external_ws) continue;
        *w.dst = dev_alloc(c, w.bytes);
        if (!*w.dst) {
            release(c);
            return fail(nullptr, MPPI_E_NOMEM, "device allocation of %zu bytes failed", w.bytes);
        }
    }
    if (c->objective == MPPI_OBJ_CONTOUR) {
        path_d = dev_alloc(c, sizeof(double) * 6 * (size_t)c->P);
        path_r = path_d ? dev_alloc(c, rs * 8 * (size_t)c->P) : nullptr;
        if (!path_d || !path_r) { release(c); return fail(nullptr, MPPI_E_NOMEM, "device allocation failed"); }
    }
    if (c->objective == MPPI_OBJ_GATE) {
        gates_d = dev_alloc(c, sizeof(double) * 12 * (size_t)c->G);  // G x 4 as given, G x 8 frames
        gates_r = gates_d ? dev_alloc(c, rs * 8 * (size_t)c->G) : nullptr;
        if (!gates_d || !gates_r) { release(c); return fail(nullptr, MPPI_E_NOMEM, "device allocation failed"); }
    }
    if (c->objective == MPPI_OBJ_TRACK) {
        xref_r = dev_alloc(c, rs * 16 * (size_t)c->R + sizeof(double) * 13 * (size_t)c->R);
        if (!xref_r) { release(c); return fail(nullptr, MPPI_E_NOMEM, "device allocation failed"); }
    }
    // the stream after the device memory: with an allocator callback, a failed
    // allocation above returns before any HIP call
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            release(c);
            return fail(nullptr, MPPI_E_DEVICE, "hipStreamCreateWithFlags failed");
        }
        c->own_stream = true;
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
    if (ws) bind_workspace(a, (char *)ws);
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
    DevCur c0;
    memset(&c0, 0, sizeof c0);
    if (e == hipSuccess) e = hipMemcpyAsync(cur, &c0, sizeof c0, hipMemcpyHostToDevice, c->stream);
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
    if (ctx->external_ws) return fail(ctx, MPPI_E_INVAL, "context has no workspace of its own (server context)");
    ctx->err.clear();
    KArgs a = ctx->args;
    a.req = d_req;
    a.u0_out = d_u0;
    return launch_iterations(ctx, a);
}

mppi_status mppi_solve_device_noalloc(mppi_ctx *ctx, const double *d_req, double *d_u0)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    if (!d_req) return fail(ctx, MPPI_E_INVAL, "d_req is NULL");
    if (ctx->ws_bytes > kScratchBytes)
        return fail(ctx, MPPI_E_INVAL, "solve workspace of %zu bytes exceeds the fixed workspace of %zu bytes",
                    ctx->ws_bytes, kScratchBytes);
    int dev = -1;
    HIP_TRY(ctx, hipGetDevice(&dev));
    if (dev != ctx->device)
        return fail(ctx, MPPI_E_INVAL, "current device %d is not the context's device %d", dev, ctx->device);
    ctx->err.clear();
    void *base = nullptr;
    HIP_TRY(ctx, scratch_address(&base));
    KArgs a = ctx->args;
    bind_workspace(a, (char *)base);
    a.req = d_req;
    a.u0_out = d_u0;
    return launch_iterations(ctx, a);
}

mppi_status mppi_set_profiling(mppi_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    if (enable && ctx->events.empty()) {
        ctx->events.resize(4 * (size_t)kProfSlots, nullptr);
        // timing-only events: no system-scope fence (cache write-back) when
        // they are recorded, so they do not stretch the kernels they bracket;
        // mppi_read_profile synchronizes the stream before reading them
        for (auto &e : ctx->events) HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
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
        info->rollout_waves = ctx->args.rollout_waves;
        info->regen_average = ctx->args.regen;
        info->rollout_draw = ctx->args.rollout_draw;
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
    const bool rate = ctx->args.input_model == MPPI_INPUT_RATE;
    if (!finite_all(x0, rate ? 17 : 13) || !isfinite(t_now))
        return fail(ctx, MPPI_E_INVAL, "x0 and t_now must be finite");
    if (ctx->external_ws) return fail(ctx, MPPI_E_INVAL, "context has no workspace of its own (server context)");
    const double qn = x0[6] * x0[6] + x0[7] * x0[7] + x0[8] * x0[8] + x0[9] * x0[9];
    if (!(qn > 0.0)) return fail(ctx, MPPI_E_INVAL, "quaternion of x0 has zero norm");
    ctx->err.clear();
    for (int i = 0; i < kReqDoubles; ++i) ctx->h_req[i] = 0.0;
    for (int i = 0; i < 13; ++i) ctx->h_req[i] = x0[i];
    ctx->h_req[13] = t_now;
    if (rate)
        for (int i = 0; i < 4; ++i) ctx->h_req[kReqThrust + i] = x0[13 + i];
    HIP_TRY(ctx, hipMemcpyAsync(ctx->req, ctx->h_req, sizeof(double) * kReqDoubles, hipMemcpyHostToDevice,
                                ctx->stream));
    KArgs a = ctx->args;
    a.req = ctx->req;
    a.u0_out = nullptr;
    mppi_status ls = launch_iterations(ctx, a);
    if (ls != MPPI_OK) return ls;
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
    if (ctx->external_ws) return fail(ctx, MPPI_E_INVAL, "context has no workspace of its own (server context)");
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
        if (ctx->no_tensor)
            return fail(ctx, MPPI_E_INVAL,
                        "the last solve's weighted average drew the samples again (MPPI_FLAG_REGEN_AVERAGE, the "
                        "autotuner's or the batch's choice): it kept no sample tensor");
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

}  // extern "C"

// What a solve changes on the device besides its workspace: the warm-start
// state, the handed-on sequences, the per-solve head values and the report.
// The autotuners copy it aside before timing real solves and back after.
struct Snapshot {
    void *buf = nullptr;
    Snapshot() = default;
    Snapshot(const Snapshot &) = delete;
    Snapshot &operator=(const Snapshot &) = delete;
    static size_t bytes() { return sizeof(DevWarm) + sizeof(double) * kNMax * 5 + sizeof(DevCur) + sizeof(DevResult); }
    hipError_t take(const KArgs &a, hipStream_t st)
    {
        if (!buf) {
            const hipError_t e = hipMalloc(&buf, bytes());
            if (e != hipSuccess) { buf = nullptr; return e; }
        }
        return copy(a, st, true);
    }
    hipError_t restore(const KArgs &a, hipStream_t st) { return copy(a, st, false); }
    hipError_t copy(const KArgs &a, hipStream_t st, bool out)
    {
        char *p = (char *)buf;
        void *dev[5] = {a.warm, a.wU, a.wV, a.cur, a.res};
        const size_t sz[5] = {sizeof(DevWarm), sizeof(double) * kNMax * 4, sizeof(double) * kNMax, sizeof(DevCur),
                              sizeof(DevResult)};
        for (int i = 0; i < 5; ++i) {
            const hipError_t e = out ? hipMemcpyAsync(p, dev[i], sz[i], hipMemcpyDeviceToDevice, st)
                                     : hipMemcpyAsync(dev[i], p, sz[i], hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
            p += sz[i];
        }
        return hipSuccess;
    }
    ~Snapshot() { if (buf) (void)hipFree(buf); }
};

static const char *objective_name(int o) { return o == MPPI_OBJ_CONTOUR ? "contour" : (o == MPPI_OBJ_TRACK ? "track" : "gate"); }

extern "C" {

mppi_status mppi_autotune(mppi_ctx *ctx, const double *d_req, int32_t reps, const char *cache_path, int32_t flags,
                          mppi_tune_result *out)
{
    if (!ctx) return fail(nullptr, MPPI_E_INVAL, "ctx is NULL");
    if (!d_req || reps < 1) return fail(ctx, MPPI_E_INVAL, "a request and reps >= 1 are required");
    if (ctx->external_ws) return fail(ctx, MPPI_E_INVAL, "context has no workspace of its own (server context)");
    ctx->err.clear();
    mppi_tune_result r{};
    if (!can_regen(ctx->args)) {
        // one choice only: the stored average
        ctx->args.regen = 0;
        if (out) *out = r;
        return MPPI_OK;
    }
    char key[256];
    snprintf(key, sizeof key, "ctx|%s|%s|%s|K%d|N%d|w%d", tune::arch_of(ctx->device).c_str(),
             objective_name(ctx->objective), tune::prec_name(ctx->fp64), tune::bucket(ctx->K), tune::bucket(ctx->N),
             ctx->args.rollout_waves);
    tune::Entry e;
    if (!(flags & MPPI_TUNE_FORCE) && tune::load(cache_path, key, e)) {
        ctx->args.regen = e.regen ? 1 : 0;
        r.regen_average = ctx->args.regen;
        r.from_cache = 1;
        (ctx->args.regen ? r.ms_regen : r.ms_stored) = e.ms;
        if (out) *out = r;
        return MPPI_OK;
    }
    Snapshot snap;
    HIP_TRY(ctx, snap.take(ctx->args, ctx->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(ctx, hipEventCreate(&e0));
    // the timed solves stay out of the per-kernel profile
    const bool profiling = ctx->profiling;
    ctx->profiling = false;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, MPPI_E_DEVICE, "hipEventCreate failed");
    }
    const int keep = ctx->args.regen;
    double ms[2] = {0.0, 0.0};
    mppi_status st = MPPI_OK;
    for (int g = 0; g < 2 && st == MPPI_OK; ++g) {
        ctx->args.regen = g;
        KArgs a = ctx->args;
        a.req = d_req;
        a.u0_out = nullptr;
        if ((st = launch_iterations(ctx, a)) != MPPI_OK) break;  // warm-up
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(ctx, MPPI_E_DEVICE, "event record failed"); break; }
        for (int i = 0; i < reps && st == MPPI_OK; ++i) st = launch_iterations(ctx, a);
        if (st != MPPI_OK) break;
        float t = 0.0f;
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            st = fail(ctx, MPPI_E_DEVICE, "timing the candidates failed");
            break;
        }
        ms[g] = t / reps;
        if (snap.restore(ctx->args, ctx->stream) != hipSuccess) st = fail(ctx, MPPI_E_DEVICE, "restore failed");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profiling = profiling;
    if (st != MPPI_OK) {
        ctx->args.regen = keep;
        (void)snap.restore(ctx->args, ctx->stream);
        (void)hipStreamSynchronize(ctx->stream);
        return st;
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->args.regen = ms[1] < ms[0] ? 1 : 0;
    r.regen_average = ctx->args.regen;
    r.ms_stored = ms[0];
    r.ms_regen = ms[1];
    e.regen = ctx->args.regen;
    e.ms = ms[ctx->args.regen];
    e.waves = ctx->args.rollout_waves;
    if (!tune::store(cache_path, key, e))
        return fail(ctx, MPPI_E_INVAL, "cannot write the autotuner cache %s", cache_path);
    if (out) *out = r;
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
    out->vtheta = w.vtheta;
    return MPPI_OK;
}

mppi_status mppi_set_warm(mppi_ctx *ctx, const mppi_warm *in)
{
    if (!ctx || !in) return fail(ctx, MPPI_E_INVAL, "ctx and in are required");
    if (in->N != ctx->N) return fail(ctx, MPPI_E_INVAL, "warm state has N=%d, context N=%d", in->N, ctx->N);
    if (ctx->objective == MPPI_OBJ_GATE && (in->g0 < 0 || in->g0 >= ctx->G))
        return fail(ctx, MPPI_E_INVAL, "g0=%d outside [0, %d)", in->g0, ctx->G);
    if (!finite_all(in->U, 4 * ctx->N) || !finite_all(in->V, ctx->N) || !finite_all(in->x_prev, 13) ||
        !isfinite(in->t_prev) || !isfinite(in->theta0) || !isfinite(in->vtheta))
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
    w.vtheta = in->vtheta;
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

mppi_status mppi_plant_step_rate(const mppi_quad *quad, const double x[17], const double tdot[4], double dt,
                                 int32_t substeps, double x_out[17])
{
    if (!quad || !x || !tdot || !x_out || substeps < 1 || !(dt > 0.0))
        return fail(nullptr, MPPI_E_INVAL, "invalid plant step arguments");
    double s[17], k1[17], k2[17], k3[17], k4[17], t[17], r[4];
    memcpy(s, x, sizeof s);
    const double h = dt / substeps;
    for (int n = 0; n < substeps; ++n) {
        // the rotors saturate: a rate may not carry a thrust past its bounds
        for (int i = 0; i < 4; ++i) {
            const double lo = (quad->t_min - s[13 + i]) / h, hi = (quad->t_max - s[13 + i]) / h;
            r[i] = tdot[i] < lo ? lo : (tdot[i] > hi ? hi : tdot[i]);
        }
        plant_deriv(quad, s, s + 13, k1);
        for (int i = 0; i < 4; ++i) k1[13 + i] = r[i];
        for (int i = 0; i < 17; ++i) t[i] = s[i] + 0.5 * h * k1[i];
        plant_deriv(quad, t, t + 13, k2);
        for (int i = 0; i < 4; ++i) k2[13 + i] = r[i];
        for (int i = 0; i < 17; ++i) t[i] = s[i] + 0.5 * h * k2[i];
        plant_deriv(quad, t, t + 13, k3);
        for (int i = 0; i < 4; ++i) k3[13 + i] = r[i];
        for (int i = 0; i < 17; ++i) t[i] = s[i] + h * k3[i];
        plant_deriv(quad, t, t + 13, k4);
        for (int i = 0; i < 4; ++i) k4[13 + i] = r[i];
        for (int i = 0; i < 17; ++i) s[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        const double nq = sqrt(s[6] * s[6] + s[7] * s[7] + s[8] * s[8] + s[9] * s[9]);
        for (int i = 6; i < 10; ++i) s[i] /= nq;
    }
    memcpy(x_out, s, sizeof s);
    return MPPI_OK;
}

}  // extern "C"

// ===================================================================== batches

namespace {

struct BatchGroup {
    int objective = 0;
    bool acc64 = false;
    std::vector<int> regs;       // registered contexts of this group
    int cap = 0;                 // = regs.size()
    size_t bytes = 0;
    void *d_block = nullptr;     // BatchDesc, items[cap], 3 x prefix[cap + 1]
    void *h_block = nullptr;     // pinned mirror
    BArgs bargs{};
    BatchLaunch launch{};
    int active = 0;              // items in the current step
    bool ctrl = false;           // a context of the group adds the control-cost term
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct mppi_batch {
    std::vector<mppi_ctx *> ctxs;
    std::vector<int> group_of, tiles_of;
    bool fp64 = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    KArgs *d_table = nullptr;
    std::vector<KArgs> h_table;  // host copy of d_table
    std::vector<BatchGroup> groups;
    mppi_batch_cfg cfg{};
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipEvent_t copy_done = nullptr;
    bool copy_pending = false;
    int n_cu = 256;
    int total_tiles = 0;
    bool has_rate = false;       // a context takes the rate input: one-wave rollouts only
    bool any_ctrl = false;       // a context adds the control-cost term: the tensor is kept
    int n_iter = 1;              // MPPI iterations per step, shared by the contexts
    std::string err;
};

static mppi_status bfail(mppi_batch *b, mppi_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
static mppi_status bfail(mppi_batch *b, mppi_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_create_err = buf;
    return s;
}

#define BHIP_TRY(b, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return bfail((b), MPPI_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

static void drop_graph(mppi_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Resolve automatic fields of the launch shape for this batch.
static hipError_t resolve_cfg(mppi_batch *b)
{
    mppi_batch_cfg &c = b->cfg;
    int waves = c.rollout_waves;
    const int cu = b->n_cu, tiles = b->total_tiles;
    if (waves < 1 || waves > 4) waves = tiles <= cu ? 4 : (tiles <= 2 * cu ? (b->fp64 ? 2 : 4) : 1);
    // a rate sample follows its thrust chain, which the sample kernel walks
    // per sample: the one-wave rollout reads it
    if (b->has_rate) waves = 1;
    // the regenerating average where the batch's rollout draws the samples,
    // unless a context's control-cost term reads the sample tensor
    const int regen = (c.regen_average && waves >= 3 && !b->any_ctrl) ? 1 : 0;
    bool changed = false;
    for (auto &t : b->h_table)
        if (t.regen != regen) { t.regen = regen; changed = true; }
    if (changed && b->d_table) {
        const hipError_t e = hipMemcpy(b->d_table, b->h_table.data(), sizeof(KArgs) * b->h_table.size(),
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
    }
    // four-wave chunk: the contexts' own when they all agree (a served solve
    // then runs exactly its stand-alone kernel), else by the batch's tiles
    int ring = b->ctxs[0]->args.ring4_b;
    for (const mppi_ctx *x : b->ctxs)
        if (x->args.ring4_b != ring) ring = 0;
    if (ring == 0) ring = (!b->fp64 && tiles <= cu) ? 4 : 2;
    // persistent rollout workgroups: what fits one CU times the CUs (one
    // four-wave workgroup with 4-step chunks or in binary64, two with 2-step
    // chunks in binary32, one three-wave, two two-wave, eight one-wave)
    int per_cu = 8;
    if (waves == 4) per_cu = (!b->fp64 && ring == 2) ? 2 : 1;
    else if (waves == 3) per_cu = 1;
    else if (waves == 2) per_cu = 2;
    int rg = c.rollout_groups > 0 ? c.rollout_groups : per_cu * cu;
    int sg = c.sample_groups > 0 ? c.sample_groups : 4 * b->n_cu;
    for (auto &g : b->groups) {
        g.launch.objective = g.objective;
        g.launch.fp64 = b->fp64;
        g.launch.acc64 = g.acc64;
        g.launch.rollout_waves = waves;
        g.launch.ring4_b = ring;
        g.launch.rollout_groups = rg;
        g.launch.sample_groups = sg;
        // kFinalThreads-thread workgroups, two per CU
        g.launch.final_groups = 2 * b->n_cu;
        // one-wave workgroups of the control-cost term, eight per CU
        g.launch.ctrl_groups = g.ctrl ? 8 * b->n_cu : 0;
    }
    return hipSuccess;
}

static void release_batch(mppi_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (auto &g : b->groups) {
        if (g.d_block) (void)hipFree(g.d_block);
        if (g.h_block) (void)hipHostFree(g.h_block);
    }
    if (b->d_table) (void)hipFree(b->d_table);
    if (b->copy_done) (void)hipEventDestroy(b->copy_done);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

extern "C" {

const char *mppi_batch_last_error(const mppi_batch *b) { return b ? b->err.c_str() : g_create_err.c_str(); }

void mppi_batch_destroy(mppi_batch *b) { release_batch(b); }

mppi_status mppi_batch_create(mppi_ctx *const *ctxs, int32_t n, void *stream, const mppi_batch_cfg *cfg,
                              mppi_batch **out)
{
    if (!out) return bfail(nullptr, MPPI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1) return bfail(nullptr, MPPI_E_INVAL, "a batch needs at least one context");
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return bfail(nullptr, MPPI_E_INVAL, "context %d is NULL", i);
        if (ctxs[i]->fp64 != ctxs[0]->fp64) return bfail(nullptr, MPPI_E_INVAL, "contexts differ in precision");
        if (ctxs[i]->n_iter != ctxs[0]->n_iter)
            return bfail(nullptr, MPPI_E_INVAL, "context %d: the contexts of a batch share n_iter", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return bfail(nullptr, MPPI_E_INVAL, "context %d registered twice", i);
    }
    mppi_batch *b = new (std::nothrow) mppi_batch();
    if (!b) return bfail(nullptr, MPPI_E_NOMEM, "host allocation failed");
    b->ctxs.assign(ctxs, ctxs + n);
    b->fp64 = ctxs[0]->fp64;
    for (int i = 0; i < n; ++i) {
        b->has_rate = b->has_rate || ctxs[i]->args.input_model == MPPI_INPUT_RATE;
        b->any_ctrl = b->any_ctrl || ctxs[i]->args.ctrl_cost != 0.0;
    }
    b->n_iter = ctxs[0]->n_iter;
    b->cfg = cfg ? *cfg : mppi_batch_cfg{0, 0, 0, 1, 0};
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (b->n_cu < 1) b->n_cu = 256;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            release_batch(b);
            return bfail(nullptr, MPPI_E_DEVICE, "hipStreamCreateWithFlags failed");
        }
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->copy_done, hipEventDisableTiming) != hipSuccess) {
        release_batch(b);
        return bfail(nullptr, MPPI_E_DEVICE, "hipEventCreate failed");
    }
    // groups by (objective, accumulation type)
    b->group_of.resize(n);
    b->tiles_of.resize(n);
    for (int i = 0; i < n; ++i) {
        const mppi_ctx *c = ctxs[i];
        int gi = -1;
        for (size_t g = 0; g < b->groups.size(); ++g)
            if (b->groups[g].objective == c->objective && b->groups[g].acc64 == c->acc64) gi = (int)g;
        if (gi < 0) {
            b->groups.emplace_back();
            b->groups.back().objective = c->objective;
            b->groups.back().acc64 = c->acc64;
            gi = (int)b->groups.size() - 1;
        }
        b->groups[gi].regs.push_back(i);
        b->groups[gi].ctrl = b->groups[gi].ctrl || c->args.ctrl_cost != 0.0;
        b->group_of[i] = gi;
        b->tiles_of[i] = (c->K + 1 + 63) / 64;
        b->total_tiles += b->tiles_of[i];
    }
    // device table of kernel arguments; whether the average draws the samples
    // again is the batch's choice (its layout is its own).  With several
    // iterations per step a second copy, marked inner, serves the later ones.
    std::vector<KArgs> &table = b->h_table;
    const int copies = b->n_iter > 1 ? 2 : 1;
    table.resize((size_t)copies * n);
    for (int i = 0; i < n; ++i) {
        table[i] = ctxs[i]->args;
        table[i].regen = 0;
        table[i].inner = 0;
        if (copies == 2) {
            table[n + i] = table[i];
            table[n + i].inner = 1;
        }
    }
    if (hipMalloc((void **)&b->d_table, sizeof(KArgs) * table.size()) != hipSuccess ||
        hipMemcpy(b->d_table, table.data(), sizeof(KArgs) * table.size(), hipMemcpyHostToDevice) != hipSuccess) {
        release_batch(b);
        return bfail(nullptr, MPPI_E_NOMEM, "device table allocation failed");
    }
    for (auto &g : b->groups) {
        g.cap = (int)g.regs.size();
        const size_t o_items = align_up(sizeof(BatchDesc), 64);
        const size_t o_sp = align_up(o_items + sizeof(BatchItem) * g.cap, 64);
        const size_t o_tp = align_up(o_sp + sizeof(int32_t) * (g.cap + 1), 64);
        const size_t o_ap = align_up(o_tp + sizeof(int32_t) * (g.cap + 1), 64);
        g.bytes = align_up(o_ap + sizeof(int32_t) * (g.cap + 1), 64);
        if (hipMalloc(&g.d_block, g.bytes) != hipSuccess || hipHostMalloc(&g.h_block, g.bytes, 0) != hipSuccess) {
            release_batch(b);
            return bfail(nullptr, MPPI_E_NOMEM, "batch descriptor allocation failed");
        }
        memset(g.h_block, 0, g.bytes);
        char *d = (char *)g.d_block;
        g.bargs.table = b->d_table;
        g.bargs.desc = (BatchDesc *)d;
        g.bargs.items = (const BatchItem *)(d + o_items);
        g.bargs.sample_prefix = (const int32_t *)(d + o_sp);
        g.bargs.tile_prefix = (const int32_t *)(d + o_tp);
        g.bargs.step_prefix = (const int32_t *)(d + o_ap);
    }
    if (resolve_cfg(b) != hipSuccess) {
        release_batch(b);
        return bfail(nullptr, MPPI_E_DEVICE, "upload of the kernel-argument table failed");
    }
    *out = b;
    return MPPI_OK;
}

mppi_status mppi_batch_set_cfg(mppi_batch *b, const mppi_batch_cfg *cfg)
{
    if (!b || !cfg) return bfail(b, MPPI_E_INVAL, "batch and cfg are required");
    if (cfg->rollout_waves < 0 || cfg->rollout_waves > 4 || cfg->rollout_groups < 0 || cfg->sample_groups < 0)
        return bfail(b, MPPI_E_INVAL, "invalid launch shape");
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    b->cfg = *cfg;
    BHIP_TRY(b, resolve_cfg(b));
    return MPPI_OK;
}

mppi_status mppi_batch_get_cfg(const mppi_batch *b, mppi_batch_cfg *cfg)
{
    if (!b || !cfg) return MPPI_E_INVAL;
    *cfg = b->cfg;
    if (!b->h_table.empty()) cfg->regen_average = b->h_table[0].regen;
    if (!b->groups.empty()) {
        cfg->rollout_waves = b->groups[0].launch.rollout_waves;
        cfg->rollout_groups = b->groups[0].launch.rollout_groups;
        cfg->sample_groups = b->groups[0].launch.sample_groups;
    }
    return MPPI_OK;
}

// The launch sequence of one step: n_iter iterations, the later ones reading
// the inner copy of the argument table (no shift, the first iteration's last
// applied input), each group's kernels in turn.
static mppi_status enqueue_groups(mppi_batch *b, bool skip_empty)
{
    for (int it = 0; it < b->n_iter; ++it) {
        for (auto &g : b->groups) {
            if (skip_empty && g.active == 0) continue;
            BArgs ba = g.bargs;
            if (it > 0) ba.table = b->d_table + b->ctxs.size();
            BHIP_TRY(b, launch_batch(ba, g.launch, b->stream));
        }
    }
    return MPPI_OK;
}

}  // extern "C"

// One batched step; ws (optional, n_active entries) lends each solve its
// workspace when its context has none of its own.
static mppi_status batch_solve(mppi_batch *b, const int32_t *active, int32_t n_active, const double *d_reqs,
                               double *d_u0s, char *const *ws)
{
    if (!b) return bfail(nullptr, MPPI_E_INVAL, "batch is NULL");
    const int n = (int)b->ctxs.size();
    if (!d_reqs) return bfail(b, MPPI_E_INVAL, "d_reqs is NULL");
    if (active == nullptr && n_active != n) return bfail(b, MPPI_E_INVAL, "NULL active list needs n_active = n");
    if (n_active < 0 || n_active > n) return bfail(b, MPPI_E_INVAL, "n_active=%d outside [0, %d]", n_active, n);
    std::vector<char> seen(n, 0);
    for (auto &g : b->groups) g.active = 0;
    std::vector<std::vector<std::pair<int, int>>> per(b->groups.size());  // (registered index, slot)
    for (int i = 0; i < n_active; ++i) {
        const int r = active ? active[i] : i;
        if (r < 0 || r >= n) return bfail(b, MPPI_E_INVAL, "active[%d]=%d outside [0, %d)", i, r, n);
        if (seen[r]) return bfail(b, MPPI_E_INVAL, "context %d listed twice", r);
        if (b->ctxs[r]->external_ws && !(ws && ws[i]))
            return bfail(b, MPPI_E_INVAL, "context %d has no workspace and none was lent", r);
        seen[r] = 1;
        per[b->group_of[r]].push_back({r, i});
    }
    for (int r = 0; r < n; ++r)
        if (seen[r]) b->ctxs[r]->no_tensor = b->h_table[r].regen != 0;
    // the previous step's descriptor copy must have left the pinned buffers
    if (b->copy_pending) BHIP_TRY(b, hipEventSynchronize(b->copy_done));
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        BatchGroup &g = b->groups[gi];
        auto &lst = per[gi];
        // longest horizon first (tile order of the persistent rollout), ties by registration
        std::stable_sort(lst.begin(), lst.end(), [&](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            return b->ctxs[x.first]->N > b->ctxs[y.first]->N;
        });
        char *h = (char *)g.h_block;
        const char *d = (const char *)g.d_block;
        BatchDesc *desc = (BatchDesc *)h;
        BatchItem *items = (BatchItem *)(h + ((const char *)g.bargs.items - d));
        int32_t *sp = (int32_t *)(h + ((const char *)g.bargs.sample_prefix - d));
        int32_t *tp = (int32_t *)(h + ((const char *)g.bargs.tile_prefix - d));
        int32_t *ap = (int32_t *)(h + ((const char *)g.bargs.step_prefix - d));
        int64_t s_units = 0, t_units = 0, a_units = 0;
        sp[0] = tp[0] = ap[0] = 0;
        for (size_t j = 0; j < lst.size(); ++j) {
            const mppi_ctx *c = b->ctxs[lst[j].first];
            items[j].ctx = lst[j].first;
            items[j].pad = 0;
            items[j].req = d_reqs + (size_t)kReqDoubles * lst[j].second;
            items[j].u0_out = d_u0s ? d_u0s + 4 * (size_t)lst[j].second : nullptr;
            items[j].ws = ws ? ws[lst[j].second] : nullptr;
            s_units += (c->K + 1 + 255) / 256;
            t_units += (c->K + 1 + 63) / 64;
            a_units += c->N;
            if (s_units > INT32_MAX || a_units > INT32_MAX) return bfail(b, MPPI_E_INVAL, "batch too large");
            sp[j + 1] = (int32_t)s_units;
            tp[j + 1] = (int32_t)t_units;
            ap[j + 1] = (int32_t)a_units;
        }
        desc->n = (int32_t)lst.size();
        desc->n_sample_units = (int32_t)s_units;
        desc->n_tiles = (int32_t)t_units;
        desc->n_steps = (int32_t)a_units;
        desc->queue = 0u;
        desc->sample_queue = 0u;
        g.active = (int)lst.size();
        BHIP_TRY(b, hipMemcpyAsync(g.d_block, g.h_block, g.bytes, hipMemcpyHostToDevice, b->stream));
    }
    BHIP_TRY(b, hipEventRecord(b->copy_done, b->stream));
    b->copy_pending = true;
    if (b->cfg.use_graph) {
        if (!b->exec) {
            BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            mppi_status st = enqueue_groups(b, false);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &graph);
            if (st != MPPI_OK) { if (graph) (void)hipGraphDestroy(graph); return st; }
            if (e != hipSuccess) return bfail(b, MPPI_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            b->graph = graph;
            BHIP_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        }
        BHIP_TRY(b, hipGraphLaunch(b->exec, b->stream));
        return MPPI_OK;
    }
    return enqueue_groups(b, true);
}

extern "C" {

mppi_status mppi_batch_solve_device(mppi_batch *b, const int32_t *active, int32_t n_active, const double *d_reqs,
                                    double *d_u0s)
{
    return batch_solve(b, active, n_active, d_reqs, d_u0s, nullptr);
}

mppi_status mppi_batch_autotune(mppi_batch *b, const double *d_reqs, double *d_u0s, int32_t reps,
                                const char *cache_path, int32_t flags, mppi_batch_cfg *best, double *best_ms,
                                int32_t *from_cache)
{
    if (!b || !d_reqs || reps < 1) return bfail(b, MPPI_E_INVAL, "batch, requests and reps >= 1 are required");
    const int n = (int)b->ctxs.size();
    if (from_cache) *from_cache = 0;
    // cache key: architecture, objectives, precision, instance count and
    // total rollout steps; then the rate input, several iterations and the
    // control-cost term where a context has them
    int objs = 0;
    double kn = 0.0;
    for (const mppi_ctx *c : b->ctxs) {
        objs |= 1 << c->objective;
        kn += (double)c->K * (double)c->N;
    }
    char key[256];
    snprintf(key, sizeof key, "batch|%s|obj%d|%s|n%d|KN%d%s%s", tune::arch_of(b->ctxs[0]->device).c_str(), objs,
             tune::prec_name(b->fp64), tune::bucket(n), tune::bucket(kn), b->has_rate ? "|rate" : "",
             b->any_ctrl ? "|cc" : "");
    if (b->n_iter > 1) {
        const size_t used = strlen(key);
        snprintf(key + used, sizeof key - used, "|it%d", b->n_iter);
    }
    tune::Entry ce;
    if (!(flags & MPPI_TUNE_FORCE) && tune::load(cache_path, key, ce)) {
        const mppi_batch_cfg c{ce.waves, ce.groups, ce.sgroups, b->cfg.use_graph, ce.regen};
        const mppi_status st = mppi_batch_set_cfg(b, &c);
        if (st != MPPI_OK) return st;
        if (best) *best = c;
        if (best_ms) *best_ms = ce.ms;
        if (from_cache) *from_cache = 1;
        return MPPI_OK;
    }
    const mppi_batch_cfg saved = b->cfg;
    std::vector<mppi_batch_cfg> cand;
    const int cu = b->n_cu;
    for (int waves = 1; waves <= (b->has_rate ? 1 : 4); ++waves) {
        const int rg_mult[] = {1, 2, 4, 8};
        for (int rm : rg_mult) {
            if (waves >= 2 && rm > 2) continue;  // one or two LDS rings fit one CU
            for (int sm : {1, 4})
                for (int regen = 0; regen <= (waves >= 3 && !b->any_ctrl ? 1 : 0); ++regen)
                    cand.push_back(mppi_batch_cfg{waves, rm * cu, sm * cu, saved.use_graph, regen});
        }
    }
    // the timed steps are real solves: every context's state is put back after
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    std::vector<Snapshot> snaps(n);
    for (int i = 0; i < n; ++i) BHIP_TRY(b, snaps[i].take(b->ctxs[i]->args, b->stream));
    auto restore_all = [&]() -> hipError_t {
        for (int i = 0; i < n; ++i) {
            const hipError_t e = snaps[i].restore(b->ctxs[i]->args, b->stream);
            if (e != hipSuccess) return e;
        }
        return hipStreamSynchronize(b->stream);
    };
    hipEvent_t e0, e1;
    BHIP_TRY(b, hipEventCreate(&e0));
    BHIP_TRY(b, hipEventCreate(&e1));
    double best_t = 1e300;
    mppi_batch_cfg best_c = saved;
    mppi_status st = MPPI_OK;
    for (const auto &c : cand) {
        if ((st = mppi_batch_set_cfg(b, &c)) != MPPI_OK) break;
        if ((st = mppi_batch_solve_device(b, nullptr, n, d_reqs, d_u0s)) != MPPI_OK) break;  // capture + warm-up
        if (hipEventRecord(e0, b->stream) != hipSuccess) { st = MPPI_E_DEVICE; break; }
        for (int r = 0; r < reps && st == MPPI_OK; ++r) st = mppi_batch_solve_device(b, nullptr, n, d_reqs, d_u0s);
        if (st != MPPI_OK) break;
        if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = MPPI_E_DEVICE;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double t = ms / reps;
        if (t < best_t) { best_t = t; best_c = c; }
        if (restore_all() != hipSuccess) { st = MPPI_E_DEVICE; break; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MPPI_OK) {
        (void)mppi_batch_set_cfg(b, &saved);
        (void)restore_all();
        return st;
    }
    if ((st = mppi_batch_set_cfg(b, &best_c)) != MPPI_OK) return st;
    tune::Entry e;
    e.waves = best_c.rollout_waves;
    e.groups = best_c.rollout_groups;
    e.sgroups = best_c.sample_groups;
    e.regen = best_c.regen_average;
    e.ms = best_t;
    if (!tune::store(cache_path, key, e))
        return bfail(b, MPPI_E_INVAL, "cannot write the autotuner cache %s", cache_path);
    if (best) *best = best_c;
    if (best_ms) *best_ms = best_t;
    return MPPI_OK;
}

}  // extern "C"

// ===================================================================== server

namespace {

// First-fit allocator over one device arena (offsets, 256-byte granules).
struct Arena {
    size_t size = 0;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, bytes), sorted by offset
    size_t in_use = 0, peak = 0;

    void reset(size_t n)
    {
        size = n;
        free_list.assign(1, {0, n});
        in_use = peak = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes, 256);
        for (size_t i = 0; i < free_list.size(); ++i) {
            if (free_list[i].second >= bytes) {
                *off = free_list[i].first;
                free_list[i].first += bytes;
                free_list[i].second -= bytes;
                if (free_list[i].second == 0) free_list.erase(free_list.begin() + (long)i);
                in_use += bytes;
                if (in_use > peak) peak = in_use;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes, 256);
        in_use -= bytes;
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
        it = free_list.insert(it, {off, bytes});
        // merge with neighbours
        size_t i = (size_t)(it - free_list.begin());
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + (long)i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + (long)i);
        }
    }
};

struct Request {
    uint64_t ticket;
    double x0[17];              // 13 states, then the four thrusts of the rate input
    double t_now, t_arrival;
};

struct InFlight {
    int drone;
    uint64_t ticket;
    double t_arrival, t_launch;
    size_t ws_off;
};

struct Slot {
    std::vector<mppi_batch *> batches;           // one per layout class of the drones
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    double *h_req = nullptr, *d_req = nullptr;   // n x 16
    double *h_u0 = nullptr, *d_u0 = nullptr;     // n x 4
    std::vector<InFlight> flight;
    bool busy = false;
};

}  // namespace

struct mppi_server {
    std::vector<mppi_ctx *> drones;
    // Drones are grouped by rollout layout (waves, four-wave chunk) and
    // iterations per solve: a launch holds drones of one class only and runs
    // their own layout, so a served solve repeats the stand-alone solve bit
    // for bit and a one-wave class (the rate input) does not slow the others
    // down.
    std::vector<int> cls, local;                 // per drone: class, index in the class's batch
    mppi_server_cfg cfg{};
    std::vector<std::vector<Request>> queue;     // per drone, FIFO (front at index head[d])
    std::vector<size_t> head;
    std::vector<char> busy;
    std::vector<Slot> slots;
    char *arena_base = nullptr;
    Arena arena;
    std::vector<mppi_result> done;
    size_t done_head = 0;
    uint64_t next_ticket = 1;
    mppi_server_stats st{};
    std::string err;
};

static mppi_status sfail(mppi_server *s, mppi_status code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
static mppi_status sfail(mppi_server *s, mppi_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_create_err = buf;
    return code;
}

static void release_server(mppi_server *s)
{
    if (!s) return;
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        for (mppi_batch *b : sl.batches) release_batch(b);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_req) (void)hipHostFree(sl.h_req);
        if (sl.h_u0) (void)hipHostFree(sl.h_u0);
        if (sl.d_req) (void)hipFree(sl.d_req);
        if (sl.d_u0) (void)hipFree(sl.d_u0);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

// Retire finished launches of every busy slot (non-blocking unless wait).
static mppi_status retire(mppi_server *s, double now, bool wait)
{
    for (auto &sl : s->slots) {
        if (!sl.busy) continue;
        hipError_t q = wait ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return sfail(s, MPPI_E_DEVICE, "launch failed: %s", hipGetErrorString(q));
        for (size_t i = 0; i < sl.flight.size(); ++i) {
            const InFlight &f = sl.flight[i];
            mppi_result r{};
            r.ticket = f.ticket;
            r.drone = f.drone;
            bool finite = true;
            for (int c = 0; c < 4; ++c) {
                r.u0[c] = sl.h_u0[4 * i + c];
                finite = finite && isfinite(r.u0[c]);
            }
            r.status = finite ? MPPI_OK : MPPI_E_NONFINITE;
            r.t_arrival = f.t_arrival;
            r.t_launch = f.t_launch;
            r.t_done = now;
            s->done.push_back(r);
            s->busy[f.drone] = 0;
            s->arena.release(f.ws_off, s->drones[f.drone]->ws_bytes);
            s->st.completed += 1;
            s->st.rollout_steps += (double)s->drones[f.drone]->K * (double)s->drones[f.drone]->N;
        }
        s->st.in_flight -= (int64_t)sl.flight.size();
        sl.flight.clear();
        sl.busy = false;
    }
    return MPPI_OK;
}

// Admit queued heads into idle slots and launch them.
static mppi_status admit(mppi_server *s, double now, int32_t *n_launched)
{
    const int nd = (int)s->drones.size();
    for (auto &sl : s->slots) {
        if (sl.busy) continue;
        // ready drones, oldest head first
        std::vector<int> ready;
        for (int d = 0; d < nd; ++d)
            if (!s->busy[d] && s->head[d] < s->queue[d].size()) ready.push_back(d);
        if (ready.empty()) return MPPI_OK;
        std::stable_sort(ready.begin(), ready.end(), [&](int x, int y) {
            return s->queue[x][s->head[x]].t_arrival < s->queue[y][s->head[y]].t_arrival;
        });
        // the launch takes the class of the oldest head
        const int c = s->cls[ready[0]];
        std::vector<int32_t> active;
        std::vector<char *> ws;
        for (int d : ready) {
            if (s->cfg.max_batch > 0 && (int)active.size() >= s->cfg.max_batch) break;
            if (s->cls[d] != c) continue;
            size_t off = 0;
            if (!s->arena.alloc(s->drones[d]->ws_bytes, &off)) continue;  // waits for memory
            const Request &rq = s->queue[d][s->head[d]];
            const int i = (int)active.size();
            for (int c = 0; c < 13; ++c) sl.h_req[kReqDoubles * i + c] = rq.x0[c];
            sl.h_req[kReqDoubles * i + 13] = rq.t_now;
            for (int c = 0; c < 4; ++c) sl.h_req[kReqDoubles * i + kReqThrust + c] = rq.x0[13 + c];
            active.push_back(s->local[d]);
            ws.push_back(s->arena_base + off);
            sl.flight.push_back(InFlight{d, rq.ticket, rq.t_arrival, now, off});
            s->busy[d] = 1;
            s->head[d] += 1;
            if (s->head[d] == s->queue[d].size()) { s->queue[d].clear(); s->head[d] = 0; }
        }
        if (active.empty()) return MPPI_OK;  // nothing fits the free memory now
        const int n = (int)active.size();
        if (s->arena.in_use > s->st.peak_bytes_in_flight) s->st.peak_bytes_in_flight = (double)s->arena.in_use;
        if (hipMemcpyAsync(sl.d_req, sl.h_req, sizeof(double) * kReqDoubles * n, hipMemcpyHostToDevice, sl.stream) !=
            hipSuccess)
            return sfail(s, MPPI_E_DEVICE, "request copy failed");
        mppi_status st = batch_solve(sl.batches[c], active.data(), n, sl.d_req, sl.d_u0, ws.data());
        if (st != MPPI_OK) return sfail(s, st, "batch launch failed: %s", sl.batches[c]->err.c_str());
        if (hipMemcpyAsync(sl.h_u0, sl.d_u0, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
            hipEventRecord(sl.done, sl.stream) != hipSuccess)
            return sfail(s, MPPI_E_DEVICE, "result copy failed");
        sl.busy = true;
        s->st.launches += 1;
        s->st.queued -= n;
        s->st.in_flight += n;
        if (n_launched) *n_launched += 1;
    }
    return MPPI_OK;
}

extern "C" {

const char *mppi_server_last_error(const mppi_server *s) { return s ? s->err.c_str() : g_create_err.c_str(); }

void mppi_server_destroy(mppi_server *s) { release_server(s); }

mppi_status mppi_server_create(mppi_ctx *const *drones, int32_t n, const mppi_server_cfg *cfg, mppi_server **out)
{
    if (!out) return sfail(nullptr, MPPI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!drones || n < 1 || !cfg) return sfail(nullptr, MPPI_E_INVAL, "drones and cfg are required");
    if (!(cfg->budget_bytes > 0.0) || cfg->n_slots < 1 || cfg->n_slots > 16 || cfg->max_batch < 0)
        return sfail(nullptr, MPPI_E_INVAL, "invalid server configuration");
    for (int i = 0; i < n; ++i) {
        if (!drones[i] || !drones[i]->external_ws)
            return sfail(nullptr, MPPI_E_INVAL, "drone %d: context must be created with MPPI_FLAG_EXTERNAL_WORKSPACE", i);
    }
    mppi_server *s = new (std::nothrow) mppi_server();
    if (!s) return sfail(nullptr, MPPI_E_NOMEM, "host allocation failed");
    s->drones.assign(drones, drones + n);
    s->cfg = *cfg;
    s->queue.resize(n);
    s->head.assign(n, 0);
    s->busy.assign(n, 0);
    // launch classes (rollout layout, iterations per solve) in order of
    // first appearance
    std::vector<int> cls_key, cls_waves;
    std::vector<std::vector<mppi_ctx *>> members;
    s->cls.resize(n);
    s->local.resize(n);
    for (int i = 0; i < n; ++i) {
        const int key = (8 * drones[i]->args.rollout_waves + drones[i]->args.ring4_b) * 128 + drones[i]->n_iter;
        int c = 0;
        while (c < (int)cls_key.size() && cls_key[c] != key) ++c;
        if (c == (int)cls_key.size()) {
            cls_key.push_back(key);
            cls_waves.push_back(drones[i]->args.rollout_waves);
            members.emplace_back();
        }
        s->cls[i] = c;
        s->local[i] = (int)members[c].size();
        members[c].push_back(drones[i]);
    }
    const size_t arena = (size_t)cfg->budget_bytes;
    if (hipMalloc((void **)&s->arena_base, arena) != hipSuccess) {
        release_server(s);
        return sfail(nullptr, MPPI_E_NOMEM, "arena of %zu bytes could not be allocated", arena);
    }
    s->arena.reset(arena);
    s->st.arena_bytes = (double)arena;
    s->slots.resize(cfg->n_slots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_req, sizeof(double) * kReqDoubles * n, 0) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_u0, sizeof(double) * 4 * n, 0) != hipSuccess ||
            hipMalloc((void **)&sl.d_req, sizeof(double) * kReqDoubles * n) != hipSuccess ||
            hipMalloc((void **)&sl.d_u0, sizeof(double) * 4 * n) != hipSuccess) {
            release_server(s);
            return sfail(nullptr, MPPI_E_NOMEM, "slot resources could not be allocated");
        }
        // one batch per class, in the class's own rollout layout
        for (size_t c = 0; c < members.size(); ++c) {
            mppi_batch_cfg bc{cls_waves[c], 0, 0, cfg->use_graph ? 1 : 0};
            mppi_batch *bt = nullptr;
            mppi_status st = mppi_batch_create(members[c].data(), (int32_t)members[c].size(), sl.stream, &bc, &bt);
            if (st != MPPI_OK) {
                std::string e = g_create_err;
                release_server(s);
                return sfail(nullptr, st, "slot batch: %s", e.c_str());
            }
            sl.batches.push_back(bt);
        }
    }
    *out = s;
    return MPPI_OK;
}

mppi_status mppi_server_submit(mppi_server *s, int32_t drone, const double *x0, double t_now, double t_arrival,
                               uint64_t *ticket)
{
    if (!s || !x0) return sfail(s, MPPI_E_INVAL, "server and x0 are required");
    if (drone < 0 || drone >= (int)s->drones.size()) return sfail(s, MPPI_E_INVAL, "drone %d out of range", drone);
    const int nx = s->drones[drone]->args.input_model == MPPI_INPUT_RATE ? 17 : 13;
    if (!finite_all(x0, nx) || !isfinite(t_now)) return sfail(s, MPPI_E_INVAL, "x0 and t_now must be finite");
    const double qn = x0[6] * x0[6] + x0[7] * x0[7] + x0[8] * x0[8] + x0[9] * x0[9];
    if (!(qn > 0.0)) return sfail(s, MPPI_E_INVAL, "quaternion of x0 has zero norm");
    if (align_up(s->drones[drone]->ws_bytes, 256) > s->arena.size)
        return sfail(s, MPPI_E_NOMEM, "drone %d needs %zu workspace bytes, the arena has %zu", drone,
                     s->drones[drone]->ws_bytes, s->arena.size);
    Request r;
    r.ticket = s->next_ticket++;
    memset(r.x0, 0, sizeof r.x0);
    memcpy(r.x0, x0, sizeof(double) * nx);
    r.t_now = t_now;
    r.t_arrival = t_arrival;
    s->queue[drone].push_back(r);
    s->st.submitted += 1;
    s->st.queued += 1;
    if (ticket) *ticket = r.ticket;
    return MPPI_OK;
}

mppi_status mppi_server_progress(mppi_server *s, double now, int32_t *n_launched)
{
    if (!s) return sfail(nullptr, MPPI_E_INVAL, "server is NULL");
    if (n_launched) *n_launched = 0;
    mppi_status st = retire(s, now, false);
    if (st != MPPI_OK) return st;
    return admit(s, now, n_launched);
}

mppi_status mppi_server_drain(mppi_server *s, double now)
{
    if (!s) return sfail(nullptr, MPPI_E_INVAL, "server is NULL");
    for (;;) {
        mppi_status st = mppi_server_progress(s, now, nullptr);
        if (st != MPPI_OK) return st;
        if (s->st.queued == 0 && s->st.in_flight == 0) return MPPI_OK;
        if ((st = retire(s, now, true)) != MPPI_OK) return st;
    }
}

mppi_status mppi_server_poll(mppi_server *s, mppi_result *out, int32_t max, int32_t *n_out)
{
    if (!s || !n_out || (max > 0 && !out)) return sfail(s, MPPI_E_INVAL, "invalid poll arguments");
    int32_t k = 0;
    while (k < max && s->done_head < s->done.size()) out[k++] = s->done[s->done_head++];
    if (s->done_head == s->done.size()) { s->done.clear(); s->done_head = 0; }
    *n_out = k;
    return MPPI_OK;
}

mppi_status mppi_server_get_stats(const mppi_server *s, mppi_server_stats *out)
{
    if (!s || !out) return MPPI_E_INVAL;
    *out = s->st;
    return MPPI_OK;
}

}  // extern "C"
