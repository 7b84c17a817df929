/*
 * FP64 CPU oracle for one MPPI sampling step -- test infrastructure only.
 *
 * Plain, slow, obviously-correct C99.  Every function states the passage of
 * the paper it follows.  Where the paper is silent the reading taken is the
 * one listed in the project's design notes; the ones that shape the numbers
 * are repeated next to the code that implements them.
 *
 * Two input models: the four rotor thrusts (13 states), or the paper's thrust
 * rates with the thrusts as states (17 states, Sec. III-A).
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -fopenmp -ffp-contract=off
 * (no fast-math, no FMA contraction: the arithmetic is exactly what is written).
 */
#include "mppi_oracle.h"

#include <math.h>
#include <stddef.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11).  Round function: two 32x32->64 products of
 * counter words 0 and 2 with the published multipliers, the high halves
 * xored with the other two counter words and the key; key bumped by the
 * published Weyl constants between rounds.                                  */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)mul0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)mul1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += weyl0;
        k1 += weyl1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1): the top 23 bits of the word, centred in their cell,
 * i.e. (2*(w>>9)+1) * 2^-24.  The numerator has at most 24 significant bits,
 * so the value is exact in binary32 as well as binary64 and never 0 or 1. */
double orc_u01(uint32_t word)
{
    return (double)(2u * (word >> 9) + 1u) * (1.0 / 16777216.0);
}

/* Four standard normals for sample m, horizon step k, solve counter s and
 * channel block ch (0: rotor thrusts, 1: contouring progress speed).
 * Philox counter = (m, k, s, ch), key = (seed low word, seed high word).
 * Box-Muller (Box & Muller 1958): pairs (u0,u1) and (u2,u3),
 * z0 = r0 cos(2 pi u1), z1 = r0 sin(2 pi u1), r0 = sqrt(-2 ln u0), etc.     */
void orc_normals(uint64_t seed, uint32_t m, uint32_t k, uint32_t s, uint32_t ch, double z[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t ctr[4] = {m, k, s, ch};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u0 = orc_u01(w[0]), u1 = orc_u01(w[1]);
    double u2 = orc_u01(w[2]), u3 = orc_u01(w[3]);
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    z[0] = r0 * cos(two_pi * u1);
    z[1] = r0 * sin(two_pi * u1);
    z[2] = r1 * cos(two_pi * u3);
    z[3] = r1 * sin(two_pi * u3);
}

/* ------------------------------------------------------------------------ */
/* Dynamics, Sec. III-A, Eq. (2).  State x = [p(3), v(3), q(4), w(3)] with the
 * quaternion q = (qw, qx, qy, qz), Hamilton convention, body-to-world, driven
 * by the four rotor thrusts T: the input of the thrust model, or four more
 * states whose derivatives are the input in the paper's rate model.        */

static void rot_matrix(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

void orc_f(const orc_quad *qd, const double x[13], const double T[4], double xd[13])
{
    const double *v = x + 3, *q = x + 6, *w = x + 10;
    const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    /* third column of R(q): the body z axis in the world frame */
    const double r3[3] = {2.0 * (qx * qz + qw * qy), 2.0 * (qy * qz - qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};

    /* collective thrust along body z, T = [0, 0, sum T_s] */
    double F = T[0] + T[1] + T[2] + T[3];
    /* torques from the X layout, Eq. (2) */
    double a = qd->arm / sqrt(2.0);
    double tau[3] = {a * (T[0] + T[1] - T[2] - T[3]),
                     a * (-T[0] + T[1] + T[2] - T[3]),
                     qd->c_tau * (T[0] - T[1] + T[2] - T[3])};

    /* p' = v */
    xd[0] = v[0]; xd[1] = v[1]; xd[2] = v[2];

    /* v' = g + R T / m - R D R^T v; the drag term vanishes for D = 0 */
    double dv[3] = {0.0, 0.0, 0.0};
    if (qd->drag[0] != 0.0 || qd->drag[1] != 0.0 || qd->drag[2] != 0.0) {
        double R[9], bv[3];
        rot_matrix(q, R);
        for (int i = 0; i < 3; ++i) bv[i] = R[0 + i] * v[0] + R[3 + i] * v[1] + R[6 + i] * v[2]; /* R^T v */
        for (int i = 0; i < 3; ++i) bv[i] *= qd->drag[i];                                        /* D R^T v */
        for (int i = 0; i < 3; ++i) dv[i] = R[3 * i + 0] * bv[0] + R[3 * i + 1] * bv[1] + R[3 * i + 2] * bv[2];
        xd[3] = r3[0] * F / qd->mass - dv[0];
        xd[4] = r3[1] * F / qd->mass - dv[1];
        xd[5] = r3[2] * F / qd->mass - qd->gravity - dv[2];
    } else {
        xd[3] = r3[0] * F / qd->mass;
        xd[4] = r3[1] * F / qd->mass;
        xd[5] = r3[2] * F / qd->mass - qd->gravity;
    }

    /* q' = 1/2 q (x) [0, w] */
    xd[6] = 0.5 * (-q[1] * w[0] - q[2] * w[1] - q[3] * w[2]);
    xd[7] = 0.5 * (q[0] * w[0] + q[2] * w[2] - q[3] * w[1]);
    xd[8] = 0.5 * (q[0] * w[1] - q[1] * w[2] + q[3] * w[0]);
    xd[9] = 0.5 * (q[0] * w[2] + q[1] * w[1] - q[2] * w[0]);

    /* w' = J^-1 (tau - w x J w) */
    const double *Jd = qd->inertia;
    double Jw[3] = {Jd[0] * w[0], Jd[1] * w[1], Jd[2] * w[2]};
    double cr[3] = {w[1] * Jw[2] - w[2] * Jw[1],
                    w[2] * Jw[0] - w[0] * Jw[2],
                    w[0] * Jw[1] - w[1] * Jw[0]};
    xd[10] = (tau[0] - cr[0]) / Jd[0];
    xd[11] = (tau[1] - cr[1]) / Jd[1];
    xd[12] = (tau[2] - cr[2]) / Jd[2];
}

/* Classical RK4 with the input held over the step, then the quaternion is
 * scaled back to unit norm (the discrete f of Eq. (1) with step dt). */
void orc_rk4(const orc_quad *qd, const double x[13], const double T[4], double dt, double xn[13])
{
    double k1[13], k2[13], k3[13], k4[13], xs[13];
    const double h2 = 0.5 * dt, h6 = dt / 6.0;
    orc_f(qd, x, T, k1);
    for (int i = 0; i < 13; ++i) xs[i] = x[i] + h2 * k1[i];
    orc_f(qd, xs, T, k2);
    for (int i = 0; i < 13; ++i) xs[i] = x[i] + h2 * k2[i];
    orc_f(qd, xs, T, k3);
    for (int i = 0; i < 13; ++i) xs[i] = x[i] + dt * k3[i];
    orc_f(qd, xs, T, k4);
    for (int i = 0; i < 13; ++i) xn[i] = x[i] + h6 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    double nq = sqrt(xn[6] * xn[6] + xn[7] * xn[7] + xn[8] * xn[8] + xn[9] * xn[9]);
    for (int i = 6; i < 10; ++i) xn[i] /= nq;
}

/* The paper's input model (Sec. III-A): the rotor thrusts are states and the
 * input is their time derivative.  f of the 13 states is Eq. (2) at the
 * current thrusts; the thrusts' own derivative is the input. */
void orc_f_rate(const orc_quad *qd, const double x[17], const double Tdot[4], double xd[17])
{
    orc_f(qd, x, x + 13, xd);
    for (int i = 0; i < 4; ++i) xd[13 + i] = Tdot[i];
}

/* Classical RK4 of the 17-state system with the rate held over the step, then
 * the quaternion scaled back to unit norm. */
void orc_rk4_rate(const orc_quad *qd, const double x[17], const double Tdot[4], double dt, double xn[17])
{
    double k1[17], k2[17], k3[17], k4[17], xs[17];
    const double h2 = 0.5 * dt, h6 = dt / 6.0;
    orc_f_rate(qd, x, Tdot, k1);
    for (int i = 0; i < 17; ++i) xs[i] = x[i] + h2 * k1[i];
    orc_f_rate(qd, xs, Tdot, k2);
    for (int i = 0; i < 17; ++i) xs[i] = x[i] + h2 * k2[i];
    orc_f_rate(qd, xs, Tdot, k3);
    for (int i = 0; i < 17; ++i) xs[i] = x[i] + dt * k3[i];
    orc_f_rate(qd, xs, Tdot, k4);
    for (int i = 0; i < 17; ++i) xn[i] = x[i] + h6 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    double nq = sqrt(xn[6] * xn[6] + xn[7] * xn[7] + xn[8] * xn[8] + xn[9] * xn[9]);
    for (int i = 6; i < 10; ++i) xn[i] /= nq;
}

/* ------------------------------------------------------------------------ */
/* Gate geometry.  Gate row = (cx, cy, cz, yaw); the gate is an upright
 * size x size square whose normal n = (cos yaw, sin yaw, 0) points in the
 * direction of travel.  A point is in front of the gate when (p-c).n < 0.
 * The segment pa->pb passes the gate when it goes from front (s<0) to behind
 * (s>=0) and meets the plane inside the closed square (Sec. IV-A, gate
 * switching).  margin receives the distance of this decision to the nearest
 * threshold that could flip it.                                             */

static double outside_aperture(const double p[3], const double gate[4], double half)
{
    double hx = -sin(gate[3]), hy = cos(gate[3]);
    double lat = (p[0] - gate[0]) * hx + (p[1] - gate[1]) * hy;
    double ver = p[2] - gate[2];
    double o = fabs(lat) - half;
    if (fabs(ver) - half > o) o = fabs(ver) - half;
    return o > 0.0 ? o : 0.0;
}

int orc_gate_cross(const double pa[3], const double pb[3], const double gate[4],
                   double size, double *margin)
{
    double nx = cos(gate[3]), ny = sin(gate[3]);
    double hx = -sin(gate[3]), hy = cos(gate[3]);
    double half = 0.5 * size;
    double sa = (pa[0] - gate[0]) * nx + (pa[1] - gate[1]) * ny;
    double sb = (pb[0] - gate[0]) * nx + (pb[1] - gate[1]) * ny;
    /* the margin is bookkeeping for the tests, computed only when asked for */
    double m = INFINITY;
    if (margin) {
        double ma = fabs(sa), oa = outside_aperture(pa, gate, half);
        double mb = fabs(sb), ob = outside_aperture(pb, gate, half);
        if ((ma > oa ? ma : oa) < m) m = (ma > oa ? ma : oa);
        if ((mb > ob ? mb : ob) < m) m = (mb > ob ? mb : ob);
    }
    int crossed = 0;
    if (sa < 0.0 && sb >= 0.0) {
        double t = sa / (sa - sb);
        double y[3] = {pa[0] + t * (pb[0] - pa[0]), pa[1] + t * (pb[1] - pa[1]),
                       pa[2] + t * (pb[2] - pa[2])};
        double lat = (y[0] - gate[0]) * hx + (y[1] - gate[1]) * hy;
        double ver = y[2] - gate[2];
        if (margin) {
            double el = fabs(fabs(lat) - half), ev = fabs(fabs(ver) - half);
            if (el < m) m = el;
            if (ev < m) m = ev;
        }
        crossed = (fabs(lat) <= half) && (fabs(ver) <= half);
    }
    if (margin) *margin = m;
    return crossed;
}

/* ------------------------------------------------------------------------ */
/* Arc-length path (contouring, Sec. IV-B-2).  The table holds P points
 * uniformly spaced in arc length over a closed path of length L, with unit
 * tangents.  The path between table points is the straight chord; theta is
 * (index + fraction) * L / P.                                                */

static double wrap_len(double th, double L)
{
    double r = fmod(th, L);
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
    return r;
}

double orc_project(const orc_cfg *c, const double p[3], double theta_prev, int global)
{
    int P = c->n_path;
    double ds = c->path_len / (double)P;
    int i_lo, i_hi, ic = 0;
    if (global) { i_lo = 0; i_hi = P - 1; }
    else {
        ic = (int)floor(wrap_len(theta_prev, c->path_len) / ds);
        if (ic >= P) ic = P - 1;
        i_lo = -c->proj_window; i_hi = c->proj_window;
    }
    double best = INFINITY, best_th = 0.0;
    for (int j = i_lo; j <= i_hi; ++j) {
        int i = global ? j : ((ic + j) % P + P) % P;
        int i1 = (i + 1) % P;
        const double *A = c->path + 6 * i, *B = c->path + 6 * i1;
        double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double ap[3] = {p[0] - A[0], p[1] - A[1], p[2] - A[2]};
        double l2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
        double t = l2 > 0.0 ? (ap[0] * ab[0] + ap[1] * ab[1] + ap[2] * ab[2]) / l2 : 0.0;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
        double d[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (d2 < best) { best = d2; best_th = ((double)i + t) * ds; }
    }
    return wrap_len(best_th, c->path_len);
}

/* ------------------------------------------------------------------------ */
/* Sampling, Eq. (3): U^m_k = U*_k + dU^m_k, dU ~ N(0, diag(sigma^2)); each
 * sample is clipped to the thrust bounds before it is rolled out, and the
 * clipped sample is what enters the average.  Contouring adds a fifth
 * channel, the progress speed, clipped to [0, v_max].                      */

static double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

void orc_sample(const orc_cfg *c, const orc_quad *q, const double *Ustar, const double *Vstar,
                uint32_t m, uint32_t s, double *U, double *V)
{
    for (int k = 0; k < c->N; ++k) {
        double z[4];
        orc_normals(c->seed, m, (uint32_t)k, s, 0u, z);
        for (int i = 0; i < 4; ++i)
            U[4 * k + i] = clampd(Ustar[4 * k + i] + c->sigma[i] * z[i], q->t_min, q->t_max);
        if (c->objective == ORC_OBJ_CONTOUR && V) {
            orc_normals(c->seed, m, (uint32_t)k, s, 1u, z);
            V[k] = clampd(Vstar[k] + c->sigma_v * z[0], 0.0, c->v_max);
        }
    }
}

/* Rate-model sampling, Eq. (3) with the paper's input u = dT/dt: each sampled
 * rate is clipped to the rate bounds (Table I) and then to the range that keeps
 * the thrust within its bounds at the end of the step (the thrust is linear
 * over the step, so it stays within them throughout); the thrust chain starts
 * at the measured T0.  Contouring samples the progress acceleration, clipped
 * to its bounds and to the range that keeps the progress speed in
 * [0, v_max].  The clipped values are the ones rolled out and averaged. */
void orc_sample_rate(const orc_cfg *c, const orc_quad *q, const double *Ustar, const double *Vstar,
                     uint32_t m, uint32_t s, int noisy, const double T0[4], double v0, double *U, double *V)
{
    double T[4] = {T0[0], T0[1], T0[2], T0[3]}, v = v0;
    for (int k = 0; k < c->N; ++k) {
        double z[4] = {0.0, 0.0, 0.0, 0.0};
        if (noisy) orc_normals(c->seed, m, (uint32_t)k, s, 0u, z);
        for (int i = 0; i < 4; ++i) {
            const double raw = noisy ? Ustar[4 * k + i] + c->sigma[i] * z[i] : Ustar[4 * k + i];
            const double r = clampd(raw, c->rate_lim[0], c->rate_lim[1]);
            const double u = clampd(r, (q->t_min - T[i]) / c->dt, (q->t_max - T[i]) / c->dt);
            U[4 * k + i] = u;
            T[i] = T[i] + c->dt * u;
        }
        if (c->objective == ORC_OBJ_CONTOUR && V) {
            double zv = 0.0;
            if (noisy) {
                orc_normals(c->seed, m, (uint32_t)k, s, 1u, z);
                zv = z[0];
            }
            const double raw = noisy ? Vstar[k] + c->sigma_v * zv : Vstar[k];
            const double r = clampd(raw, c->dv_lim[0], c->dv_lim[1]);
            const double a = clampd(r, (0.0 - v) / c->dt, (c->v_max - v) / c->dt);
            V[k] = a;
            v = v + c->dt * a;
        }
    }
}

/* Feasibility penalty (Sec. III-B: states outside their limits are charged an
 * extra cost): quadratic hinge on each body rate beyond w_max. */
static double limit_cost(const orc_cfg *c, const orc_quad *q, const double x[13])
{
    double J = 0.0;
    for (int i = 0; i < 3; ++i) {
        double e = fabs(x[10 + i]) - q->w_max;
        if (e > 0.0) J += c->w_lim * e * e;
    }
    return J;
}

static double sqdist3(const double a[3], const double b[3])
{
    double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return d0 * d0 + d1 * d1 + d2 * d2;
}

static void set_bit(uint32_t *mask, int j, int v)
{
    if (v) mask[j >> 5] |= (1u << (j & 31));
    else mask[j >> 5] &= ~(1u << (j & 31));
}

static int get_bit(const uint32_t *mask, int j)
{
    return (int)((mask[j >> 5] >> (j & 31)) & 1u);
}

/* Roll one control sequence out from x0 and return its cost (Alg. 1, inner
 * loop, with the objective selected by c->objective).
 *   gate     (Sec. IV-A, Eq. (6)-(7)): for k = 0..N-1
 *              near term  Q_near |p_k - p_gate0|^2 when |p_k - p_gate0| < r_near,
 *                          always w.r.t. the current gate g0;
 *              progress   |p_{k+1} - p_g|^2 - |p_k - p_g|^2, g = gate targeted by state k;
 *              limit      on w_{k+1};
 *              switching  if p_k -> p_{k+1} passes gate g, state k+1 and later
 *                          target gate g+1 (mod G); the first pass of the
 *                          horizon is registered only where allow bit k+1 is set
 *                          (the previous iteration's prediction had state k+1 in
 *                          front of the gate: temporal-consistency rule).
 *   tracking (Eq. (8)): stage |x_k - r_k|_Q^2 + |dT_k|_R^2, terminal |x_N - r_N|_QN^2,
 *              dT_k = (U_k - U_{k-1}) / dt with U_{-1} the last applied input.
 *   contour  (Eq. (9)): lag/contour error of p_k at theta_k, |w_k|_Qw^2,
 *              r_dv ((V_k - V_{k-1})/dt)^2, |dT_k|_R^2, -mu V_k;
 *              theta_{k+1} = theta_k + V_k dt (mod L).
 * When front is non-NULL the rollout is the nominal one and bit j of front is
 * set when state j (j = 0..N) is in front of gate g0.                        */
double orc_rollout_cost_ex(const orc_cfg *c, const orc_quad *q, const double *x0,
                           const double *U, const double *V, int32_t g0, const uint32_t *allow,
                           const double u_prev[4], double v_prev, double theta0, int32_t i0,
                           double *margin, uint32_t *front, uint32_t *front_amb, double *abs_sum)
{
    const int rate = c->input_model == ORC_INPUT_RATE;
    const int nx = rate ? 17 : 13;
    double x[17], xn[17];
    memcpy(x, x0, sizeof(double) * nx);
    double vth = v_prev; /* rate model, contouring: the progress speed state */
    double J = 0.0;
    double Jabs = 0.0; /* sum of the magnitudes of the quantities added to or
                          subtracted from J */
#define ORC_ADD(t) do { const double t_ = (t); J += t_; Jabs += fabs(t_); } while (0)
    double mrg = INFINITY;
    int g = g0, passes = 0;
    const double *gate0 = c->gates ? c->gates + 4 * g0 : NULL;

    if (front) {
        for (int j = 0; j < ORC_MASK_WORDS; ++j) { front[j] = 0u; front_amb[j] = 0u; }
    }
    double theta = theta0;
    double ds = c->n_path > 0 ? c->path_len / (double)c->n_path : 1.0;

    for (int k = 0; k < c->N; ++k) {
        const double *Uk = U + 4 * k;
        if (front) {
            double s = (x[0] - gate0[0]) * cos(gate0[3]) + (x[1] - gate0[1]) * sin(gate0[3]);
            set_bit(front, k, s < 0.0);
            set_bit(front_amb, k, fabs(s) < c->eps_dec);
        }
        if (c->objective == ORC_OBJ_TRACK) {
            int r = i0 + k < c->n_ref ? i0 + k : c->n_ref - 1;
            const double *xr = c->xref + 13 * r;
            for (int i = 0; i < 13; ++i) ORC_ADD(c->Q[i] * (x[i] - xr[i]) * (x[i] - xr[i]));
            if (rate) {
                /* the input itself is the thrust rate of Eq. (8)'s u_k */
                for (int i = 0; i < 4; ++i) ORC_ADD(c->R_dT[i] * Uk[i] * Uk[i]);
            } else {
                const double *Up = k > 0 ? U + 4 * (k - 1) : u_prev;
                for (int i = 0; i < 4; ++i) {
                    double d = (Uk[i] - Up[i]) / c->dt;
                    ORC_ADD(c->R_dT[i] * d * d);
                }
            }
        } else if (c->objective == ORC_OBJ_CONTOUR) {
            double sr = theta / ds;
            double fl = floor(sr);
            double f = sr - fl;
            int i = ((int)fl % c->n_path + c->n_path) % c->n_path;
            int i1 = (i + 1) % c->n_path;
            const double *A = c->path + 6 * i, *B = c->path + 6 * i1;
            double pi_[3], t[3], e[3], el[3], ec[3];
            for (int d = 0; d < 3; ++d) {
                pi_[d] = (1.0 - f) * A[d] + f * B[d];
                t[d] = (1.0 - f) * A[3 + d] + f * B[3 + d];
            }
            double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            for (int d = 0; d < 3; ++d) t[d] /= tn;
            for (int d = 0; d < 3; ++d) e[d] = x[d] - pi_[d];
            double et = e[0] * t[0] + e[1] * t[1] + e[2] * t[2];
            for (int d = 0; d < 3; ++d) { el[d] = et * t[d]; ec[d] = e[d] - el[d]; }
            ORC_ADD(c->q_l * (el[0] * el[0] + el[1] * el[1] + el[2] * el[2]));
            ORC_ADD(c->q_c * (ec[0] * ec[0] + ec[1] * ec[1] + ec[2] * ec[2]));
            for (int d = 0; d < 3; ++d) ORC_ADD(c->Q_w[d] * x[10 + d] * x[10 + d]);
            if (rate) {
                /* Eq. (9) literally: the sampled progress acceleration, the
                 * thrust rates, and the progress speed state v_theta,k */
                ORC_ADD(c->r_dv * V[k] * V[k]);
                for (int d = 0; d < 4; ++d) ORC_ADD(c->R_dT[d] * Uk[d] * Uk[d]);
                ORC_ADD(-c->mu * vth);
                const double vn = vth + c->dt * V[k];
                theta = wrap_len(theta + 0.5 * c->dt * (vth + vn), c->path_len);
                vth = vn;
            } else {
                double Vp = k > 0 ? V[k - 1] : v_prev;
                double dv = (V[k] - Vp) / c->dt;
                ORC_ADD(c->r_dv * dv * dv);
                const double *Up = k > 0 ? U + 4 * (k - 1) : u_prev;
                for (int d = 0; d < 4; ++d) {
                    double dT = (Uk[d] - Up[d]) / c->dt;
                    ORC_ADD(c->R_dT[d] * dT * dT);
                }
                ORC_ADD(-c->mu * V[k]);
                theta = wrap_len(theta + V[k] * c->dt, c->path_len);
            }
        } else {
            /* near-gate term, Eq. (7), w.r.t. the current gate g0 */
            double d2 = sqdist3(x, gate0);
            double d = sqrt(d2);
            if (d < c->r_near) ORC_ADD(c->q_near * d2);
            if (margin && fabs(d - c->r_near) < mrg) mrg = fabs(d - c->r_near);
        }

        if (rate) orc_rk4_rate(q, x, Uk, c->dt, xn);
        else orc_rk4(q, x, Uk, c->dt, xn);

        if (c->objective == ORC_OBJ_GATE) {
            const double *gc = c->gates + 4 * g;
            /* progress term, Eq. (6), toward the gate targeted by state k: a
             * difference of two squared distances, whose rounding scales with
             * the squares, so both count toward the magnitude sum */
            const double dn = sqdist3(xn, gc), dp = sqdist3(x, gc);
            J += dn - dp;
            Jabs += dn + dp;
        }
        ORC_ADD(limit_cost(c, q, xn));

        if (c->objective == ORC_OBJ_GATE) {
            const double *gc = c->gates + 4 * g;
            double mk = INFINITY;
            int crossed = orc_gate_cross(x, xn, gc, c->gate_size, margin ? &mk : NULL);
            if (mk < mrg) mrg = mk;
            if (crossed && (passes > 0 || get_bit(allow, k + 1))) {
                g = (g + 1) % c->n_gates;
                ++passes;
            }
        }
        memcpy(x, xn, sizeof(double) * nx);
    }
    if (c->objective == ORC_OBJ_TRACK) {
        int r = i0 + c->N < c->n_ref ? i0 + c->N : c->n_ref - 1;
        const double *xr = c->xref + 13 * r;
        for (int i = 0; i < 13; ++i) ORC_ADD(c->QN[i] * (x[i] - xr[i]) * (x[i] - xr[i]));
    }
    if (front) {
        double s = (x[0] - gate0[0]) * cos(gate0[3]) + (x[1] - gate0[1]) * sin(gate0[3]);
        set_bit(front, c->N, s < 0.0);
        set_bit(front_amb, c->N, fabs(s) < c->eps_dec);
    }
    if (margin) *margin = mrg;
    if (abs_sum) *abs_sum = Jabs;
#undef ORC_ADD
    return J;
}

double orc_rollout_cost(const orc_cfg *c, const orc_quad *q, const double *x0,
                        const double *U, const double *V, int32_t g0, const uint32_t *allow,
                        const double u_prev[4], double v_prev, double theta0, int32_t i0,
                        double *margin, uint32_t *front, uint32_t *front_amb)
{
    return orc_rollout_cost_ex(c, q, x0, U, V, g0, allow, u_prev, v_prev, theta0, i0, margin, front,
                               front_amb, NULL);
}

/* ------------------------------------------------------------------------ */

void orc_warm_init(orc_warm *w, int32_t g0)
{
    memset(w, 0, sizeof *w);
    w->g0 = g0;
}

static int cfg_valid(const orc_quad *q, const orc_cfg *c)
{
    if (c->K < 1 || c->N < 1 || c->N > ORC_NMAX) return 0;
    if (!(c->dt > 0.0) || !(c->lambda > 0.0)) return 0;
    for (int i = 0; i < 4; ++i) if (!(c->sigma[i] >= 0.0)) return 0;
    if (c->n_iter < 0 || c->n_iter > 64 || !(c->ctrl_cost >= 0.0) || !isfinite(c->ctrl_cost)) return 0;
    if (c->input_model != ORC_INPUT_THRUST && c->input_model != ORC_INPUT_RATE) return 0;
    if (c->input_model == ORC_INPUT_RATE &&
        (!(c->rate_lim[0] <= 0.0) || !(c->rate_lim[1] >= 0.0) || !(c->dv_lim[0] <= 0.0) || !(c->dv_lim[1] >= 0.0)))
        return 0;
    if (!(q->mass > 0.0) || !(q->t_max >= q->t_min)) return 0;
    for (int i = 0; i < 3; ++i) if (!(q->inertia[i] > 0.0)) return 0;
    if (c->objective == ORC_OBJ_GATE) {
        if (!c->gates || c->n_gates < 1) return 0;
    } else if (c->objective == ORC_OBJ_CONTOUR) {
        if (!c->path || c->n_path < 2 || !(c->path_len > 0.0)) return 0;
    } else if (c->objective == ORC_OBJ_TRACK) {
        if (!c->xref || c->n_ref < 1 || !(c->ref_dt > 0.0)) return 0;
    } else {
        return 0;
    }
    return 1;
}

/* The control-cost term of information-theoretic MPPI (Williams et al., the
 * MPPI line of work the paper builds on, Sec. II-A): gamma times
 * sum_k sum_i U*_k,i (U^m_k,i - U*_k,i) / sigma_i^2 over the channels with
 * sigma_i > 0 (the four thrusts, then the contouring speed), summed in step
 * order with the channels inside.  The perturbation is the one applied, after
 * clipping.  abs_sum receives the sum of the magnitudes of the products. */
static double control_cost(const orc_cfg *c, const double *Ustar, const double *Vstar, const double *U,
                           const double *V, double *abs_sum)
{
    double C = 0.0, A = 0.0;
    for (int k = 0; k < c->N; ++k) {
        for (int i = 0; i < 4; ++i) {
            if (!(c->sigma[i] > 0.0)) continue;
            const double t = c->ctrl_cost * Ustar[4 * k + i] * (U[4 * k + i] - Ustar[4 * k + i]) /
                             (c->sigma[i] * c->sigma[i]);
            C += t;
            A += fabs(t);
        }
        if (c->objective == ORC_OBJ_CONTOUR && c->sigma_v > 0.0) {
            const double t = c->ctrl_cost * Vstar[k] * (V[k] - Vstar[k]) / (c->sigma_v * c->sigma_v);
            C += t;
            A += fabs(t);
        }
    }
    *abs_sum = A;
    return C;
}

/* One MPPI iteration from the inherited state (Sec. III-B, Alg. 1).  An inner
 * iteration (the second and later of one control step, same x0 and t_now)
 * samples around the previous iteration's solution without shifting it and
 * keeps the last applied input (u_keep, v_keep) of the first iteration for
 * the rate terms; *u_used / *v_used return the ones this iteration used. */
static int solve_iteration(const orc_quad *q, const orc_cfg *c, orc_warm *warm, const double *x0,
                           double t_now, const double *J_rep, const uint8_t *rep_mask, orc_out *out,
                           int inner, const double u_keep[4], double v_keep, double u_used[4],
                           double *v_used)
{
    const int K = c->K, N = c->N;
    const int rate = c->input_model == ORC_INPUT_RATE;
    /* cold start: hover thrust for the thrust input; for the rate input the
     * zero sequence of Alg. 1 (it holds the measured thrusts) */
    const double hover = rate ? 0.0 : q->mass * q->gravity / 4.0;

    /* ---- inherited state (receding horizon, Sec. III-B / Alg. 1) ---- */
    double Ustar[ORC_NMAX * 4], Vstar[ORC_NMAX], u_prev[4], v_prev;
    uint32_t allow[ORC_MASK_WORDS];
    int32_t g0 = warm->g0, shift = 0;
    double theta0 = 0.0;
    const int same_step = inner && warm->warm && warm->t_prev == t_now;
    if (warm->warm) {
        /* shift the previous solution by the elapsed steps, repeat its tail */
        double el = (t_now - warm->t_prev) / c->dt;
        if (!(el < 1.0e6)) el = 1.0e6; /* keeps the conversion to int defined */
        if (el < 0.0) el = 0.0;
        shift = (int32_t)floor(el + 0.5);
        if (shift < 1) shift = 1;
        if (same_step) shift = 0;
        for (int k = 0; k < N; ++k) {
            int src = k + shift < N ? k + shift : N - 1;
            for (int i = 0; i < 4; ++i) Ustar[4 * k + i] = warm->U[4 * src + i];
            Vstar[k] = warm->V[src];
        }
        for (int i = 0; i < 4; ++i) u_prev[i] = same_step ? u_keep[i] : warm->U[i];
        v_prev = same_step ? v_keep : warm->V[0];
        memcpy(allow, warm->allow, sizeof allow);
        /* the measured motion since the previous solve passed gate g0 */
        if (c->objective == ORC_OBJ_GATE &&
            orc_gate_cross(warm->x_prev, x0, c->gates + 4 * g0, c->gate_size, NULL)) {
            g0 = (g0 + 1) % c->n_gates;
            for (int j = 0; j < ORC_MASK_WORDS; ++j) allow[j] = 0xffffffffu;
        }
        if (c->objective == ORC_OBJ_CONTOUR) theta0 = orc_project(c, x0, warm->theta0, 0);
    } else {
        for (int k = 0; k < N; ++k) {
            for (int i = 0; i < 4; ++i) Ustar[4 * k + i] = hover;
            Vstar[k] = 0.0;
        }
        for (int i = 0; i < 4; ++i) u_prev[i] = hover;
        v_prev = 0.0;
        for (int j = 0; j < ORC_MASK_WORDS; ++j) allow[j] = 0xffffffffu;
        if (c->objective == ORC_OBJ_CONTOUR) theta0 = orc_project(c, x0, 0.0, 1);
    }
    /* rate model, contouring: the progress speed state.  The previous solve's
     * initial speed advanced over the shift by its averaged accelerations
     * (clamped to [0, v_max] at each step) and held beyond that solution's
     * horizon; an inner iteration keeps it. */
    double v0 = 0.0;
    if (rate && warm->warm) {
        v0 = warm->vtheta;
        for (int j = 0; j < shift && j < N; ++j) v0 = clampd(v0 + c->dt * warm->V[j], 0.0, c->v_max);
    }
    if (rate) v_prev = v0;
    for (int i = 0; i < 4; ++i) u_used[i] = u_prev[i];
    *v_used = v_prev;
    if (c->objective == ORC_OBJ_GATE && (g0 < 0 || g0 >= c->n_gates)) return ORC_EINVAL;
    /* reference row of x0, held at the last row past the end of the table */
    int32_t i0 = 0;
    if (c->objective == ORC_OBJ_TRACK) {
        double r = floor(t_now / c->ref_dt + 0.5);
        if (!(r >= 0.0)) r = 0.0;
        if (r > (double)(c->n_ref - 1)) r = (double)(c->n_ref - 1);
        i0 = (int32_t)r;
    }
    const uint32_t s = warm->s;

    /* ---- samples, rollouts, costs (Alg. 1, inner loop) ---- */
    double Jmin = INFINITY;
    int n_amb = 0;
    int nt = c->n_threads > 0 ? c->n_threads : 1;
    double *Jv = out->J, *Mv = out->margin, *Av = out->absJ;
#pragma omp parallel num_threads(nt) reduction(+ : n_amb)
    {
        double Um[ORC_NMAX * 4], Vm[ORC_NMAX];
#pragma omp for schedule(dynamic, 16)
        for (int m = 0; m < K; ++m) {
            if (rate) orc_sample_rate(c, q, Ustar, Vstar, (uint32_t)m, s, 1, x0 + 13, v0, Um, Vm);
            else orc_sample(c, q, Ustar, Vstar, (uint32_t)m, s, Um, Vm);
            double mg, am;
            double Jm = orc_rollout_cost_ex(c, q, x0, Um, Vm, g0, allow, u_prev, v_prev, theta0, i0,
                                            &mg, NULL, NULL, &am);
            if (c->ctrl_cost != 0.0) {
                double ac;
                Jm += control_cost(c, Ustar, Vstar, Um, Vm, &ac);
                am += ac;
            }
            if (Jv) Jv[m] = Jm;
            if (Mv) Mv[m] = mg;
            if (Av) Av[m] = am;
            if (mg < c->eps_dec) n_amb += 1;
        }
    }

    /* ---- weights, Eq. (4), shifted by the minimum (identical by shift
     *      invariance); non-finite costs get zero weight ---- */
    for (int m = 0; m < K; ++m) {
        double Je = (rep_mask && rep_mask[m]) ? J_rep[m] : Jv[m];
        if (!isfinite(Je)) Je = INFINITY;
        if (Je < Jmin) Jmin = Je;
    }
    out->J_min = Jmin;
    out->n_amb = n_amb;
    out->g0 = g0; out->i0 = i0; out->shift = shift; out->theta0 = theta0;
    memcpy(out->allow, allow, sizeof allow);
    if (!isfinite(Jmin)) { out->status = ORC_ENONFINITE; return ORC_ENONFINITE; }

    double S = 0.0;
    for (int m = 0; m < K; ++m) {
        double Je = (rep_mask && rep_mask[m]) ? J_rep[m] : Jv[m];
        if (!isfinite(Je)) Je = INFINITY;
        S += exp(-(Je - Jmin) / c->lambda);
    }
    double ess_den = 0.0;
    /* normalised weights w_m (kept in a local buffer when not requested) */
    double *w = out->w;
    for (int m = 0; m < K; ++m) {
        double Je = (rep_mask && rep_mask[m]) ? J_rep[m] : Jv[m];
        if (!isfinite(Je)) Je = INFINITY;
        double wm = exp(-(Je - Jmin) / c->lambda) / S;
        if (w) w[m] = wm;
        ess_den += wm * wm;
    }
    out->S = S;
    out->ess = 1.0 / ess_den;

    /* ---- update, Eq. (5): U = sum_m w_m U^m, index order over m ---- */
    double Ubar[ORC_NMAX * 4], Vbar[ORC_NMAX];
    if (rate) {
        /* a rate sample follows its thrust chain along the horizon: draw each
         * sample whole; every element still adds the samples in index order */
        for (int i = 0; i < 4 * N; ++i) Ubar[i] = 0.0;
        for (int k = 0; k < N; ++k) Vbar[k] = 0.0;
        double Um[ORC_NMAX * 4], Vm[ORC_NMAX];
        for (int m = 0; m < K; ++m) {
            double Je = (rep_mask && rep_mask[m]) ? J_rep[m] : Jv[m];
            if (!isfinite(Je)) Je = INFINITY;
            const double wm = exp(-(Je - Jmin) / c->lambda) / S;
            orc_sample_rate(c, q, Ustar, Vstar, (uint32_t)m, s, 1, x0 + 13, v0, Um, Vm);
            for (int i = 0; i < 4 * N; ++i) Ubar[i] += wm * Um[i];
            if (c->objective == ORC_OBJ_CONTOUR)
                for (int k = 0; k < N; ++k) Vbar[k] += wm * Vm[k];
        }
    } else
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int k = 0; k < N; ++k) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0}, accv = 0.0;
        for (int m = 0; m < K; ++m) {
            double Je = (rep_mask && rep_mask[m]) ? J_rep[m] : Jv[m];
            if (!isfinite(Je)) Je = INFINITY;
            double wm = exp(-(Je - Jmin) / c->lambda) / S;
            double z[4];
            orc_normals(c->seed, (uint32_t)m, (uint32_t)k, s, 0u, z);
            for (int i = 0; i < 4; ++i)
                acc[i] += wm * clampd(Ustar[4 * k + i] + c->sigma[i] * z[i], q->t_min, q->t_max);
            if (c->objective == ORC_OBJ_CONTOUR) {
                orc_normals(c->seed, (uint32_t)m, (uint32_t)k, s, 1u, z);
                accv += wm * clampd(Vstar[k] + c->sigma_v * z[0], 0.0, c->v_max);
            }
        }
        for (int i = 0; i < 4; ++i) Ubar[4 * k + i] = acc[i];
        Vbar[k] = c->objective == ORC_OBJ_CONTOUR ? accv : 0.0;
    }

    /* ---- nominal rollout (noise-free sample of U*), whose states in front of
     *      gate g0 become the next solve's temporal-consistency mask ---- */
    double Un[ORC_NMAX * 4], Vn[ORC_NMAX];
    if (rate) {
        orc_sample_rate(c, q, Ustar, Vstar, 0u, s, 0, x0 + 13, v0, Un, Vn);
    } else {
        for (int k = 0; k < N; ++k) {
            for (int i = 0; i < 4; ++i) Un[4 * k + i] = clampd(Ustar[4 * k + i], q->t_min, q->t_max);
            Vn[k] = clampd(Vstar[k], 0.0, c->v_max);
        }
    }
    uint32_t front[ORC_MASK_WORDS], front_amb[ORC_MASK_WORDS];
    for (int j = 0; j < ORC_MASK_WORDS; ++j) { front[j] = 0xffffffffu; front_amb[j] = 0u; }
    double Jnom, Anom = 0.0;
    if (c->objective == ORC_OBJ_GATE)
        Jnom = orc_rollout_cost_ex(c, q, x0, Un, Vn, g0, allow, u_prev, v_prev, theta0, i0, NULL,
                                   front, front_amb, &Anom);
    else
        Jnom = orc_rollout_cost_ex(c, q, x0, Un, Vn, g0, allow, u_prev, v_prev, theta0, i0, NULL,
                                   NULL, NULL, &Anom);
    out->J_nom = Jnom;
    out->absJ_nom = Anom;
    memcpy(out->front, front, sizeof front);
    memcpy(out->front_amb, front_amb, sizeof front_amb);

    if (out->U) memcpy(out->U, Ubar, sizeof(double) * 4 * N);
    if (out->V) memcpy(out->V, Vbar, sizeof(double) * N);
    if (out->Ustar) memcpy(out->Ustar, Ustar, sizeof(double) * 4 * N);
    if (out->Vstar) memcpy(out->Vstar, Vstar, sizeof(double) * N);

    /* ---- the state the next solve inherits ---- */
    warm->warm = 1;
    warm->g0 = g0;
    warm->s = s + 1u;
    memcpy(warm->allow, front, sizeof front);
    warm->t_prev = t_now;
    memcpy(warm->x_prev, x0, sizeof warm->x_prev);
    warm->theta0 = theta0;
    warm->vtheta = rate ? v0 : 0.0;
    memcpy(warm->U, Ubar, sizeof(double) * 4 * N);
    memcpy(warm->V, Vbar, sizeof(double) * N);
    out->status = ORC_OK;
    return ORC_OK;
}

int orc_solve(const orc_quad *q, const orc_cfg *c, orc_warm *warm, const double *x0,
              double t_now, const double *J_rep, const uint8_t *rep_mask, orc_out *out)
{
    if (!cfg_valid(q, c) || !warm || !x0 || !out || !out->J || !isfinite(t_now)) return ORC_EINVAL;
    if ((J_rep == NULL) != (rep_mask == NULL)) return ORC_EINVAL;
    for (int i = 0; i < (c->input_model == ORC_INPUT_RATE ? 17 : 13); ++i)
        if (!isfinite(x0[i])) return ORC_EINVAL;
    /* several iterations per control step; the replayed costs belong to the last */
    const int n_iter = c->n_iter > 1 ? c->n_iter : 1;
    double u_keep[4] = {0.0, 0.0, 0.0, 0.0}, v_keep = 0.0;
    int n_amb_earlier = 0, st = ORC_OK;
    for (int it = 0; it < n_iter; ++it) {
        const int last = it == n_iter - 1;
        double u_used[4], v_used;
        st = solve_iteration(q, c, warm, x0, t_now, last ? J_rep : NULL, last ? rep_mask : NULL, out, it > 0,
                             u_keep, v_keep, u_used, &v_used);
        if (it == 0) {
            memcpy(u_keep, u_used, sizeof u_keep);
            v_keep = v_used;
        }
        if (!last) n_amb_earlier += out->n_amb;
    }
    out->n_amb_earlier = n_amb_earlier;
    return st;
}
