/*
 * FP64 CPU oracle for one MPPI sampling step (test infrastructure only).
 *
 * This library is the slow, obviously-correct reference that the HIP path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it; the product library never links or calls it, and
 * it shares no source, header or constant table with the HIP path.
 *
 * What it computes, and where the paper defines it:
 *   - quadrotor dynamics f(x,u) and its RK4 discretisation ...... Sec. III-A, Eq. (2)
 *   - sampling U^m = U* + dU^m, dU ~ N(0, Sigma) .................. Sec. III-B, Eq. (3)
 *   - per-sample cost: gate progress (Eq. 6), its near-gate
 *     augmentation (Eq. 7) and in-horizon gate switching with the
 *     temporal-consistency rule ..................................... Sec. IV-A
 *   - trajectory-tracking cost .................................... Sec. IV-B-1, Eq. (8)
 *   - contouring cost ............................................. Sec. IV-B-2, Eq. (9)
 *   - softmax weights and weighted update ......................... Eq. (4), Eq. (5)
 *   - receding horizon / warm start ............................... Sec. III-B, Alg. 1
 *   - two standard MPPI variants the paper does not use, off by default:
 *     several iterations per control step, and the information-theoretic
 *     control-cost term (Williams et al.)  ........................ cited in Sec. II-A
 * The noise source (Philox4x32-10, Salmon et al., SC'11, with Box-Muller) is a
 * design choice of this project; the paper only requires Gaussian noise.
 *
 * Every floating-point quantity is IEEE double.  Summations run in index order.
 */
#ifndef MPPI_ORACLE_H
#define MPPI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NMAX 256          /* longest horizon the oracle accepts            */
#define ORC_MASK_WORDS 9      /* holds (ORC_NMAX + 1) bits of per-state flags   */

enum { ORC_OBJ_GATE = 0, ORC_OBJ_CONTOUR = 1, ORC_OBJ_TRACK = 2 };
/* Input models: the four rotor thrusts (13-state model), or their time
 * derivatives with the thrusts as four more states (the paper's model,
 * Sec. III-A: u = dT/dt, 17 states; contouring then samples the progress
 * acceleration and carries the progress speed as a state, Sec. IV-B-2). */
enum { ORC_INPUT_THRUST = 0, ORC_INPUT_RATE = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONFINITE = -4 };

typedef struct {
    double mass;          /* kg                                               */
    double arm;           /* l, m (X layout, rotors at 45 deg)                */
    double inertia[3];    /* diag(J), kg m^2                                  */
    double c_tau;         /* yaw torque per unit thrust, m                    */
    double drag[3];       /* diag(D) of the rotor-drag term, 1/s              */
    double gravity;       /* m/s^2, acts along -z                             */
    double t_min, t_max;  /* per-rotor thrust bounds, N                       */
    double w_max;         /* body-rate bound used by the limit penalty, rad/s */
} orc_quad;

typedef struct {
    int32_t K, N, objective, n_threads;
    double dt, lambda;
    double sigma[4];      /* per-rotor noise std, N                           */
    double sigma_v;       /* std of the contouring progress-speed channel     */
    uint64_t seed;
    /* feasibility penalty (all objectives) */
    double w_lim;
    /* gate objective */
    double q_near, r_near, eps_dec;
    /* tracking objective */
    double Q[13], QN[13], R_dT[4];
    /* contouring objective */
    double q_l, q_c, Q_w[3], r_dv, mu, v_max;
    /* problem data (caller-owned) */
    const double *gates; int32_t n_gates; double gate_size;   /* G x 4: cx cy cz yaw */
    const double *path;  int32_t n_path;  double path_len;    /* P x 6: p, unit tangent */
    const double *xref;  int32_t n_ref;   double ref_dt;      /* R x 13 */
    int32_t proj_window;  /* +- points searched around the previous arc length */
    /* standard MPPI variants the paper does not use (0 = off) */
    int32_t n_iter;       /* MPPI iterations per control step (0 or 1: one)      */
    double ctrl_cost;     /* gamma of the control-cost term gamma u*^T Sigma^-1 e */
    /* input model (ORC_INPUT_RATE: x0 has 17 entries, thrusts last) */
    int32_t input_model, pad3_;
    double rate_lim[2];   /* bounds of the sampled thrust rate, N/s              */
    double dv_lim[2];     /* bounds of the sampled progress acceleration, m/s^2  */
} orc_cfg;

/* Everything the next solve inherits from this one (receding horizon). */
typedef struct {
    int32_t warm;                  /* 0: cold start                              */
    int32_t g0;                    /* current target gate                         */
    uint32_t s;                    /* solve counter, Philox counter word 2        */
    int32_t pad_;
    uint32_t allow[ORC_MASK_WORDS];/* bit j: state j may register the first pass  */
    double t_prev;
    double x_prev[13];
    double theta0;                 /* arc length of the previous solve            */
    double U[ORC_NMAX * 4];        /* previous solution, N x 4                    */
    double V[ORC_NMAX];            /* previous progress-speed (or acceleration) solution, N */
    double vtheta;                 /* rate model, contouring: progress speed state at the
                                      previous solve's initial time                   */
} orc_warm;

typedef struct {
    /* caller-owned output arrays, each may be NULL */
    double *J;       /* K   sample costs (non-finite kept as computed)     */
    double *w;       /* K   normalised weights                             */
    double *U;       /* N*4 weighted update                                */
    double *V;       /* N   weighted progress speed (contouring)           */
    double *margin;  /* K   smallest distance of a discrete decision to its threshold */
    double *Ustar;   /* N*4 nominal sequence used for sampling             */
    double *Vstar;   /* N                                                  */
    /* scalars */
    double J_min, S, ess, J_nom, theta0;
    int32_t g0, i0, shift, n_amb, status, pad_;
    uint32_t allow[ORC_MASK_WORDS];     /* mask used by this solve                     */
    uint32_t front[ORC_MASK_WORDS];     /* nominal rollout states in front of gate g0  */
    uint32_t front_amb[ORC_MASK_WORDS]; /* front decisions within eps_dec of the plane */
    double *absJ;    /* K   sum of the magnitudes of the quantities a sample's cost adds or
                        subtracts (both squared distances of each Eq. (6) term; may be NULL) */
    double absJ_nom; /* the same sum for the nominal rollout                           */
    int32_t n_amb_earlier; /* ambiguous samples in the iterations before the last  */
    int32_t pad2_;
} orc_out;

/* ---- building blocks (exported for the pin tests) ---------------------- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t word);
void   orc_normals(uint64_t seed, uint32_t m, uint32_t k, uint32_t s, uint32_t ch, double z[4]);
void   orc_f(const orc_quad *q, const double x[13], const double T[4], double xd[13]);
void   orc_rk4(const orc_quad *q, const double x[13], const double T[4], double dt, double xn[13]);
/* The paper's model: x = (13 states, thrusts T[4]), input dT/dt held over the
 * step, RK4 of the 17-state system (the thrusts vary linearly over the step). */
void   orc_f_rate(const orc_quad *q, const double x[17], const double Tdot[4], double xd[17]);
void   orc_rk4_rate(const orc_quad *q, const double x[17], const double Tdot[4], double dt, double xn[17]);
/* Rate-model samples: the sampled rates are clipped to the rate bounds and then
 * to the range that keeps each thrust (speed) within its bounds over the step,
 * following the thrust (speed) chain from T0 (v0); z == NULL: no noise. */
void   orc_sample_rate(const orc_cfg *c, const orc_quad *q, const double *Ustar, const double *Vstar,
                       uint32_t m, uint32_t s, int noisy, const double T0[4], double v0, double *U,
                       double *V);
int    orc_gate_cross(const double pa[3], const double pb[3], const double gate[4],
                      double size, double *margin);
double orc_project(const orc_cfg *c, const double p[3], double theta_prev, int global);
void   orc_sample(const orc_cfg *c, const orc_quad *q, const double *Ustar, const double *Vstar,
                  uint32_t m, uint32_t s, double *U, double *V);
double orc_rollout_cost(const orc_cfg *c, const orc_quad *q, const double *x0,
                        const double *U, const double *V, int32_t g0, const uint32_t *allow,
                        const double u_prev[4], double v_prev, double theta0, int32_t i0,
                        double *margin, uint32_t *front, uint32_t *front_amb);
/* The same, also returning the sum of the magnitudes of the terms added to
 * the cost (the scale of its rounding error). */
double orc_rollout_cost_ex(const orc_cfg *c, const orc_quad *q, const double *x0,
                           const double *U, const double *V, int32_t g0, const uint32_t *allow,
                           const double u_prev[4], double v_prev, double theta0, int32_t i0,
                           double *margin, uint32_t *front, uint32_t *front_amb, double *abs_sum);

/* ---- one MPPI step --------------------------------------------------------
 * x0 holds 13 states (17 for ORC_INPUT_RATE: the thrusts appended).
 * warm is read (inherited state) and, on success, replaced by the state the
 * next solve inherits.  J_rep/rep_mask (both NULL or both K long) substitute
 * the given cost for every sample whose mask byte is non-zero before the
 * weights are formed; they let a test resolve a decision that lies within
 * rounding distance of its threshold the way the device resolved it. */
int orc_solve(const orc_quad *q, const orc_cfg *c, orc_warm *warm, const double *x0,
              double t_now, const double *J_rep, const uint8_t *rep_mask, orc_out *out);

void orc_warm_init(orc_warm *w, int32_t g0);

#ifdef __cplusplus
}
#endif
#endif
