// Quadrotor dynamics (Sec. III-A, Eq. (2)) and one RK4 step in registers.
//
// State x = [p, v, q = (w, x, y, z), omega]; input = four rotor thrusts held
// over the step.  The quaternion is scaled back to unit norm after every
// step.  Binary32 rollouts carry the state in plain binary32: over horizons
// of up to 256 steps their cost errors stay near 1e-6 of the cost scale (the
// magnitudes of the terms), and the cost sums themselves are compensated.
#pragma once

#include "device.hpp"

namespace mppi {

template <typename Real> struct Model {
    Real inv_m, g, arm_s, c_tau;
    Real ijx, ijy, ijz, gx, gy, gz;
    Real d0, d1, d2;
    bool drag;

    __device__ __forceinline__ explicit Model(const KArgs &a)
        : inv_m((Real)a.inv_mass), g((Real)a.gravity), arm_s((Real)a.arm_s), c_tau((Real)a.c_tau),
          ijx((Real)a.inv_J[0]), ijy((Real)a.inv_J[1]), ijz((Real)a.inv_J[2]),
          gx((Real)a.gyro[0]), gy((Real)a.gyro[1]), gz((Real)a.gyro[2]),
          d0((Real)a.drag[0]), d1((Real)a.drag[1]), d2((Real)a.drag[2]), drag(a.has_drag != 0) {}
};

// Per-step input terms: collective thrust over mass and torque over inertia.
template <typename Real> struct StepInput {
    Real fm, tx, ty, tz;
};

template <typename Real>
__device__ __forceinline__ StepInput<Real> step_input(const Model<Real> &M, Real u0, Real u1, Real u2,
                                                       Real u3)
{
    StepInput<Real> s;
    s.fm = ((u0 + u1) + (u2 + u3)) * M.inv_m;
    s.tx = M.arm_s * ((u0 + u1) - (u2 + u3)) * M.ijx;
    s.ty = M.arm_s * ((u1 + u2) - (u0 + u3)) * M.ijy;
    s.tz = M.c_tau * ((u0 + u2) - (u1 + u3)) * M.ijz;
    return s;
}

template <typename Real>
__device__ __forceinline__ void deriv(const Model<Real> &M, const StepInput<Real> &in, const Real *x,
                                      Real *d)
{
    const Real qw = x[6], qx = x[7], qy = x[8], qz = x[9];
    const Real wx = x[10], wy = x[11], wz = x[12];
    d[0] = x[3];
    d[1] = x[4];
    d[2] = x[5];
    // thrust direction: third column of R(q)
    const Real r3x = Real(2) * (qx * qz + qw * qy);
    const Real r3y = Real(2) * (qy * qz - qw * qx);
    const Real r3z = Real(1) - Real(2) * (qx * qx + qy * qy);
    d[3] = in.fm * r3x;
    d[4] = in.fm * r3y;
    d[5] = in.fm * r3z - M.g;
    if (M.drag) {
        // - R D R^T v
        const Real r11 = Real(1) - Real(2) * (qy * qy + qz * qz), r12 = Real(2) * (qx * qy - qw * qz);
        const Real r21 = Real(2) * (qx * qy + qw * qz), r22 = Real(1) - Real(2) * (qx * qx + qz * qz);
        const Real r31 = Real(2) * (qx * qz - qw * qy), r32 = Real(2) * (qy * qz + qw * qx);
        const Real vx = x[3], vy = x[4], vz = x[5];
        const Real b0 = M.d0 * (r11 * vx + r21 * vy + r31 * vz);
        const Real b1 = M.d1 * (r12 * vx + r22 * vy + r32 * vz);
        const Real b2 = M.d2 * (r3x * vx + r3y * vy + r3z * vz);
        d[3] -= r11 * b0 + r12 * b1 + r3x * b2;
        d[4] -= r21 * b0 + r22 * b1 + r3y * b2;
        d[5] -= r31 * b0 + r32 * b1 + r3z * b2;
    }
    // q' = 1/2 q (x) (0, omega)
    d[6] = Real(0.5) * (-qx * wx - qy * wy - qz * wz);
    d[7] = Real(0.5) * (qw * wx + qy * wz - qz * wy);
    d[8] = Real(0.5) * (qw * wy - qx * wz + qz * wx);
    d[9] = Real(0.5) * (qw * wz + qx * wy - qy * wx);
    // omega' = J^-1 (tau - omega x J omega)
    d[10] = in.tx - M.gx * wy * wz;
    d[11] = in.ty - M.gy * wz * wx;
    d[12] = in.tz - M.gz * wx * wy;
}

// Scale a quaternion back to unit norm: the hardware reciprocal square root
// in binary32, the correctly rounded square root and division in binary64.
__device__ __forceinline__ void renormalize(float *q)
{
    const float r = inv_sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] *= r;
}
__device__ __forceinline__ void renormalize(double *q)
{
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] /= nq;
}

template <typename Real> struct State {
    Real x[13];
};

template <typename Real> __device__ __forceinline__ void load_state(State<Real> &s, const double *x0)
{
#pragma unroll
    for (int i = 0; i < 13; ++i) s.x[i] = (Real)x0[i];
}

// Add the increment of one step, then renormalise the quaternion.
template <typename Real> __device__ __forceinline__ void commit(State<Real> &s, const Real *dx)
{
#pragma unroll
    for (int i = 0; i < 13; ++i) s.x[i] += dx[i];
    renormalize(s.x + 6);
}

// dx = dt/6 (k1 + 2 k2 + 2 k3 + k4) for the input held over the step.
template <typename Real>
__device__ __forceinline__ void rk4_increment(const Model<Real> &M, const StepInput<Real> &in,
                                              const Real *x, Real dt, Real *dx)
{
    Real k[13], xs[13];
    const Real h2 = Real(0.5) * dt;
    deriv(M, in, x, k);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        dx[i] = k[i];
        xs[i] = x[i] + h2 * k[i];
    }
    deriv(M, in, xs, k);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        dx[i] += Real(2) * k[i];
        xs[i] = x[i] + h2 * k[i];
    }
    deriv(M, in, xs, k);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        dx[i] += Real(2) * k[i];
        xs[i] = x[i] + dt * k[i];
    }
    deriv(M, in, xs, k);
    const Real dt6 = dt / Real(6);
#pragma unroll
    for (int i = 0; i < 13; ++i) dx[i] = dt6 * (dx[i] + k[i]);
}

// The same for the rate model: the thrusts move linearly over the step, so
// the stages see the inputs in1 (start), in2 (middle, stages 2 and 3) and in4
// (end of the step).
template <typename Real>
__device__ __forceinline__ void rk4_increment_stages(const Model<Real> &M, const StepInput<Real> &in1,
                                                     const StepInput<Real> &in2, const StepInput<Real> &in4,
                                                     const Real *x, Real dt, Real *dx)
{
    Real k[13], xs[13];
    const Real h2 = Real(0.5) * dt;
    deriv(M, in1, x, k);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        dx[i] = k[i];
        xs[i] = x[i] + h2 * k[i];
    }
    deriv(M, in2, xs, k);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        dx[i] += Real(2) * k[i];
        xs[i] = x[i] + h2 * k[i];
    }
    deriv(M, in2, xs, k);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        dx[i] += Real(2) * k[i];
        xs[i] = x[i] + dt * k[i];
    }
    deriv(M, in4, xs, k);
    const Real dt6 = dt / Real(6);
#pragma unroll
    for (int i = 0; i < 13; ++i) dx[i] = dt6 * (dx[i] + k[i]);
}

}  // namespace mppi
