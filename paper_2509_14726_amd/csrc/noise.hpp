// Counter-based Gaussian noise in registers for the sampling step, Eq. (3).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each taking
// the two 32x32->64-bit products of counter words 0 and 2 with the published
// multipliers; the high halves are xored with the other two counter words
// and the key, and the key advances by the published Weyl constants.  One
// block yields four 32-bit words for counter (m, k, s, ch) under key = seed.
//
// Uniforms: (2 * (word >> 9) + 1) * 2^-24, exact in binary32 and binary64,
// inside (0, 1).  Normals: Box-Muller on the pairs (u0, u1) and (u2, u3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

struct Words4 { uint32_t x, y, z, w; };

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kMul0 * c0;
        const uint64_t p2 = (uint64_t)kMul1 * c2;
        const uint32_t n0 = (uint32_t)(p2 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p2;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Words4{c0, c1, c2, c3};
}

template <typename Real> __device__ __forceinline__ Real unit_open(uint32_t w)
{
    return (Real)(int32_t)(2u * (w >> 9) + 1u) * (Real)(1.0 / 16777216.0);
}

template <typename Real> struct Normal4 { Real z0, z1, z2, z3; };

// binary32: the hardware transcendentals -- v_sin_f32 / v_cos_f32 take their
// argument in revolutions, v_log_f32 is log2 -- each within a few ulps on
// (0, 1), which bounds the error of a normal by about 1e-6.
__device__ __forceinline__ void sincos_2pi(float u, float *s, float *c)
{
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}
__device__ __forceinline__ float radius(float u)
{
    // sqrt(-2 ln u) = sqrt(-2 ln(2) log2(u))
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
}
// binary64: the accurate library functions
__device__ __forceinline__ void sincos_2pi(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }
__device__ __forceinline__ double radius(double u) { return sqrt(-2.0 * log(u)); }

template <typename Real>
__device__ __forceinline__ Normal4<Real> normals4(uint32_t m, uint32_t k, uint32_t s, uint32_t ch,
                                                  uint32_t key0, uint32_t key1)
{
    const Words4 w = philox4x32_10(m, k, s, ch, key0, key1);
    const Real r0 = radius(unit_open<Real>(w.x));
    const Real r1 = radius(unit_open<Real>(w.z));
    Real s0, c0, s1, c1;
    sincos_2pi(unit_open<Real>(w.y), &s0, &c0);
    sincos_2pi(unit_open<Real>(w.w), &s1, &c1);
    return Normal4<Real>{r0 * c0, r0 * s0, r1 * c1, r1 * s1};
}

// Only the first normal of a block (contouring progress-speed channel).
template <typename Real>
__device__ __forceinline__ Real normal1(uint32_t m, uint32_t k, uint32_t s, uint32_t ch,
                                        uint32_t key0, uint32_t key1)
{
    const Words4 w = philox4x32_10(m, k, s, ch, key0, key1);
    Real sn, cs;
    sincos_2pi(unit_open<Real>(w.y), &sn, &cs);
    return radius(unit_open<Real>(w.x)) * cs;
}

}  // namespace mppi
