// Device helpers shared by the dense step kernel and the matrix-free
// (Conjugate Residual) step kernel: the actuation noise generator, the
// contact tangent basis, the Coulomb cone projection and lane-level
// reductions of a wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace kamx {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// A standard normal for (world, step, slot) by Box-Muller on two 24-bit
// uniforms (u1 in (0, 1], u2 in [0, 1)).
__device__ inline float noise_normal(uint32_t seed_lo, uint32_t seed_hi, uint32_t world, uint32_t step,
                                     uint32_t slot) {
    uint32_t c[4] = {world, step, slot, 0u};
    philox4x32_10(c, seed_lo, seed_hi);
    const float inv = 1.0f / 16777216.0f;
    float u1 = ((float)(c[0] >> 8) + 1.0f) * inv;
    float u2 = (float)(c[1] >> 8) * inv;
    return sqrtf(-2.0f * logf(u1)) * cosf(6.28318530717958647692f * u2);
}

// Orthonormal tangents completing a unit normal (Duff et al., JCGT 2017).
__device__ inline void tangents(const float n[3], float t1[3], float t2[3]) {
    float sg = n[2] >= 0.f ? 1.f : -1.f;
    float a = -1.f / (sg + n[2]);
    float b = n[0] * n[1] * a;
    t1[0] = 1.f + sg * n[0] * n[0] * a;
    t1[1] = sg * b;
    t1[2] = -sg * n[0];
    t2[0] = b;
    t2[1] = sg + n[1] * n[1] * a;
    t2[2] = -n[1];
}

// Projection on the Coulomb cone K_mu = {|l_t| <= mu l_n}.
// Square root and reciprocal by the hardware instructions (within 1 ulp;
// the correctly rounded forms take about ten instructions each), for the
// scalars the iteration recomputes every step.
__device__ inline float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ inline void proj_cone(float mu, float w0, float w1, float w2, float &o0, float &o1, float &o2) {
    float tn = hw_sqrt(w1 * w1 + w2 * w2);
    if (tn <= mu * w0) {
        o0 = w0;
        o1 = w1;
        o2 = w2;
    } else if (mu * tn <= -w0) {
        o0 = o1 = o2 = 0.f;
    } else {
        float ln = (mu * tn + w0) * hw_rcp(1.f + mu * mu);
        float s = tn > 0.f ? mu * ln * hw_rcp(tn) : 0.f;
        o0 = ln;
        o1 = s * w1;
        o2 = s * w2;
    }
}

// Lane permutations inside a row of 16 lanes (DPP): swap neighbours
// (lane ^ 1), swap pairs (lane ^ 2), mirror within 8 and within 16 lanes.
// Every lane of the wave must be active where these are used.
enum { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppMirror8 = 0x141, kDppMirror16 = 0x140 };

template <int CTRL>
__device__ inline float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ inline double dpp(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of 2, 4, 8 or 16 lanes; every lane of a group
// ends with the same bits (each step adds two values that the partner adds
// in the other order).
template <int G, typename T>
__device__ inline T lane_group_sum(T v) {
    if (G >= 2) v += dpp<kDppXor1>(v);
    if (G >= 4) v += dpp<kDppXor2>(v);
    if (G >= 8) v += dpp<kDppMirror8>(v);
    if (G >= 16) v += dpp<kDppMirror16>(v);
    return v;
}

// Maximum of values that are +0 or above, or NaN of either sign: as
// unsigned integers their bit patterns order like the numbers and every NaN
// lies above +inf, so one integer max keeps a NaN (a NaN residual must stop
// the solve). Negative numbers and -0 would compare wrongly: callers pass
// absolute values.
__device__ inline float max_nonneg(float a, float b) {
    const unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
    return __uint_as_float(ub > ua ? ub : ua);
}

template <int G>
__device__ inline float lane_group_max(float v) {
    if (G >= 2) v = max_nonneg(v, dpp<kDppXor1>(v));
    if (G >= 4) v = max_nonneg(v, dpp<kDppXor2>(v));
    if (G >= 8) v = max_nonneg(v, dpp<kDppMirror8>(v));
    if (G >= 16) v = max_nonneg(v, dpp<kDppMirror16>(v));
    return v;
}

// Sum over the G lanes that share a row (fixed butterfly order).
template <int G, typename T>
__device__ inline T group_sum(T v) {
    return lane_group_sum<G>(v);
}

// Broadcast a lane's value to the whole wave (lane index uniform).
__device__ inline float rdlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

}  // namespace kamx
