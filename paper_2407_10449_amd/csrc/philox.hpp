// Counter-based Gaussian and uniform draws on the device.
//
// Philox4x32-10 (Salmon et al., SC'11): a 4 x 32-bit counter and a 2 x 32-bit
// key pass through ten rounds.  A round multiplies counter words 0 and 2 by
// two odd constants, and the new counter is (hi(word2 product) ^ c1 ^ k0,
// lo(word2 product), hi(word0 product) ^ c3 ^ k1, lo(word0 product)); the key
// grows by two Weyl increments between rounds.
// Box-Muller (1958) turns two uniforms into two normals, in float64.
//
// Stream layout: key = (seed low, seed high); counter = (j, chain, step,
// stream | problem << 8).  Stream 0 with pair index j yields nu[2j], nu[2j+1];
// stream 1 with j = 0 yields the uniform that picks theta.  A uniform is built
// from two words as (k + 0.5) * 2^-52, k = (w0 >> 6) * 2^26 + (w1 >> 6).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ess {

constexpr double kTwoPi = 6.283185307179586;
constexpr double kPi = 3.141592653589793;

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ double uniform52(uint32_t w0, uint32_t w1) {
    const uint64_t k = (static_cast<uint64_t>(w0 >> 6) << 26) | static_cast<uint64_t>(w1 >> 6);
    return (static_cast<double>(k) + 0.5) * 0x1p-52;
}

struct Rng {
    uint32_t k0, k1;
    __device__ explicit Rng(uint64_t seed)
        : k0(static_cast<uint32_t>(seed)), k1(static_cast<uint32_t>(seed >> 32)) {}

    // The two normals of pair j for (chain, step, problem).
    __device__ __forceinline__ void normal_pair(uint32_t j, uint32_t chain, uint32_t step,
                                                uint32_t problem, double& z0, double& z1) const {
        const u32x4 w = philox4x32_10(u32x4{j, chain, step, 0u | (problem << 8)}, k0, k1);
        const double u1 = uniform52(w.x, w.y);
        const double u2 = uniform52(w.z, w.w);
        const double rad = sqrt(-2.0 * log(u1));
        double s, c;
        sincos(kTwoPi * u2, &s, &c);
        z0 = rad * c;
        z1 = rad * s;
    }

    __device__ __forceinline__ double theta_uniform(uint32_t chain, uint32_t step,
                                                    uint32_t problem) const {
        const u32x4 w = philox4x32_10(u32x4{0u, chain, step, 1u | (problem << 8)}, k0, k1);
        return uniform52(w.x, w.y);
    }
};

}  // namespace ess
