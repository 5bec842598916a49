// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Box-Muller
// Gaussian pair that define the Gaussian mode factors Omega_j: key = (seed
// lo, seed hi), counter = (row pair p, global column c, mode j,
// 0x4B525031); the two 53-bit uniforms from words (w0,w1) and (w2,w3) give
// Omega_j(2p, c) and Omega_j(2p+1, c).  Shared by every kernel that draws
// Omega, so all of them produce the same values.
#pragma once

#include "common.hpp"

namespace ttr {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kOmegaTag = 0x4B525031u;

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
    const uint32_t lo0 = kPhiloxM0 * c0, hi0 = __umulhi(kPhiloxM0, c0);
    const uint32_t lo1 = kPhiloxM1 * c2, hi1 = __umulhi(kPhiloxM1, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
}

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        philox_round(c[0], c[1], c[2], c[3], k0, k1);
    }
}

__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
    const uint64_t v = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 11;
    return ((double)v + 0.5) * 0x1.0p-53;
}

// Omega_mode(2p, c) and Omega_mode(2p+1, c).
__device__ __forceinline__ void omega_pair(uint64_t seed, int64_t p, uint64_t c, int mode, double& g0,
                                           double& g1) {
    uint32_t w[4] = {(uint32_t)p, (uint32_t)c, (uint32_t)mode, kOmegaTag};
    philox10(w, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double u1 = uniform53(w[0], w[1]);
    const double u2 = uniform53(w[2], w[3]);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    g0 = rad * cos(ang);
    g1 = rad * sin(ang);
}

}  // namespace ttr
