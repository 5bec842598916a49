// Gaussian mode factors Omega_j (the paper's "random Gaussian matrices",
// Sec. 3.2 and the residual sketching of Sec. 3.3), generated on the device
// by Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
//
// key = (seed lo, seed hi), counter = (row pair p, global column c, mode j,
// 0x4B525031); the two 53-bit uniforms from words (w0,w1) and (w2,w3) give
// Omega_j(2p, c) and Omega_j(2p+1, c).
#include "kernels.hpp"

namespace ttr {

namespace {
constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
constexpr uint32_t kOmegaTag = 0x4B525031u;

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
    const uint32_t lo0 = kM0 * c0, hi0 = __umulhi(kM0, c0);
    const uint32_t lo1 = kM1 * c2, hi1 = __umulhi(kM1, c2);
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
            k0 += kW0;
            k1 += kW1;
        }
        philox_round(c[0], c[1], c[2], c[3], k0, k1);
    }
}

__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
    const uint64_t v = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 11;
    return ((double)v + 0.5) * 0x1.0p-53;
}

// One thread per (mode, row pair, column).
__global__ void __launch_bounds__(256) omega_kernel(OmegaArgs a) {
    const int mi = blockIdx.y;  // index into the mode list
    const int mode = a.first_mode + mi;
    const int64_t n = a.n[mi];
    const int64_t npairs = (n + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npairs * a.ncols) return;
    const int64_t p = t / a.ncols;
    const int64_t cl = t - p * a.ncols;  // local column
    const uint64_t cg = (uint64_t)(a.col0 + cl);
    uint32_t c[4] = {(uint32_t)p, (uint32_t)cg, (uint32_t)mode, kOmegaTag};
    philox10(c, (uint32_t)(a.seed & 0xffffffffu), (uint32_t)(a.seed >> 32));
    const double u1 = uniform53(c[0], c[1]);
    const double u2 = uniform53(c[2], c[3]);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    double* out = a.base + a.off[mi];
    const int64_t col = a.store_col0 + cl;
    out[(2 * p) * a.ld + col] = rad * cos(ang);
    if (2 * p + 1 < n) out[(2 * p + 1) * a.ld + col] = rad * sin(ang);
}

__global__ void __launch_bounds__(256) philox_kernel(const uint32_t* __restrict__ ctr,
                                                     const uint32_t* __restrict__ key,
                                                     uint32_t* __restrict__ out, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    uint32_t c[4] = {ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3]};
    philox10(c, key[2 * t], key[2 * t + 1]);
#pragma unroll
    for (int i = 0; i < 4; ++i) out[4 * t + i] = c[i];
}
}  // namespace

void launch_omega(const OmegaArgs& a, int nmodes, int64_t max_n, hipStream_t s) {
    if (nmodes <= 0 || a.ncols <= 0) return;
    const int64_t work = ((max_n + 1) / 2) * a.ncols;
    dim3 grid(ceil_div(work, 256), nmodes);
    hipLaunchKernelGGL(omega_kernel, grid, dim3(256), 0, s, a);
    TTR_CHECK_LAUNCH();
}

void launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                   hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(philox_kernel, dim3(ceil_div(count, 256)), dim3(256), 0, s, ctr, key, out,
                       count);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
