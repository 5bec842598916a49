// Gaussian mode factors Omega_j (the paper's "random Gaussian matrices",
// Sec. 3.2 and the residual sketching of Sec. 3.3), generated on the device
// by Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
//
// The generator and its counter layout are defined in philox.hpp.
#include "kernels.hpp"
#include "philox.hpp"

namespace ttr {

namespace {

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
    double g0, g1;
    omega_pair(a.seed, p, cg, mode, g0, g1);
    double* out = a.base + a.off[mi];
    const int64_t col = a.store_col0 + cl;
    out[(2 * p) * a.ld + col] = g0;
    if (2 * p + 1 < n) out[(2 * p + 1) * a.ld + col] = g1;
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
