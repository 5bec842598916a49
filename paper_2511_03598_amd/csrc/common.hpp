// Shared device/host helpers for libttround (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace ttr {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Host-side error carrying a status code across the C++ runtime; the C ABI
// converts it into a tt_status and a thread-local message.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TTR_HIP(expr)                                                             \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess)                                                     \
            throw ::ttr::Error(-4, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define TTR_CHECK_LAUNCH() TTR_HIP(hipGetLastError())

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---- MFMA wrappers -------------------------------------------------------
// v_mfma_f64_16x16x4_f64: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element v of lane l is C[(l/16) + 4*v][l%16] (rows interleave
// across the four lane groups; checked on gfx950 with one-hot operands).
__device__ __forceinline__ double4_t mfma_f64_16x16x4(double a, double b, double4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// v_mfma_f32_16x16x4_f32: same operand layout; accumulator element v of
// lane l is C[4*(l/16) + v][l%16] (four consecutive rows per lane group).
__device__ __forceinline__ float4_t mfma_f32_16x16x4(float a, float b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of accumulator element v held by lane group g = l/16.
__device__ __forceinline__ int mfma_row_f64(int g, int v) { return g + 4 * v; }
__device__ __forceinline__ int mfma_row_f32(int g, int v) { return 4 * g + v; }

// ---- wave reductions (full 64-lane butterflies) --------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
// DPP move of a double (two 32-bit halves) with a constant control word.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
// Sum over the 16 lanes of a DPP row (lanes 16g..16g+15), result in every
// lane: swap neighbours, swap pairs (quad_perm), then fold the row with
// row_half_mirror and row_mirror.  All 16 lanes must be active.
__device__ __forceinline__ double group16_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}
// 1/sqrt(x) for normal positive x: hardware estimate (v_rsq_f64) plus two
// Newton steps, each of which squares the relative error; a few ulp.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
    y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
    return y;
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// Block-wide sum for blockDim.x == 256 (4 waves); every thread gets the sum.
// `red` must hold 4 doubles of LDS.  Contains two barriers.
__device__ __forceinline__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace ttr
