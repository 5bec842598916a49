// General float64 GEMM on MFMA (v_mfma_f64_16x16x4_f64) for the
// randomize-then-orthogonalize sweep (Sec. 3.2-3.3): the sketch
// S_k = V(Y_k) W_{k+1}, the projections Q^T S and Q^T V(Y_k), the next core
// M_k H(X_{k+1}) and the recompression products.
//
// 64x64 output tile per 256-thread workgroup, K staged through LDS in
// 32-deep double-buffered slabs (eight loads per operand and thread in
// flight per slab), each wave owning a 32x32 quadrant
// (2x2 MFMA blocks).  Operands are addressed by element strides so one
// kernel serves every transpose; the global->LDS thread mapping follows the
// contiguous dimension so loads stay coalesced.  Split-K writes partial
// tiles that a second kernel sums in a fixed order (deterministic).
#include "kernels.hpp"

namespace ttr {
namespace {

constexpr int BM = 64, BN = 64, BK = 32, LDP = BM + 4;
constexpr int TE = BM * BK / 256;  // elements per operand and thread per slab

struct Tile {
    double a[TE], b[TE];
};

// Element offset of C(row, col); with cdiv > 0 the column index splits as
// (col / cdiv, col % cdiv) with strides (cs_hi, scn).
__device__ __forceinline__ size_t c_offset(const GemmArgs& g, int row, int col) {
    if (g.cdiv > 0)
        return (size_t)row * g.scm + (size_t)(col / g.cdiv) * g.cs_hi + (size_t)(col % g.cdiv) * g.scn;
    return (size_t)row * g.scm + (size_t)col * g.scn;
}

// TE elements of B as double: FP64 storage, or FP32 / bfloat16 storage
// scaled by 2^bexp[n] when the sketch is kept in reduced precision.  A
// sliced B is the sum of its slices in slice order, taken in the storage's
// arithmetic type (FP64, or FP32 for both reduced formats); the loads of
// one slice are issued together before they are added.
__device__ __forceinline__ float stored_f32(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float stored_f32(const unsigned short* p, size_t i) {
    return __uint_as_float((unsigned)p[i] << 16);
}

template <typename T>
__device__ __forceinline__ void load_b_reduced(const GemmArgs& g, const T* B, const size_t (&off)[TE],
                                               const int (&nn)[TE], double (&out)[TE]) {
    float v[TE];
#pragma unroll
    for (int q = 0; q < TE; ++q) v[q] = stored_f32(B, off[q]);
    for (int s = 1; s < g.bslices; ++s) {
        const size_t so = (size_t)s * g.bstride;
#pragma unroll
        for (int q = 0; q < TE; ++q) v[q] += stored_f32(B, so + off[q]);
    }
#pragma unroll
    for (int q = 0; q < TE; ++q) out[q] = g.bexp ? ldexp((double)v[q], g.bexp[nn[q]]) : (double)v[q];
}

__device__ __forceinline__ void load_b(const GemmArgs& g, const size_t (&off)[TE],
                                       const int (&nn)[TE], double (&out)[TE]) {
    if (g.Bf) {
        load_b_reduced(g, g.Bf, off, nn, out);
    } else if (g.Bh) {
        load_b_reduced(g, g.Bh, off, nn, out);
    } else {
#pragma unroll
        for (int q = 0; q < TE; ++q) out[q] = g.B[off[q]];
        for (int s = 1; s < g.bslices; ++s) {
            const size_t so = (size_t)s * g.bstride;
#pragma unroll
            for (int q = 0; q < TE; ++q) out[q] += g.B[so + off[q]];
        }
    }
}

// Global -> registers for one K slab.  Indices are clamped into the matrix
// so every load is issued unconditionally (a masked load serialises on its
// own wait); out-of-range elements are zeroed afterwards.  The caller
// guarantees k0 < kend.
__device__ __forceinline__ void load_tiles(const GemmArgs& g, int m0, int n0, int k0, int kend,
                                           Tile& t) {
    const int tid = threadIdx.x;
    // A: 64 (m) x 32 (k)
    if (g.sak == 1) {
        // k contiguous: row m, 8 consecutive k
        const int m = tid >> 2, kk = (tid & 3) * TE;
        const int gm = m0 + m, gmc = min(gm, g.M - 1);
#pragma unroll
        for (int q = 0; q < TE; ++q) {
            const int gk = k0 + kk + q;
            const double v = g.A[(size_t)gmc * g.sam + min(gk, kend - 1)];
            t.a[q] = (gm < g.M && gk < kend) ? v : 0.0;
        }
    } else {
        // m contiguous (or strided): slab row kk, 8 consecutive m
        const int kk = tid >> 3, m = (tid & 7) * TE;
        const int gk = k0 + kk, gkc = min(gk, kend - 1);
#pragma unroll
        for (int q = 0; q < TE; ++q) {
            const int gm = m0 + m + q;
            const double v = g.A[(size_t)min(gm, g.M - 1) * g.sam + (size_t)gkc * g.sak];
            t.a[q] = (gm < g.M && gk < kend) ? v : 0.0;
        }
    }
    // B: 32 (k) x 64 (n)
    size_t off[TE];
    int nn[TE];
    bool ok[TE];
    if (g.sbn == 1 || g.sbk != 1) {
        const int kk = tid >> 3, n1 = (tid & 7) * TE;
        const int gk = k0 + kk, gkc = min(gk, kend - 1);
#pragma unroll
        for (int q = 0; q < TE; ++q) {
            const int gn = n0 + n1 + q, gnc = min(gn, g.N - 1);
            off[q] = (size_t)gkc * g.sbk + (size_t)gnc * g.sbn;
            nn[q] = gnc;
            ok[q] = gk < kend && gn < g.N;
        }
    } else {
        const int n1 = tid >> 2, kk = (tid & 3) * TE;
        const int gn = n0 + n1, gnc = min(gn, g.N - 1);
#pragma unroll
        for (int q = 0; q < TE; ++q) {
            const int gk = k0 + kk + q;
            off[q] = (size_t)min(gk, kend - 1) + (size_t)gnc * g.sbn;
            nn[q] = gnc;
            ok[q] = gk < kend && gn < g.N;
        }
    }
    load_b(g, off, nn, t.b);
#pragma unroll
    for (int q = 0; q < TE; ++q) t.b[q] = ok[q] ? t.b[q] : 0.0;
}

__device__ __forceinline__ void store_tiles(const GemmArgs& g, const Tile& t, double (*As)[LDP],
                                            double (*Bs)[LDP]) {
    const int tid = threadIdx.x;
    if (g.sak == 1) {
        const int m = tid >> 2, kk = (tid & 3) * TE;
#pragma unroll
        for (int q = 0; q < TE; ++q) As[kk + q][m] = t.a[q];
    } else {
        const int kk = tid >> 3, m = (tid & 7) * TE;
#pragma unroll
        for (int q = 0; q < TE; ++q) As[kk][m + q] = t.a[q];
    }
    if (g.sbn == 1 || g.sbk != 1) {
        const int kk = tid >> 3, nn = (tid & 7) * TE;
#pragma unroll
        for (int q = 0; q < TE; ++q) Bs[kk][nn + q] = t.b[q];
    } else {
        const int nn = tid >> 2, kk = (tid & 3) * TE;
#pragma unroll
        for (int q = 0; q < TE; ++q) Bs[kk + q][nn] = t.b[q];
    }
}

__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g, int kchunk, double* partials) {
    __shared__ double As[2][BK][LDP];
    __shared__ double Bs[2][BK][LDP];
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(g.K, kbeg + kchunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;

    double4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0, 0, 0, 0};

    Tile t;
    int buf = 0;
    if (kbeg < kend) {
        load_tiles(g, m0, n0, kbeg, kend, t);
        store_tiles(g, t, As[0], Bs[0]);
    }
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        const bool more = k0 + BK < kend;
        if (more) load_tiles(g, m0, n0, k0 + BK, kend, t);
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            const int kk = 4 * s + lg;
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[buf][kk][wm + i * 16 + li];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[buf][kk][wn + j * 16 + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64_16x16x4(av[i], bv[j], acc[i][j]);
        }
        if (more) store_tiles(g, t, As[buf ^ 1], Bs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
    }
    const bool split = gridDim.z > 1;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + i * 16 + mfma_row_f64(lg, v);
                const int col = n0 + wn + j * 16 + li;
                if (row < g.M && col < g.N) {
                    if (split) {
                        partials[((size_t)blockIdx.z * g.M + row) * g.N + col] = acc[i][j][v];
                    } else {
                        double* c = g.C + c_offset(g, row, col);
                        double val = g.alpha * acc[i][j][v];
                        if (g.beta != 0.0) val += g.beta * (*c);
                        *c = val;
                    }
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) gemm_reduce_kernel(GemmArgs g, int splits,
                                                          const double* partials) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t mn = (int64_t)g.M * g.N;
    if (t >= mn) return;
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += partials[(size_t)z * mn + t];
    const int row = (int)(t / g.N), col = (int)(t - (int64_t)row * g.N);
    double* c = g.C + c_offset(g, row, col);
    double val = g.alpha * s;
    if (g.beta != 0.0) val += g.beta * (*c);
    *c = val;
}

}  // namespace

void launch_gemm(const GemmArgs& g, int splits, double* partials, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return;
    if (g.K <= 0) splits = 1;
    if (splits < 1) splits = 1;
    int kchunk = g.K;
    if (splits > 1) {
        kchunk = ((ceil_div(g.K, splits) + BK - 1) / BK) * BK;
        splits = ceil_div(g.K, kchunk);
    }
    if (splits <= 1) {
        splits = 1;
        kchunk = g.K > 0 ? g.K : 1;
    }
    dim3 grid(ceil_div(g.M, BM), ceil_div(g.N, BN), splits);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, g, kchunk, partials);
    TTR_CHECK_LAUNCH();
    if (splits > 1) {
        const int64_t mn = (int64_t)g.M * g.N;
        hipLaunchKernelGGL(gemm_reduce_kernel, dim3(ceil_div(mn, 256)), dim3(256), 0, s, g, splits,
                           partials);
        TTR_CHECK_LAUNCH();
    }
}

}  // namespace ttr
