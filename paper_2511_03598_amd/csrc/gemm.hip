// General float64 GEMM on MFMA (v_mfma_f64_16x16x4_f64) for the
// randomize-then-orthogonalize sweep (Sec. 3.2-3.3): the sketch
// S_k = V(Y_k) W_{k+1}, the projections Q^T S and Q^T V(Y_k), the next core
// M_k H(X_{k+1}) and the recompression products.
//
// 64x64 output tile per 256-thread workgroup, K staged through LDS in
// 32-deep double-buffered slabs with two more slabs in flight in registers
// (eight loads per operand and thread per slab), each wave owning a 32x32
// quadrant
// (2x2 MFMA blocks).  Operands are addressed by element strides so one
// kernel serves every transpose; the global->LDS thread mapping follows the
// contiguous dimension so loads stay coalesced.  Split-K writes partial
// tiles that a second kernel sums in a fixed order (deterministic).
#include <type_traits>

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

    // Three-stage pipeline: while slab k is multiplied from LDS, slab k+1
    // waits in registers (ta) and slab k+2 is being loaded (tb), so each
    // slab's global loads have two slabs of MFMA work to arrive.
    Tile ta, tb;
    int buf = 0;
    if (kbeg < kend) {
        load_tiles(g, m0, n0, kbeg, kend, ta);
        store_tiles(g, ta, As[0], Bs[0]);
        if (kbeg + BK < kend) load_tiles(g, m0, n0, kbeg + BK, kend, ta);
    }
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        const bool more = k0 + BK < kend;
        if (k0 + 2 * BK < kend) load_tiles(g, m0, n0, k0 + 2 * BK, kend, tb);
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
        if (more) store_tiles(g, ta, As[buf ^ 1], Bs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
        ta = tb;
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
    // slice order; eight loads issued together per step
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partials[(size_t)(z + u) * mn + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < splits; ++z) s += partials[(size_t)z * mn + t];
    const int row = (int)(t / g.N), col = (int)(t - (int64_t)row * g.N);
    double* c = g.C + c_offset(g, row, col);
    double val = g.alpha * s;
    if (g.beta != 0.0) val += g.beta * (*c);
    *c = val;
}

// ---------------------------------------------------------------------------
// Direct-operand kernel (K <= 256, or K <= 1024 on grids of >= 64 tiles): a
// 32x32 output tile per 256-thread workgroup; K is taken in chunks of up to
// 256, and within a chunk wave w multiplies its quarter of the k range for
// the whole tile (2x2 MFMA blocks), loading its operands from global memory
// straight into MFMA operand layout, all before the chunk's first MFMA (no
// LDS staging, no barrier); the four partial tiles are added in LDS in wave
// order.  With
// f64 MFMA issue as the bound, four waves per 32x32 tile finish a K = 200
// product about four times sooner than one 64x64 tile per workgroup, and the
// grid has four times as many workgroups.
// ---------------------------------------------------------------------------
constexpr int DKW_MAX = 16;  // k-steps of 4 per wave and chunk at most (chunks of 256)

// B's storage for the direct kernel: FP64, FP32 or bfloat16 (BT = 0, 1, 2),
// with per-column exponents 2^bexp[n] (EXP) and slices summed in slice order
// in the storage's arithmetic type (MS), as in load_b.  Compile-time choices
// keep every operand load unconditional, so they are all issued together.
template <int BT>
struct BStore;
template <>
struct BStore<0> {
    typedef double T;
    static __device__ __forceinline__ const double* ptr(const GemmArgs& g) { return g.B; }
};
template <>
struct BStore<1> {
    typedef float T;
    static __device__ __forceinline__ const float* ptr(const GemmArgs& g) { return g.Bf; }
};
template <>
struct BStore<2> {
    typedef unsigned short T;
    static __device__ __forceinline__ const unsigned short* ptr(const GemmArgs& g) { return g.Bh; }
};
__device__ __forceinline__ double stored_f64(const double* p, size_t i) { return p[i]; }
__device__ __forceinline__ float stored_f64(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float stored_f64(const unsigned short* p, size_t i) { return stored_f32(p, i); }

// DKW: k-steps of 4 per wave the kernel loads (4, 8 or 16: K <= 16 DKW),
// so short products do not issue loads they do not use.  Split-K: slice
// z = blockIdx.z takes k in [z kchunk, (z+1) kchunk) and writes its raw
// tile to partials[z] (M x N row-major) for gemm_reduce_kernel; without
// partials the one slice covers K and the tile goes to C.
template <int BT, bool EXP, bool MS, int DKW>
__global__ void __launch_bounds__(256) gemm_direct_kernel(GemmArgs g, int kchunk, double* partials) {
    typedef typename BStore<BT>::T ST;
    typedef typename std::conditional<BT == 0, double, float>::type AT;  // B's arithmetic type
    __shared__ double red[4][32][33];
    const int m0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const ST* Bp = BStore<BT>::ptr(g);
    // operands: A(m0 + 16 i + li, k), B(k, n0 + 16 j + li), k = 4 ks + lg
    int rows[2], cols[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        rows[i] = min(m0 + 16 * i + li, g.M - 1);
        cols[i] = min(n0 + 16 * i + li, g.N - 1);
    }
    int bex[2] = {0, 0};
    if (EXP) {
#pragma unroll
        for (int i = 0; i < 2; ++i) bex[i] = g.bexp[cols[i]];
    }
    double4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0, 0, 0, 0};
    // K in chunks of 16 DKW; within a chunk wave w takes its quarter of the
    // k-steps
    const int kbeg = blockIdx.z * kchunk, kend = min(g.K, kbeg + kchunk);
    for (int kb = kbeg; kb < kend; kb += 16 * DKW) {
        const int nks = (min(kend - kb, 16 * DKW) + 3) / 4;
        const int ks0 = (w * nks) / 4, ks1 = ((w + 1) * nks) / 4;
        double av[DKW][2];
        AT bs[DKW][2];
#pragma unroll
        for (int t = 0; t < DKW; ++t) {
            const int kc = min(kb + 4 * (ks0 + t) + lg, kend - 1);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[t][i] = g.A[(size_t)rows[i] * g.sam + (size_t)kc * g.sak];
                bs[t][i] = stored_f64(Bp, (size_t)kc * g.sbk + (size_t)cols[i] * g.sbn);
            }
        }
        if (MS) {
            for (int sl = 1; sl < g.bslices; ++sl) {
                const ST* Bs = Bp + (size_t)sl * g.bstride;
#pragma unroll
                for (int t = 0; t < DKW; ++t) {
                    const int kc = min(kb + 4 * (ks0 + t) + lg, kend - 1);
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        bs[t][i] += stored_f64(Bs, (size_t)kc * g.sbk + (size_t)cols[i] * g.sbn);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < DKW; ++t) {
            const int ks = ks0 + t;
            if (ks < ks1) {  // uniform per wave
                // k beyond K: the clamped operands are finite copies; zero A's
                const bool kok = kb + 4 * ks + lg < kend;
                const double a0 = kok ? av[t][0] : 0.0, a1 = kok ? av[t][1] : 0.0;
                double b0 = (double)bs[t][0], b1 = (double)bs[t][1];
                if (EXP) {
                    b0 = ldexp(b0, bex[0]);
                    b1 = ldexp(b1, bex[1]);
                }
                acc[0][0] = mfma_f64_16x16x4(a0, b0, acc[0][0]);
                acc[0][1] = mfma_f64_16x16x4(a0, b1, acc[0][1]);
                acc[1][0] = mfma_f64_16x16x4(a1, b0, acc[1][0]);
                acc[1][1] = mfma_f64_16x16x4(a1, b1, acc[1][1]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[w][16 * i + mfma_row_f64(lg, v)][16 * j + li] = acc[i][j][v];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = threadIdx.x + 256 * e, r = idx >> 5, c = idx & 31;
        const int row = m0 + r, col = n0 + c;
        if (row < g.M && col < g.N) {
            const double sum = ((red[0][r][c] + red[1][r][c]) + red[2][r][c]) + red[3][r][c];
            if (partials) {
                partials[((size_t)blockIdx.z * g.M + row) * g.N + col] = sum;
                continue;
            }
            double* cp = g.C + c_offset(g, row, col);
            double val = g.alpha * sum;
            if (g.beta != 0.0) val += g.beta * (*cp);
            *cp = val;
        }
    }
}

template <int BT, bool EXP, int DKW>
void launch_direct_k(const GemmArgs& g, dim3 grid, int kchunk, double* partials, hipStream_t s) {
    if (g.bslices > 1)
        hipLaunchKernelGGL((gemm_direct_kernel<BT, EXP, true, DKW>), grid, dim3(256), 0, s, g, kchunk,
                           partials);
    else
        hipLaunchKernelGGL((gemm_direct_kernel<BT, EXP, false, DKW>), grid, dim3(256), 0, s, g, kchunk,
                           partials);
}
template <int BT, bool EXP>
void launch_direct(const GemmArgs& g, dim3 grid, int kchunk, double* partials, hipStream_t s) {
    const int per_wave = ceil_div(ceil_div(std::min(kchunk, 16 * DKW_MAX), 4), 4);  // busiest wave's k-steps
    if (per_wave <= 4)
        launch_direct_k<BT, EXP, 4>(g, grid, kchunk, partials, s);
    else if (per_wave <= 8)
        launch_direct_k<BT, EXP, 8>(g, grid, kchunk, partials, s);
    else
        launch_direct_k<BT, EXP, 16>(g, grid, kchunk, partials, s);
}

// ---------------------------------------------------------------------------
// K-segmented product (launch_seg_gemm): a 32x32 output tile per workgroup,
// wave w takes segments w, w+4, ... whole (the segment index is uniform per
// wave, so its table entries are scalar loads), each in 64-deep chunks with
// all operand loads of a chunk issued before its MFMAs; the four wave tiles
// are added in LDS in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) seg_gemm_kernel(SegGemm g) {
    __shared__ double red[4][32][33];
    const int m0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    int rows[2], cols[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        rows[i] = min(m0 + 16 * i + li, g.M - 1);
        cols[i] = min(n0 + 16 * i + li, g.N - 1);
    }
    double4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0, 0, 0, 0};
    for (int sg = w; sg < g.nseg; sg += 4) {
        const double* A = g.A[sg];
        const double* B = g.B[sg];
        const int64_t lda = g.lda[sg], ldb = g.ldb[sg], ss = g.ss[sg];
        const double al = g.alpha[sg];
        const int K = g.K[sg], nsl = g.slices[sg];
        for (int kb = 0; kb < K; kb += 64) {
            double av[16][2], bv[16][2];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int kc = min(kb + 4 * t + lg, K - 1);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    av[t][i] = A[(size_t)rows[i] * lda + kc];
                    bv[t][i] = B[(size_t)cols[i] * ldb + kc];
                }
            }
            for (int q = 1; q < nsl; ++q) {
                const double* Bq = B + (size_t)q * ss;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int kc = min(kb + 4 * t + lg, K - 1);
#pragma unroll
                    for (int i = 0; i < 2; ++i) bv[t][i] += Bq[(size_t)cols[i] * ldb + kc];
                }
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                if (kb + 4 * t < K) {  // uniform
                    const bool kok = kb + 4 * t + lg < K;
                    const double a0 = kok ? al * av[t][0] : 0.0, a1 = kok ? al * av[t][1] : 0.0;
                    acc[0][0] = mfma_f64_16x16x4(a0, bv[t][0], acc[0][0]);
                    acc[0][1] = mfma_f64_16x16x4(a0, bv[t][1], acc[0][1]);
                    acc[1][0] = mfma_f64_16x16x4(a1, bv[t][0], acc[1][0]);
                    acc[1][1] = mfma_f64_16x16x4(a1, bv[t][1], acc[1][1]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[w][16 * i + mfma_row_f64(lg, v)][16 * j + li] = acc[i][j][v];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = threadIdx.x + 256 * e, r = idx & 31, c = idx >> 5;
        const int row = m0 + r, col = n0 + c;
        if (row < g.M && col < g.N)
            g.C[(size_t)col * g.ldc + row] = ((red[0][r][c] + red[1][r][c]) + red[2][r][c]) + red[3][r][c];
    }
}

}  // namespace

void launch_seg_gemm(const SegGemm& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return;
    if (g.nseg < 1 || g.nseg > kSegGemmMax) throw Error(-1, "segmented GEMM: 1..16 segments");
    for (int i = 0; i < g.nseg; ++i)
        if (g.K[i] < 1 || g.slices[i] < 1) throw Error(-1, "segmented GEMM: empty segment");
    hipLaunchKernelGGL(seg_gemm_kernel, dim3(ceil_div(g.M, 32), ceil_div(g.N, 32)), dim3(256), 0, s, g);
    TTR_CHECK_LAUNCH();
}

namespace {
bool plain_direct(int M, int N, int K) {
    const int64_t dtiles = (int64_t)ceil_div(M, 32) * ceil_div(N, 32);
    return K >= 1 && (K <= 16 * DKW_MAX || (K <= 64 * DKW_MAX && dtiles >= 64));
}
bool split_direct(int M, int N, int K) { return !plain_direct(M, N, K) && (int64_t)M * N <= 65536; }
}  // namespace

int gemm_splits(int M, int N, int K) {
    if (M <= 0 || N <= 0 || K <= 0 || plain_direct(M, N, K)) return 1;
    // small outputs (e.g. Q^T V(Y_k)): direct tiles, one 256-deep chunk per
    // slice, with at most 2^18 partial doubles
    if (split_direct(M, N, K))
        return std::max(1, std::min({64, ceil_div(K, 16 * DKW_MAX), (int)(262144 / ((int64_t)M * N))}));
    // tiled kernel: enough workgroups to cover the chip, K slices of >= 128
    const int tiles = ceil_div(M, 64) * ceil_div(N, 64);
    if (tiles < 128 && K >= 512) return std::min(64, std::min(ceil_div(K, 128), std::max(1, 256 / tiles)));
    return 1;
}

void launch_gemm(const GemmArgs& g, int splits, double* partials, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return;
    // direct kernel: K <= 256, or K <= 1024 on a grid of at least 64 tiles,
    // or split over K when the output is small
    const bool split = split_direct(g.M, g.N, g.K) && splits > 1 && partials != nullptr;
    if (plain_direct(g.M, g.N, g.K) || split) {
        const int ns = split ? splits : 1;
        const int kchunk = split ? ceil_div(ceil_div(g.K, ns), 16) * 16 : g.K;
        const int nz = ceil_div(g.K, kchunk);  // <= ns
        dim3 grid(ceil_div(g.M, 32), ceil_div(g.N, 32), nz);
        double* part = split ? partials : nullptr;
        const bool ex = g.bexp != nullptr;
        if (g.Bf)
            ex ? launch_direct<1, true>(g, grid, kchunk, part, s) : launch_direct<1, false>(g, grid, kchunk, part, s);
        else if (g.Bh)
            ex ? launch_direct<2, true>(g, grid, kchunk, part, s) : launch_direct<2, false>(g, grid, kchunk, part, s);
        else
            launch_direct<0, false>(g, grid, kchunk, part, s);
        TTR_CHECK_LAUNCH();
        if (split) {
            const int64_t mn = (int64_t)g.M * g.N;
            hipLaunchKernelGGL(gemm_reduce_kernel, dim3(ceil_div(mn, 256)), dim3(256), 0, s, g, nz,
                               partials);
            TTR_CHECK_LAUNCH();
        }
        return;
    }
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
