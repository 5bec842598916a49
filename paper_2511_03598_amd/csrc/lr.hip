// Left-to-right KRP partial contractions (Sec. 3.1, the recurrence of the
// right-to-left contractions taken from the first core onwards):
//   W^L_k(b, c) = sum_{a, i} X_k(a, i, b) W^L_{k-1}(a, c) Omega_k(i, c),
// W^L_0 = 1.  Core by core this is the tall contraction V(X_k)^T K_k with
// K_k the Khatri-Rao product whose row (a, i) is W^L_{k-1}(a, :) times
// Omega_k(i, :) elementwise; K_k is formed in registers as its rows are
// consumed and never stored.  V(X_k) (r_{k-1} n_k x r_k, rows contiguous) is
// streamed once; W^L_{k-1} and Omega_k are small and stay in cache.
//
// MFMA f64 16x16x4: a 32 (b) x 64 (c) output tile per 256-thread workgroup,
// the k range of a workgroup taken in chunks of 64 rows (a, i) of which
// each wave multiplies a quarter, operands loaded from global memory
// straight into MFMA layout one chunk ahead of its MFMAs.  The four wave
// tiles are added in LDS in a fixed order; split-K slices are summed by a
// second kernel in slice order, so results do not depend on timing.
#include <algorithm>

#include "kernels.hpp"

namespace ttr {
namespace {

constexpr int LR_TM = 32, LR_TN = 64;
constexpr int LR_DKW = 4;                 // k-steps of 4 per wave and chunk
constexpr int LR_CHUNK = 16 * LR_DKW;     // rows (a, i) per chunk (4 waves)

// One chunk's operands for this lane: rows (a, i) = kb + 4 (ks0 + t) + lg
// of V(X_k) (clamped into the slice; copies past it are never multiplied)
// and the matching Khatri-Rao entries W^L_{k-1}(a, c) Omega_k(i, c).
struct LrOps {
    double a[LR_DKW][2], b[LR_DKW][4];
};

template <bool FIRST>
__device__ __forceinline__ void lr_load(const LrArgs& g, int kb, int ks0, int kend, const int (&rows)[2],
                                        const int (&cols)[4], int lg, LrOps& o) {
#pragma unroll
    for (int t = 0; t < LR_DKW; ++t) {
        const int kc = min(kb + 4 * (ks0 + t) + lg, kend - 1);
        const int a = FIRST ? 0 : (int)((unsigned)kc / (unsigned)g.n);
        const int i = kc - a * g.n;
        const double* xr = g.X + (size_t)kc * g.r1;
        const double* orow = g.Om + (size_t)i * g.ldo;
#pragma unroll
        for (int u = 0; u < 2; ++u) o.a[t][u] = xr[rows[u]];
        if (FIRST) {
#pragma unroll
            for (int j = 0; j < 4; ++j) o.b[t][j] = orow[cols[j]];
        } else {
            const double* wrow = g.Wp + (size_t)a * g.ldw;
#pragma unroll
            for (int j = 0; j < 4; ++j) o.b[t][j] = wrow[cols[j]] * orow[cols[j]];
        }
    }
}

// The wave's k-steps [ks0, ks1) of the chunk at kb: its quarter of the
// chunk's k-steps of 4 rows.
__device__ __forceinline__ void lr_split(int kb, int kend, int w, int& ks0, int& ks1) {
    const int nks = (min(kend - kb, LR_CHUNK) + 3) / 4;
    ks0 = (w * nks) / 4;
    ks1 = ((w + 1) * nks) / 4;
}

// Split-K: slice z = blockIdx.z takes rows [z kchunk, (z+1) kchunk) and
// writes its tile to partials[z] (r1 x nc) for lr_reduce_kernel; without
// partials the one slice covers every row and writes W directly.  (Summing
// the slices in the last slice to finish would need a device-wide release
// per workgroup, an L2 write-back on this chip that costs more than the
// second launch.)
template <bool FIRST>
__global__ void __launch_bounds__(256) lr_kernel(LrArgs g, int kchunk, double* partials) {
    __shared__ double red[2][LR_TM][LR_TN + 1];
    const int m0 = blockIdx.x * LR_TM, n0 = blockIdx.y * LR_TN;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int K = g.r0 * g.n;
    int rows[2], cols[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) rows[i] = min(m0 + 16 * i + li, g.r1 - 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) cols[j] = min(n0 + 16 * j + li, g.nc - 1);
    double4_t acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = double4_t{0, 0, 0, 0};

    // two chunks in flight: the next chunk's loads are issued before the
    // current chunk's MFMAs
    const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
    LrOps cur, nxt;
    int ks0 = 0, ks1 = 0;
    if (kbeg < kend) {
        lr_split(kbeg, kend, w, ks0, ks1);
        lr_load<FIRST>(g, kbeg, ks0, kend, rows, cols, lg, cur);
    }
    for (int kb = kbeg; kb < kend; kb += LR_CHUNK) {
        int ns0 = 0, ns1 = 0;
        const bool more = kb + LR_CHUNK < kend;
        if (more) {
            lr_split(kb + LR_CHUNK, kend, w, ns0, ns1);
            lr_load<FIRST>(g, kb + LR_CHUNK, ns0, kend, rows, cols, lg, nxt);
        }
#pragma unroll
        for (int t = 0; t < LR_DKW; ++t) {
            const int ks = ks0 + t;
            if (ks < ks1) {  // uniform per wave
                const bool kok = kb + 4 * ks + lg < kend;
                const double a0 = kok ? cur.a[t][0] : 0.0, a1 = kok ? cur.a[t][1] : 0.0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[0][j] = mfma_f64_16x16x4(a0, cur.b[t][j], acc[0][j]);
                    acc[1][j] = mfma_f64_16x16x4(a1, cur.b[t][j], acc[1][j]);
                }
            }
        }
        if (more) {
            cur = nxt;
            ks0 = ns0;
            ks1 = ns1;
        }
    }
    // wave tiles: (w0 + w2) + (w1 + w3)
    if (w < 2) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[w][16 * i + mfma_row_f64(lg, v)][16 * j + li] = acc[i][j][v];
    }
    __syncthreads();
    if (w >= 2) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[w - 2][16 * i + mfma_row_f64(lg, v)][16 * j + li] += acc[i][j][v];
    }
    __syncthreads();
    constexpr int E = (LR_TM * LR_TN) / 256;
    if (!partials) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + 256 * e, r = idx / LR_TN, c = idx % LR_TN;
            const int row = m0 + r, col = n0 + c;
            if (row < g.r1 && col < g.nc) g.W[(size_t)row * g.ldwo + col] = red[0][r][c] + red[1][r][c];
        }
        return;
    }
    const size_t mn = (size_t)g.r1 * g.nc;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = threadIdx.x + 256 * e, r = idx / LR_TN, c = idx % LR_TN;
        const int row = m0 + r, col = n0 + c;
        if (row < g.r1 && col < g.nc)
            partials[blockIdx.z * mn + (size_t)row * g.nc + col] = red[0][r][c] + red[1][r][c];
    }
}

// W(row, col) = sum over slices z in order of partials[z](row, col).
__global__ void __launch_bounds__(256) lr_reduce_kernel(LrArgs g, int splits, const double* partials) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t mn = (int64_t)g.r1 * g.nc;
    if (t >= mn) return;
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
    const int row = (int)(t / g.nc), col = (int)(t - (int64_t)row * g.nc);
    g.W[(size_t)row * g.ldwo + col] = s;
}

// Rows (a, i) per split-K slice: whole chunks, at least two per wave pass.
int lr_kchunk(int K, int splits) { return ceil_div(ceil_div(K, splits), LR_CHUNK) * LR_CHUNK; }

}  // namespace

int lr_splits(int r0, int n, int r1, int nc) {
    const int64_t K = (int64_t)r0 * n;
    if (K <= 0 || r1 <= 0 || nc <= 0) return 1;
    const int tiles = ceil_div(r1, LR_TM) * ceil_div(nc, LR_TN);
    // about two workgroups per compute unit, slices of >= 4 chunks
    const int want = std::max(1, ceil_div(512, tiles));
    const int most = std::max(1, ceil_div(K, 4 * LR_CHUNK));
    const int s = std::min({want, most, 256});
    return ceil_div(K, lr_kchunk((int)K, s));  // slices actually used
}

void launch_lr(const LrArgs& g, int splits, double* partials, hipStream_t s) {
    if (g.r1 <= 0 || g.nc <= 0) return;
    const int K = g.r0 * g.n;
    if (K <= 0) throw Error(-1, "empty left-to-right contraction");
    if (splits < 1 || (splits > 1 && !partials)) splits = 1;
    const int kchunk = splits > 1 ? lr_kchunk(K, splits) : K;
    const int nz = ceil_div(K, kchunk);
    dim3 grid(ceil_div(g.r1, LR_TM), ceil_div(g.nc, LR_TN), nz);
    double* part = nz > 1 ? partials : nullptr;
    if (g.Wp)
        hipLaunchKernelGGL((lr_kernel<false>), grid, dim3(256), 0, s, g, kchunk, part);
    else
        hipLaunchKernelGGL((lr_kernel<true>), grid, dim3(256), 0, s, g, kchunk, part);
    TTR_CHECK_LAUNCH();
    if (nz > 1) {
        const int64_t mn = (int64_t)g.r1 * g.nc;
        hipLaunchKernelGGL(lr_reduce_kernel, dim3(ceil_div(mn, 256)), dim3(256), 0, s, g, nz, part);
        TTR_CHECK_LAUNCH();
    }
}


}  // namespace ttr
