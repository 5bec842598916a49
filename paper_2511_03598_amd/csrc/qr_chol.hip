// Fast path of the thin QR: CholeskyQR2, or shifted CholeskyQR3 for
// ill-conditioned panels, all decided on the device.
//
//   gram    : per-block partial Grams G = S^T S (MFMA), written to a buffer;
//   reduce  : sums the partials in a fixed order (64 workgroups);
//   apply   : every workgroup factors the summed Gram, G = R^T R
//             (Cholesky), and forms R^{-1} in LDS -- the same deterministic
//             computation in each, so all take the same route -- then
//             Q_next = Q_prev R^{-1} for its row block (MFMA), plus the
//             partial Grams of Q_next when another pass follows.  Workgroup
//             0 records R and the route flags for the kernels after it.
//
// Pass 1 first tries the plain Cholesky and certifies the panel: every pivot
// must keep at least 1e-10 of its column's squared norm, i.e. the
// column-equilibrated condition number is below ~1e5 and CholeskyQR2 is as
// accurate as Householder QR (Yamamoto, Nakatsukasa, Yanagisawa, Fukaya
// 2015).  Otherwise it factors G + sI with the shift s = 11 (m b + b (b+1))
// u tr(G) of shifted CholeskyQR (Fukaya, Kannan, Nakatsukasa, Zhang,
// Yamamoto 2020), which makes Q1 = S R1^{-1} well enough conditioned for two
// more passes (three in total).  Every route ends with diag(R) > 0, i.e.
// the unique thin-QR Q of a full-rank panel.  A pass whose Cholesky breaks
// down (a rank-deficient panel) raises the fallback flag: the panel is left
// untouched and the Householder TSQR (qr.hip) runs in its place.
#include <algorithm>

#include "kernels.hpp"

namespace ttr {
namespace {

constexpr int TB = 64;       // rows per LDS tile
constexpr int LDT = 64 + 1;  // padded row stride (doubles)

// flags[0]: 1 = fall back to Householder; flags[1]: 1 = shifted route;
// flags[2]: bit p-2 set when pass p used the near-identity factor.
struct CqDev {
    int m, b, lda, P;
    double* a;      // panel (m x b, column-major, lda): S in, Q out
    double* q1;     // m x b temporaries (ld m)
    double* q2;
    double* gpart;  // P x 64 x 64 partial Grams
    double* g;      // 64 x 64 summed Gram of the current pass
    double* rfac;   // 3 x 64 x 64 R per pass (row-major, identity-padded)
    double* r_out;  // optional b x b column-major R of the panel
    int* flags;
    int* sticky;    // optional: set to 1 as well when a pass breaks down
};

__device__ __forceinline__ void block_rows(const CqDev& q, int blk, int& r0, int& r1) {
    r0 = (int)(((int64_t)blk * q.m) / q.P);
    r1 = (int)(((int64_t)(blk + 1) * q.m) / q.P);
}

// acc (wave w: G rows w*16.., all 64 cols) += T^T T for an LDS tile T
// (TB rows x 64 cols, row stride LDT, zero padded).
__device__ __forceinline__ void gram_tile(const double* T, double4_t acc[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < TB; kk += 4) {
        const double* row = T + (kk + lg) * LDT;
        const double av = row[w * 16 + li];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma_f64_16x16x4(av, row[nb * 16 + li], acc[nb]);
    }
}

// T (TB rows x 64 cols, zero padded) <- rows [r, r_end) of the column-major
// panel, in two halves so the loads can be issued early.  Indices are
// clamped so every load is issued unconditionally (a masked load would
// serialise on its own wait); the padding is selected when storing.  256
// threads, 16 loads each.
__device__ __forceinline__ void load_regs(const double* src, int ld, int r, int r_end, int b,
                                          double (&v)[16]) {
    const int i = threadIdx.x & (TB - 1), c0 = threadIdx.x / TB;
    const int row = min(r + i, r_end - 1);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int c = min(c0 + 4 * e, b - 1);
        v[e] = src[(size_t)c * ld + row];
    }
}
__device__ __forceinline__ void store_regs(double* T, const double (&v)[16], int r, int r_end,
                                           int b) {
    const int i = threadIdx.x & (TB - 1), c0 = threadIdx.x / TB;
    const bool row_ok = (r + i) < r_end;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int c = c0 + 4 * e;
        T[i * LDT + c] = (row_ok && c < b) ? v[e] : 0.0;
    }
}
__device__ __forceinline__ void load_tile(const double* src, int ld, int r, int r_end, int b,
                                          double* T) {
    double v[16];
    load_regs(src, ld, r, r_end, b, v);
    store_regs(T, v, r, r_end, b);
}

__device__ __forceinline__ void store_partial(double* gp, const double4_t acc[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = w * 16 + mfma_row_f64(lg, v), j = nb * 16 + li;
            gp[i * 64 + j] = acc[nb][v];
        }
}

__global__ void __launch_bounds__(256) cq_gram_kernel(CqDev q) {
    // route flags of this QR start at zero (read only by later kernels)
    if (blockIdx.x == 0 && threadIdx.x < 3) q.flags[threadIdx.x] = 0;
    __shared__ double T[TB * LDT];
    int r0, r1;
    block_rows(q, blockIdx.x, r0, r1);
    double4_t acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = double4_t{0, 0, 0, 0};
    for (int r = r0; r < r1; r += TB) {
        __syncthreads();
        load_tile(q.a, q.lda, r, r1, q.b, T);
        __syncthreads();
        gram_tile(T, acc);
    }
    store_partial(q.gpart + (size_t)blockIdx.x * 4096, acc);
}

// ---------------------------------------------------------------------------
// Cholesky G + sI = L L^T (L = R^T) and X = L^{-1} of the 64 x 64 Gram, in
// LDS, by 256 threads (4 waves), blocked by 16 columns; lane i is row i.
//   panel kb: wave kb factors columns 16kb .. 16kb+15 for all rows with no
//     barrier.  Per pivot k the column-k values of the 16 diagonal-block rows
//     go through LDS to every lane (the LDS accesses of one wave complete in
//     order): L(i,k) = a(i,k)/sqrt(d_k), a(i,j) -= L(i,k) L(j,k), with the
//     next pivot's reciprocal square root overlapping the exchange;
//   one barrier; then wave w > kb subtracts the panel's rank-16 product from
//     its own block column (MFMA) while wave kb inverts its diagonal block
//     (lane c: column c of L_kk^{-1} by forward substitution, no exchange)
//     and forms the rest of block row kb of X from
//     X_kj = -X_kk sum_{m=j}^{k-1} L_km X_mj (MFMA), which only needs blocks
//     finished before the barrier.  The sums of the last block row are formed
//     by the idle waves while the last diagonal block is inverted.
// Padding beyond b is the identity, so L and X are the identity there; only
// the ceil(b/16) panels that hold columns of G are factored.
// ---------------------------------------------------------------------------
struct __align__(16) FactorLds {
    double L[64 * LDT];  // working matrix, then L (zero above the diagonal)
    double X[64 * LDT];  // L^{-1} (zero above the diagonal)
    double col[2][128];  // column exchange of the panel wave (two values per row)
    double d0[64];       // diagonal of G + sI (pivot certificate)
    double sinv[64];     // 1 / L(k,k)
};

// L <- G + sI (first b diagonal entries shifted), identity-padded; X <- 0
// with identity diagonal blocks past the factored panels.  All loads of a
// thread are issued before the first store.
__device__ __forceinline__ void factor_init(const double* G, double shift, int b, int nkb,
                                            FactorLds& F) {
    double gv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = threadIdx.x + 256 * e, i = t >> 6, j = t & 63;
        gv[e] = G[(i < b && j < b) ? t : 0];
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = threadIdx.x + 256 * e, i = t >> 6, j = t & 63;
        double v = (i < b && j < b) ? gv[e] : (i == j ? 1.0 : 0.0);
        if (i == j && i < b) v += shift;
        F.L[i * LDT + j] = v;
        F.X[i * LDT + j] = (i == j && i >= 16 * nkb) ? 1.0 : 0.0;
        if (i == j) F.d0[i] = v;
    }
    __syncthreads();
}

__device__ __forceinline__ int pivot_fails(double piv, double d0, double rel) {
    return !(d0 > 0.0 && piv > rel * d0 && piv < INFINITY);
}

// Panel kb by its own wave.  Returns 1 if a pivot falls to <= rel * (its
// value in G + sI) or is not finite.  Two chains run side by side: at pivot
// k, columns k+1 and k+2 are updated first and published together (the
// exchange brings column k+1 at the block's rows and the diagonal entry of
// column k+2), and the pivot of step k+1 is formed from uniform values by
// the same operation its owner applies (bit-identical), so its reciprocal
// square root overlaps the exchange; the rest of the update follows.
__device__ __forceinline__ int factor_panel(FactorLds& F, int kb, double rel) {
    const int i = threadIdx.x & 63;
    const int c0 = 16 * kb;
    double a[16], dd0[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        a[jj] = F.L[i * LDT + c0 + jj];
        dd0[jj] = F.d0[c0 + jj];
    }
    double c[16];  // column kk at the block's rows jj > kk
    double dn;     // diagonal entry of column kk+1 before step kk
    double s;      // 1 / sqrt(pivot kk)
    {
        double2_t* cb = reinterpret_cast<double2_t*>(F.col[0]);
        cb[i] = double2_t{a[0], a[1]};
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) c[jj] = F.col[0][2 * (c0 + jj)];
        dn = F.col[0][2 * (c0 + 1) + 1];
    }
    int bad = pivot_fails(c[0], dd0[0], rel);
    s = rsqrt_nr(fmax(c[0], 1e-300));
    double sv = 0.0;  // lane jj < 16 keeps 1/L(c0+jj, c0+jj)
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        sv = (i == kk) ? s : sv;
        const double li = a[kk] * s;
        const double t = li * s;
        a[kk] = li;
        double cn[16], dnn = 0.0, s_next = 0.0;
        if (kk < 15) {
            a[kk + 1] = fma(-t, c[kk + 1], a[kk + 1]);
            if (kk < 14) a[kk + 2] = fma(-t, c[kk + 2], a[kk + 2]);
            double* cb = F.col[(kk + 1) & 1];
            reinterpret_cast<double2_t*>(cb)[i] = double2_t{a[kk + 1], kk < 14 ? a[kk + 2] : 0.0};
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int jj = kk + 2; jj < 16; ++jj) cn[jj] = cb[2 * (c0 + jj)];
            if (kk < 14) dnn = cb[2 * (c0 + kk + 2) + 1];
            __builtin_amdgcn_sched_barrier(0);
            // pivot kk+1 as its owner forms it
            const double piv = fma(-((c[kk + 1] * s) * s), c[kk + 1], dn);
            bad |= pivot_fails(piv, dd0[kk + 1], rel);
            s_next = rsqrt_nr(fmax(piv, 1e-300));
        }
#pragma unroll
        for (int jj = kk + 3; jj < 16; ++jj) a[jj] = fma(-t, c[jj], a[jj]);
#pragma unroll
        for (int jj = kk + 2; jj < 16; ++jj) c[jj] = cn[jj];
        dn = dnn;
        s = s_next;
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) F.L[i * LDT + c0 + jj] = (i >= c0 + jj) ? a[jj] : 0.0;
    if (i < 16) F.sinv[c0 + i] = sv;
    return bad;
}

// Wave w > kb: block column w (rows 16w..63) -= L(:, panel kb) L(w rows,
// panel kb)^T.  The (up to three) tiles are computed together, clamped
// duplicates discarded.
__device__ __forceinline__ void update_block_column(FactorLds& F, int kb, int w) {
    const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
    const int p0 = 16 * kb, c0 = 16 * w;
    double4_t acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
        const double bv = F.L[(c0 + li) * LDT + p0 + k4 + lg];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int ti = min(w + t, 3);
            acc[t] = mfma_f64_16x16x4(F.L[(16 * ti + li) * LDT + p0 + k4 + lg], bv, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (w + t < 4) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                F.L[(16 * (w + t) + mfma_row_f64(lg, v)) * LDT + c0 + li] -= acc[t][v];
        }
    }
}

// X_kk = L_kk^{-1}; lane c solves L_kk x = e_c.
__device__ __forceinline__ void invert_diag(FactorLds& F, int kb) {
    const int lane = threadIdx.x & 63, c = lane & 15;
    const int c0 = 16 * kb;
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const double* lr = F.L + (c0 + r) * LDT + c0;
        double acc0 = (r == c) ? 1.0 : 0.0, acc1 = 0.0;
#pragma unroll
        for (int j = 0; j < r; ++j) {
            if (j & 1)
                acc1 = fma(-lr[j], x[j], acc1);
            else
                acc0 = fma(-lr[j], x[j], acc0);
        }
        x[r] = (acc0 + acc1) * F.sinv[c0 + r];
    }
    if (lane < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) F.X[(c0 + r) * LDT + c0 + c] = x[r];
    }
}

// U = sum_{m=j}^{k-1} L_km X_mj (one wave; accumulator layout).
__device__ __forceinline__ double4_t xblock_sum(const FactorLds& F, int k, int j) {
    const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
    double4_t u = {0.0, 0.0, 0.0, 0.0};
    for (int m = j; m < k; ++m) {
#pragma unroll
        for (int k4 = 0; k4 < 16; k4 += 4) {
            const double av = F.L[(16 * k + li) * LDT + 16 * m + k4 + lg];
            const double bv = F.X[(16 * m + k4 + lg) * LDT + 16 * j + li];
            u = mfma_f64_16x16x4(av, bv, u);
        }
    }
    return u;
}
// X_kj = -X_kk U, with U passed through the block's own place in X.
__device__ __forceinline__ void xblock_finish(FactorLds& F, int k, int j, double4_t u) {
    const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
    double* xkj = F.X + 16 * k * LDT + 16 * j;
#pragma unroll
    for (int v = 0; v < 4; ++v) xkj[mfma_row_f64(lg, v) * LDT + li] = u[v];
    __builtin_amdgcn_wave_barrier();
    double4_t x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
        const double av = F.X[(16 * k + li) * LDT + 16 * k + k4 + lg];
        const double bv = xkj[(k4 + lg) * LDT + li];
        x = mfma_f64_16x16x4(av, bv, x);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int v = 0; v < 4; ++v) xkj[mfma_row_f64(lg, v) * LDT + li] = -x[v];
}

// Returns 1 (block-wide) if the certificate or the factorization fails.
__device__ int chol_factor(const double* G, double shift, double rel, int b, FactorLds& F) {
    const int nkb = (b + 15) / 16, last = nkb - 1;
    factor_init(G, shift, b, nkb, F);
    const int w = threadIdx.x >> 6;
    int bad = 0;
    for (int kb = 0; kb < nkb; ++kb) {
        if (w == kb) bad |= factor_panel(F, kb, rel);
        __syncthreads();
        if (w == kb) {
            invert_diag(F, kb);
            if (kb < last)
                for (int j = kb - 1; j >= 0; --j) xblock_finish(F, kb, j, xblock_sum(F, kb, j));
        } else if (w > kb) {
            update_block_column(F, kb, w);
        }
    }
    // last block row: sums by the waves left of it, then X_last,j = -X_last,last U_j
    double4_t u = {0.0, 0.0, 0.0, 0.0};
    if (w < last) u = xblock_sum(F, last, w);
    __syncthreads();
    if (w < last) xblock_finish(F, last, w, u);
    return __syncthreads_or(bad);
}

// Factor of a Gram within 1e-9 of the identity (the second pass of
// CholeskyQR2, or the third of the shifted route, on a well-conditioned
// panel), without the pivot chain.  With G = I + E and U the strict upper
// triangle of E plus half its diagonal, the exact factor is R = I + U -
// U(R'^T R') with R' = R - I, and (I + U)^{-1} = I - U + U^2 - ..., so
// R = I + U and R^{-1} = I - U are exact up to entries of 64 max|E|^2 <=
// 6.4e-17, below the rounding of the factorization they replace.  Fills
// F.L = R^T and F.X = R^{-T} as chol_factor does and returns true, or
// returns false (F untouched) when some |E_ij| exceeds 1e-9 or is not
// finite.  Block-uniform; every thread must call it.
__device__ bool near_identity_factor(const double* G, int b, FactorLds& F) {
    double gv[16];
    bool fine = true;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = threadIdx.x + 256 * e, i = t >> 6, j = t & 63;
        gv[e] = (i < b && j < b) ? G[t] : (i == j ? 1.0 : 0.0);
        fine = fine && fabs(gv[e] - (i == j ? 1.0 : 0.0)) <= 1e-9;
    }
    if (!__syncthreads_and(fine)) return false;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = threadIdx.x + 256 * e, i = t >> 6, j = t & 63;
        const double u = (i > j) ? gv[e] : (i == j ? 0.5 * (gv[e] - 1.0) : 0.0);
        F.L[i * LDT + j] = (i > j) ? u : (i == j ? 1.0 + u : 0.0);
        F.X[i * LDT + j] = (i > j) ? -u : (i == j ? 1.0 - u : 0.0);
    }
    __syncthreads();
    return true;
}

// Sum of the P partial Grams: 64 workgroups of 64 entries; wave g sums the
// partials p in [g P/4, (g+1) P/4) in order (all loads issued together, 16
// at a time), and the four group sums are added in the order g = 0..3.
// Pass 3 runs only on the shifted route.
__global__ void __launch_bounds__(256) cq_reduce_kernel(CqDev q, int pass) {
    if (q.flags[0]) return;
    if (pass == 3 && !q.flags[1]) return;
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int p0 = (g * q.P) / 4, p1 = ((g + 1) * q.P) / 4;
    double s = 0.0;
    for (int p = p0; p < p1; p += 16) {
        double v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = q.gpart[(size_t)min(p + t, p1 - 1) * 4096 + e];
#pragma unroll
        for (int t = 0; t < 16; ++t)
            if (p + t < p1) s += v[t];
    }
    part[g][lane] = s;
    __syncthreads();
    if (g == 0) q.g[e] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// Pass p (1..3): factor the pass's Gram (pass 1 with the certificate and,
// if it fails, the shifted retry; pass 2 with the 0.5 certificate on the
// plain route; pass 3 only on the shifted route; passes 2 and 3 by the
// near-identity factor when their Gram allows), then out = src * R^{-1}
// per row block (MFMA) with the partial Grams of out when another pass
// follows.  Pass 1 reads S and writes Q1; pass 2 reads Q1 and writes Q2 or,
// on the plain route, the final Q into the panel; pass 3 reads Q2 and writes
// the final Q.  On a failed factorization nothing is written but the flag.
__global__ void __launch_bounds__(256) cq_apply_kernel(CqDev q, int pass) {
    if (q.flags[0]) return;
    const bool shifted_in = q.flags[1] != 0;  // meaningful from pass 2 on
    if (pass == 3 && !shifted_in) return;
    __shared__ FactorLds F;
    __shared__ double T[TB * LDT];
    const int tid = threadIdx.x, b = q.b;
    const double* src = (pass == 1) ? q.a : (pass == 2 ? q.q1 : q.q2);
    const int lds = (pass == 1) ? q.lda : q.m;
    int r0, r1;
    block_rows(q, blockIdx.x, r0, r1);
    // the first row tile is requested before the factorization, which hides
    // its latency
    double v[16];
    if (r0 < r1) load_regs(src, lds, r0, r1, b, v);

    double shift = 0.0;
    double rel = (pass == 1) ? 1e-10 : ((pass == 2 && !shifted_in) ? 0.5 : 0.0);
    int bad = 0;
    // a later pass whose Gram is within 1e-9 of I needs no pivot chain
    const bool near_id = pass >= 2 && near_identity_factor(q.g, b, F);
#pragma unroll 1
    for (int attempt = 0; !near_id; ++attempt) {
        bad = chol_factor(q.g, shift, rel, b, F);
        if (pass != 1 || !bad || attempt == 1) break;
        double tr = 0.0;
        for (int j = 0; j < b; ++j) tr += F.d0[j];
        shift = 11.0 * ((double)q.m * b + (double)b * (b + 1)) * 1.1102230246251565e-16 * tr;
        rel = 0.0;
        __syncthreads();  // d0 is read before the retry overwrites it
    }
    const bool shifted = (pass == 1) ? (shift > 0.0) : shifted_in;
    if (blockIdx.x == 0) {
        if (tid == 0 && bad) {
            q.flags[0] = 1;
            if (q.sticky) *q.sticky = 1;
        }
        if (tid == 0 && pass == 1) q.flags[1] = shifted ? 1 : 0;
        if (tid == 0 && near_id) q.flags[2] |= 1 << (pass - 2);
        double* rf = q.rfac + (size_t)(pass - 1) * 4096;  // R(j, i) = L(i, j)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = tid + 256 * e, j = t >> 6, i = t & 63;
            rf[t] = (i >= j) ? F.L[i * LDT + j] : 0.0;
        }
    }
    if (bad) return;  // block-uniform; the panel stays as it was
    // R^{-1} = X^T, row-major into the space of L (which is no longer needed)
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = tid + 256 * e, k = t >> 6, c = t & 63;
        F.L[k * LDT + c] = F.X[c * LDT + k];
    }

    const bool final_pass = (pass == 3) || (pass == 2 && !shifted);
    const bool gram = !final_pass;
    double* dst = final_pass ? q.a : (pass == 1 ? q.q1 : q.q2);
    const int ldd = final_pass ? q.lda : q.m;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    double4_t gacc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) gacc[nb] = double4_t{0, 0, 0, 0};
    for (int r = r0; r < r1; r += TB) {
        if (r > r0) load_regs(src, lds, r, r1, b, v);
        __syncthreads();
        store_regs(T, v, r, r1, b);
        __syncthreads();
        double4_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = double4_t{0, 0, 0, 0};
        // R^{-1} is upper triangular: column block nb only needs k < 16 (nb + 1)
#pragma unroll
        for (int kb4 = 0; kb4 < 4; ++kb4) {
#pragma unroll 2
            for (int k4 = 0; k4 < 16; k4 += 4) {
                const int kk = 16 * kb4 + k4;
                const double av = T[(w * 16 + li) * LDT + kk + lg];
#pragma unroll
                for (int nb = kb4; nb < 4; ++nb)
                    acc[nb] = mfma_f64_16x16x4(av, F.L[(kk + lg) * LDT + nb * 16 + li], acc[nb]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                const int i = w * 16 + mfma_row_f64(lg, vv), c = nb * 16 + li;
                const int row = r + i;
                const bool ok = (row < r1 && c < q.b);
                if (ok) dst[(size_t)c * ldd + row] = acc[nb][vv];
                T[i * LDT + c] = ok ? acc[nb][vv] : 0.0;
            }
        if (gram) {
            __syncthreads();
            gram_tile(T, gacc);
        }
    }
    if (gram) store_partial(q.gpart + (size_t)blockIdx.x * 4096, gacc);
}

// R of the panel: R = R_last ... R_1 (upper triangular, identity-padded),
// written column-major b x b.  One workgroup; each product is a 64x64x64
// MFMA (f64 16x16x4) from LDS, wave w computing rows 16w .. 16w+15.
__global__ void __launch_bounds__(256) cq_rout_kernel(CqDev q) {
    if (q.flags[0]) return;
    const int npass = q.flags[1] ? 3 : 2;
    const int b = q.b, tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6, li = lane & 15, lg = lane >> 4;
    __shared__ double A[64 * LDT];
    __shared__ double B[64 * LDT];
    // all loads of a matrix are issued before its LDS stores
    double ra[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) ra[e] = q.rfac[tid + 256 * e];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = tid + 256 * e;
        A[(t >> 6) * LDT + (t & 63)] = ra[e];
    }
    for (int p = 1; p < npass; ++p) {
#pragma unroll
        for (int e = 0; e < 16; ++e) ra[e] = q.rfac[(size_t)p * 4096 + tid + 256 * e];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = tid + 256 * e;
            B[(t >> 6) * LDT + (t & 63)] = ra[e];
        }
        __syncthreads();
        // C = B A
        double4_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = double4_t{0, 0, 0, 0};
#pragma unroll 4
        for (int kk = 0; kk < 64; kk += 4) {
            const double bv = B[(w * 16 + li) * LDT + kk + lg];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[nb] = mfma_f64_16x16x4(bv, A[(kk + lg) * LDT + nb * 16 + li], acc[nb]);
        }
        __syncthreads();
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                A[(w * 16 + mfma_row_f64(lg, v)) * LDT + nb * 16 + li] = acc[nb][v];
        __syncthreads();
    }
    // column-major b x b: thread (column tid/4, rows tid%4 + 4u)
    {
        const int col = tid >> 2;
        if (col < b)
            for (int i = tid & 3; i < b; i += 4) q.r_out[(size_t)col * b + i] = (i <= col) ? A[i * LDT + col] : 0.0;
    }
}

}  // namespace

namespace {
int cq_blocks(int m) { return std::max(1, std::min(64, ceil_div(m, TB))); }
}  // namespace

size_t cq_workspace_doubles(int m, int b) {
    return 2 * (size_t)m * b + (size_t)cq_blocks(m) * 4096 + 4 * 4096 + 64;
}

void launch_cq(double* a, int m, int b, int lda, double* r_out, double* ws, int* flags,
               hipStream_t s, int* sticky) {
    CqDev q{};
    q.m = m;
    q.b = b;
    q.lda = lda;
    q.P = cq_blocks(m);
    q.a = a;
    q.q1 = ws;
    q.q2 = ws + (size_t)m * b;
    q.gpart = q.q2 + (size_t)m * b;
    q.g = q.gpart + (size_t)q.P * 4096;
    q.rfac = q.g + 4096;
    q.r_out = r_out;
    q.flags = flags;
    q.sticky = sticky;
    hipLaunchKernelGGL(cq_gram_kernel, dim3(q.P), dim3(256), 0, s, q);
    TTR_CHECK_LAUNCH();
    for (int pass = 1; pass <= 3; ++pass) {
        hipLaunchKernelGGL(cq_reduce_kernel, dim3(64), dim3(256), 0, s, q, pass);
        TTR_CHECK_LAUNCH();
        hipLaunchKernelGGL(cq_apply_kernel, dim3(q.P), dim3(256), 0, s, q, pass);
        TTR_CHECK_LAUNCH();
    }
    if (r_out != nullptr) {
        hipLaunchKernelGGL(cq_rout_kernel, dim3(1), dim3(256), 0, s, q);
        TTR_CHECK_LAUNCH();
    }
}

}  // namespace ttr
