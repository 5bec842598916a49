// Fast path of the thin QR: CholeskyQR2, or shifted CholeskyQR3 for
// ill-conditioned panels, all decided on the device.
//
//   gram    : per-block partial Grams G = S^T S (MFMA), written to a buffer;
//   chol    : one workgroup sums the partials in a fixed order, factors
//             G = R^T R (Cholesky), forms R^{-1} in the same sweep and sets
//             the route flags;
//   apply   : Q_next = Q_prev R^{-1} per row block (MFMA), plus the partial
//             Grams of Q_next when another pass follows.
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

// flags[0]: 1 = fall back to Householder; flags[1]: 1 = shifted route.
struct CqDev {
    int m, b, lda, P;
    double* a;      // panel (m x b, column-major, lda): S in, Q out
    double* q1;     // m x b temporaries (ld m)
    double* q2;
    double* gpart;  // P x 64 x 64 partial Grams
    double* rinv;   // 3 x 64 x 64 R^{-1} per pass (row-major, identity-padded)
    double* rfac;   // 3 x 64 x 64 R per pass
    double* r_out;  // optional b x b column-major R of the panel
    int* flags;
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
// panel.  Indices are clamped so every load is issued unconditionally (a
// masked load would serialise on its own wait); the padding is selected
// afterwards.  256 threads, 16 loads each.
__device__ __forceinline__ void load_tile(const double* src, int ld, int r, int r_end, int b,
                                          double* T) {
    const int i = threadIdx.x & (TB - 1), c0 = threadIdx.x / TB;
    const int row = min(r + i, r_end - 1);
    double v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int c = min(c0 + 4 * e, b - 1);
        v[e] = src[(size_t)c * ld + row];
    }
    const bool row_ok = (r + i) < r_end;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int c = c0 + 4 * e;
        T[i * LDT + c] = (row_ok && c < b) ? v[e] : 0.0;
    }
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
    if (blockIdx.x == 0 && threadIdx.x < 2) q.flags[threadIdx.x] = 0;
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

// Cholesky G = R^T R of the LDS matrix G0 (64 x LDT, identity-padded beyond
// b, `shift` added to the first b diagonal entries) together with R^{-1},
// 512 threads.  Lane i of every wave is row i.  Waves 0-3 hold columns
// 16w .. 16w+15 of G; waves 4-7 hold the same columns of an identity matrix
// A that the elimination turns into L^{-1} (L = R^T), so R^{-1} = (L^{-1})^T
// comes out of the same sweep.  Step k (k < b; padding steps are no-ops):
//   - wave k/16 publishes column k of G, lane k of each A wave publishes its
//     part of row k of A (double-buffered LDS, one barrier per step);
//   - L(i,k) = G(i,k)/sqrt(G(k,k)); G waves right of the pivot update their
//     columns j > k: G(i,j) -= L(i,k) L(j,k) (the column test is static
//     within the unrolled block, waves left of the pivot are done and skip);
//   - A waves: row k becomes A_k / L(k,k) and rows i > k lose L(i,k) times it.
// Rows above the pivot keep stale values in the upper triangle of G, which
// the factor never reads.  Writes R (row-major, identity-padded) to rfac and
// R^{-1} to rinv.  Returns 1 (block-wide) if a pivot falls to <= rel * (its
// original value) or is not finite; the owner of the diagonal checks it.
__device__ int chol_inv(const double* G0, double shift, double rel, int b, double* colbuf,
                        double* rowbuf, double* rfac, double* rinv) {
    const int tid = threadIdx.x, i = tid & 63, w = tid >> 6;
    const bool gw = w < 4;
    const int cb0 = 16 * (w & 3);  // first column of this wave's block
    double g[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = cb0 + jj;
        g[jj] = gw ? G0[i * LDT + j] + ((i == j && i < b) ? shift : 0.0) : (i == j ? 1.0 : 0.0);
    }
    const double d0 = G0[i * LDT + i] + (i < b ? shift : 0.0);
    int bad = 0;
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int k = 16 * kb + kk;
            if (k < b) {  // uniform
                double* cb = colbuf + (kk & 1) * 64;
                double* rb = rowbuf + (kk & 1) * 64;
                if (w == kb) cb[i] = g[kk];
                if (!gw && i == k) {
                    double2_t* dst = reinterpret_cast<double2_t*>(rb + cb0);
#pragma unroll
                    for (int h = 0; h < 8; ++h) dst[h] = double2_t{g[2 * h], g[2 * h + 1]};
                }
                __syncthreads();
                const double dkk = cb[k];
                const double ci = cb[i];
                if (gw) {
                    if (w >= kb) {  // uniform
                        double cv[16];
                        const double2_t* src = reinterpret_cast<const double2_t*>(cb + cb0);
#pragma unroll
                        for (int h = 0; h < 8; ++h) {
                            const double2_t v = src[h];
                            cv[2 * h] = v[0];
                            cv[2 * h + 1] = v[1];
                        }
                        const double rinv_k = rsqrt_nr(fmax(dkk, 1e-300));
                        const double li = ci * rinv_k;
                        const double t = li * rinv_k;
                        if (w > kb) {
#pragma unroll
                            for (int jj = 0; jj < 16; ++jj) g[jj] = fma(-t, cv[jj], g[jj]);
                        } else {
#pragma unroll
                            for (int jj = kk + 1; jj < 16; ++jj) g[jj] = fma(-t, cv[jj], g[jj]);
                            g[kk] = li;
                            if (i == k && !(d0 > 0.0 && dkk > rel * d0 && dkk < INFINITY)) bad = 1;
                        }
                    }
                } else {
                    double x[16];
                    const double2_t* src = reinterpret_cast<const double2_t*>(rb + cb0);
#pragma unroll
                    for (int h = 0; h < 8; ++h) {
                        const double2_t v = src[h];
                        x[2 * h] = v[0];
                        x[2 * h + 1] = v[1];
                    }
                    const double rinv_k = rsqrt_nr(fmax(dkk, 1e-300));
                    const double c1 = (i == k) ? rinv_k : 1.0;
                    const double c2 = (i > k) ? ci * rinv_k * rinv_k : 0.0;
#pragma unroll
                    for (int jj = 0; jj < 16; ++jj) g[jj] = fma(-c2, x[jj], g[jj] * c1);
                }
            }
        }
    }
    // R(j, i) = L(i, j) for i >= j; R^{-1}(j, i) = L^{-1}(i, j)
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = cb0 + jj;
        if (gw)
            rfac[j * 64 + i] = (i >= j) ? g[jj] : 0.0;
        else
            rinv[j * 64 + i] = (i >= j) ? g[jj] : 0.0;
    }
    return __syncthreads_or(bad);
}

// One workgroup: sum the P partial Grams (fixed order), factor, invert.
//   pass 0: plain Cholesky with the 1e-10 certificate; if it fails, redo it
//           on G + sI and mark the shifted route;
//   pass 1: plain Cholesky of Q1^T Q1 (fallback flag on breakdown);
//   pass 2: only on the shifted route, Cholesky of Q2^T Q2.
__global__ void __launch_bounds__(512) cq_chol_kernel(CqDev q, int pass) {
    if (q.flags[0]) return;
    if (pass == 2 && !q.flags[1]) return;
    __shared__ double G0[64 * LDT];
    __shared__ __align__(16) double colbuf[128];
    __shared__ __align__(16) double rowbuf[128];
    const int tid = threadIdx.x;
    const int b = q.b;
    // 8 consecutive entries per thread, partials summed in order p = 0..P-1
    {
        const int i = tid >> 3, j0 = (tid & 7) * 8;
        const int ic = min(i, b - 1);
        double acc[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) acc[jj] = 0.0;
#pragma unroll 4
        for (int p = 0; p < q.P; ++p) {
            const double2_t* src =
                reinterpret_cast<const double2_t*>(q.gpart + (size_t)p * 4096 + ic * 64 + j0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double2_t x = src[v];
                acc[2 * v] += x[0];
                acc[2 * v + 1] += x[1];
            }
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int j = j0 + jj;
            G0[i * LDT + j] = (i < b && j < b) ? acc[jj] : ((i == j) ? 1.0 : 0.0);
        }
    }
    __syncthreads();
    double* rfac = q.rfac + (size_t)pass * 4096;
    double* rinv = q.rinv + (size_t)pass * 4096;
    // pass 0 retries once with the shift when the certificate fails
    double shift = 0.0;
    double rel = (pass == 0) ? 1e-10 : ((pass == 1 && !q.flags[1]) ? 0.5 : 0.0);
    int bad;
#pragma unroll 1
    for (int attempt = 0;; ++attempt) {
        bad = chol_inv(G0, shift, rel, b, colbuf, rowbuf, rfac, rinv);
        if (pass != 0 || !bad || attempt == 1) break;
        double tr = 0.0;
        for (int j = 0; j < b; ++j) tr += G0[j * LDT + j];
        shift = 11.0 * ((double)q.m * b + (double)b * (b + 1)) * 1.1102230246251565e-16 * tr;
        rel = 0.0;
    }
    if (pass == 0 && tid == 0) q.flags[1] = (shift > 0.0) ? 1 : 0;
    if (tid == 0 && bad) q.flags[0] = 1;
}

// out = src * Rinv(pass) per row block (MFMA); with GRAM, also the partial
// Grams of out.  pass 1 reads S and writes Q1; pass 2 reads Q1 and writes Q2
// or, when the route is not shifted, the final Q into the panel; pass 3
// (shifted route only) reads Q2 and writes the final Q.
__global__ void __launch_bounds__(256) cq_apply_kernel(CqDev q, int pass) {
    if (q.flags[0]) return;
    const bool shifted = q.flags[1] != 0;
    if (pass == 3 && !shifted) return;
    const bool final_pass = (pass == 3) || (pass == 2 && !shifted);
    const bool gram = !final_pass;
    __shared__ double T[TB * LDT];
    __shared__ double Ri[64 * LDT];
    const double* src = (pass == 1) ? q.a : (pass == 2 ? q.q1 : q.q2);
    const int lds = (pass == 1) ? q.lda : q.m;
    double* dst = final_pass ? q.a : (pass == 1 ? q.q1 : q.q2);
    const int ldd = final_pass ? q.lda : q.m;
    const double* rinv = q.rinv + (size_t)(pass - 1) * 4096;
    for (int t = threadIdx.x; t < 64 * 64; t += 256) Ri[(t >> 6) * LDT + (t & 63)] = rinv[t];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    int r0, r1;
    block_rows(q, blockIdx.x, r0, r1);
    double4_t gacc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) gacc[nb] = double4_t{0, 0, 0, 0};
    for (int r = r0; r < r1; r += TB) {
        __syncthreads();
        load_tile(src, lds, r, r1, q.b, T);
        __syncthreads();
        double4_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = double4_t{0, 0, 0, 0};
#pragma unroll 4
        for (int kk = 0; kk < 64; kk += 4) {
            const double av = T[(w * 16 + li) * LDT + kk + lg];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[nb] = mfma_f64_16x16x4(av, Ri[(kk + lg) * LDT + nb * 16 + li], acc[nb]);
        }
        __syncthreads();
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = w * 16 + mfma_row_f64(lg, v), c = nb * 16 + li;
                const int row = r + i;
                const bool ok = (row < r1 && c < q.b);
                if (ok) dst[(size_t)c * ldd + row] = acc[nb][v];
                T[i * LDT + c] = ok ? acc[nb][v] : 0.0;
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
    for (int t = tid; t < 64 * 64; t += 256) A[(t >> 6) * LDT + (t & 63)] = q.rfac[t];
    for (int p = 1; p < npass; ++p) {
        for (int t = tid; t < 64 * 64; t += 256)
            B[(t >> 6) * LDT + (t & 63)] = q.rfac[(size_t)p * 4096 + t];
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
    for (int t = tid; t < b * b; t += 256) {
        const int col = t / b, i = t - col * b;
        q.r_out[t] = (i <= col) ? A[i * LDT + col] : 0.0;
    }
}

}  // namespace

size_t cq_workspace_doubles(int m, int b) {
    const int P = std::max(1, std::min(16, ceil_div(m, 128)));
    return 2 * (size_t)m * b + (size_t)P * 4096 + 6 * 4096 + 64;
}

void launch_cq(double* a, int m, int b, int lda, double* r_out, double* ws, int* flags,
               hipStream_t s) {
    CqDev q{};
    q.m = m;
    q.b = b;
    q.lda = lda;
    q.P = std::max(1, std::min(16, ceil_div(m, 128)));
    q.a = a;
    q.q1 = ws;
    q.q2 = ws + (size_t)m * b;
    q.gpart = q.q2 + (size_t)m * b;
    q.rinv = q.gpart + (size_t)q.P * 4096;
    q.rfac = q.rinv + 3 * 4096;
    q.r_out = r_out;
    q.flags = flags;
    hipLaunchKernelGGL(cq_gram_kernel, dim3(q.P), dim3(256), 0, s, q);
    TTR_CHECK_LAUNCH();
    for (int pass = 1; pass <= 3; ++pass) {
        hipLaunchKernelGGL(cq_chol_kernel, dim3(1), dim3(512), 0, s, q, pass - 1);
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
