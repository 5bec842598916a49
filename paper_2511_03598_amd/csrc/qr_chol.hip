// Fast path of the thin QR: CholeskyQR2, or shifted CholeskyQR3 for
// ill-conditioned panels, all decided on the device.
//
//   gram    : per-block partial Grams G = S^T S (MFMA), written to a buffer;
//   chol    : one wave sums the partials in a fixed order, factors
//             G = R^T R (Cholesky), forms R^{-1} and sets the route flags;
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
    double* rinv;   // 3 x 64 x 64 (one per pass)
    double* rfac;   // 3 x 64 x 64
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

__device__ __forceinline__ void load_tile(const double* src, int ld, int r, int r_end, int b,
                                          double* T) {
    for (int t = threadIdx.x; t < TB * 64; t += blockDim.x) {
        const int c = t / TB, i = t - c * TB;
        const int row = r + i;
        T[i * LDT + c] = (c < b && row < r_end) ? src[(size_t)c * ld + row] : 0.0;
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

// Cholesky G = R^T R of the LDS matrix G (64 x LDT, identity-padded beyond
// b, `shift` added to the first b diagonal entries), 256 threads: four lanes
// share row i = tid/4, each keeping 16 columns in registers (the unrolled
// step loop keeps register indices static).  At step k the owners of column
// k publish it through LDS (double-buffered, one barrier per step); every
// lane forms L(i,k) = G(i,k)/sqrt(G(k,k)) and updates its columns j > k:
// G(i,j) -= L(i,k) L(j,k).  R (row-major, zero below the diagonal) is
// written to R.  Returns 1 (block-wide) if a pivot falls to <= rel * (its
// original value) or is not finite.
__device__ int chol_quad(const double* G, double shift, double rel, int b, double* R,
                         double* colbuf) {
    const int tid = threadIdx.x, i = tid >> 2, qd = tid & 3;
    double g[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * qd + jj;
        g[jj] = G[i * LDT + j] + ((i == j && i < b) ? shift : 0.0);
    }
    int bad = 0;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        double* cb = colbuf + (k & 1) * 64;
        if (qd == (k >> 4)) cb[i] = g[k & 15];
        __syncthreads();
        const double dkk = cb[k];
        if (k < b) {
            const double d0 = G[k * LDT + k] + shift;
            if (!(d0 > 0.0 && dkk > rel * d0 && dkk < INFINITY)) bad = 1;
        }
        const double rinv = 1.0 / sqrt(fmax(dkk, 1e-300));
        const double li = cb[i] * rinv;
        const double* cj = cb + 16 * qd;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            if (16 * qd + jj > k) g[jj] -= li * (cj[jj] * rinv);
        if (qd == (k >> 4)) g[k & 15] = li;
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int k = 16 * qd + jj;
        R[k * LDT + i] = (k <= i) ? g[jj] : 0.0;
    }
    return __syncthreads_or(bad);
}

// X <- X R^{-1} for the 64 rows of an LDS tile X (row stride LDT), R upper
// triangular (identity-padded): four lanes share a row (16 columns each);
// column l is solved by its owner lane, broadcast inside the quad (DPP
// quad_perm) and eliminated from the later columns.  No barriers inside.
template <int L>
__device__ __forceinline__ double quad_bcast(double v) {
    return dpp_f64<(L) | ((L) << 2) | ((L) << 4) | ((L) << 6)>(v);
}

__device__ void rsolve_rows(const double* R, double* X) {
    const int tid = threadIdx.x, r = tid >> 2, qd = tid & 3;
    double s[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) s[jj] = X[r * LDT + 16 * qd + jj];
#pragma unroll
    for (int l = 0; l < 64; ++l) {
        double x = s[l & 15] * (1.0 / R[l * LDT + l]);
        switch (l >> 4) {
            case 0: x = quad_bcast<0>(x); break;
            case 1: x = quad_bcast<1>(x); break;
            case 2: x = quad_bcast<2>(x); break;
            default: x = quad_bcast<3>(x); break;
        }
        const double* rl = R + l * LDT + 16 * qd;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) s[jj] -= x * rl[jj];
        if (qd == (l >> 4)) s[l & 15] = x;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) X[r * LDT + 16 * qd + jj] = s[jj];
    __syncthreads();
}

// One workgroup: sum the P partial Grams (fixed order), Cholesky, R^{-1}.
//   pass 0: plain Cholesky with the 1e-10 certificate; if it fails, redo it
//           on G + sI and mark the shifted route;
//   pass 1: plain Cholesky of Q1^T Q1 (fallback flag on breakdown);
//   pass 2: only on the shifted route, Cholesky of Q2^T Q2.
__global__ void __launch_bounds__(256) cq_chol_kernel(CqDev q, int pass) {
    if (q.flags[0]) return;
    if (pass == 2 && !q.flags[1]) return;
    __shared__ double G0[64 * LDT];
    __shared__ double G[64 * LDT];
    const int tid = threadIdx.x;
    const int b = q.b;
    // 16 consecutive entries per thread, partials summed in order p = 0..P-1
    {
        const int i = tid >> 2, j0 = (tid & 3) * 16;
        double acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
        if (i < b) {
            for (int p = 0; p < q.P; ++p) {
                const double2_t* src =
                    reinterpret_cast<const double2_t*>(q.gpart + (size_t)p * 4096 + i * 64 + j0);
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const double2_t x = src[v];
                    acc[2 * v] += x[0];
                    acc[2 * v + 1] += x[1];
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = j0 + jj;
            G0[i * LDT + j] = (i < b && j < b) ? acc[jj] : ((i == j) ? 1.0 : 0.0);
        }
    }
    __syncthreads();
    __shared__ double colbuf[128];
    int bad;
    if (pass == 0) {
        bad = chol_quad(G0, 0.0, 1e-10, b, G, colbuf);
        if (bad) {
            double tr = 0.0;
            for (int j = 0; j < b; ++j) tr += G0[j * LDT + j];
            const double shift =
                11.0 * ((double)q.m * b + (double)b * (b + 1)) * 1.1102230246251565e-16 * tr;
            bad = chol_quad(G0, shift, 0.0, b, G, colbuf);
            if (tid == 0) q.flags[1] = 1;
        } else if (tid == 0) {
            q.flags[1] = 0;
        }
    } else {
        bad = chol_quad(G0, 0.0, (pass == 1 && !q.flags[1]) ? 0.5 : 0.0, b, G, colbuf);
    }
    // R^{-1} = I R^{-1}: identity rows through the row solver (G0 is free)
    for (int t = tid; t < 64 * 64; t += 256)
        G0[(t >> 6) * LDT + (t & 63)] = ((t >> 6) == (t & 63)) ? 1.0 : 0.0;
    __syncthreads();
    rsolve_rows(G, G0);
    double* rinv = q.rinv + (size_t)pass * 4096;
    double* rfac = q.rfac + (size_t)pass * 4096;
    for (int t = tid; t < 64 * 64; t += 256) {
        const int r = t >> 6, c = t & 63;
        const bool in = (r < b && c < b);
        rinv[t] = in ? G0[r * LDT + c] : 0.0;
        rfac[t] = in ? G[r * LDT + c] : 0.0;
    }
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

// R of the panel: R = R_last ... R_1 (upper triangular), column-major,
// multiplied in LDS by one workgroup.
__global__ void __launch_bounds__(256) cq_rout_kernel(CqDev q) {
    if (q.flags[0]) return;
    const int npass = q.flags[1] ? 3 : 2;
    const int b = q.b, tid = threadIdx.x;
    __shared__ double A[64 * LDT];
    __shared__ double B[64 * LDT];
    for (int t = tid; t < 64 * 64; t += 256) A[(t >> 6) * LDT + (t & 63)] = q.rfac[t];
    for (int p = 1; p < npass; ++p) {
        for (int t = tid; t < 64 * 64; t += 256)
            B[(t >> 6) * LDT + (t & 63)] = q.rfac[(size_t)p * 4096 + t];
        __syncthreads();
        double c[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = tid + 256 * e, i = t >> 6, j = t & 63;
            double s = 0.0;
            for (int l = i; l <= j; ++l) s += B[i * LDT + l] * A[l * LDT + j];
            c[e] = s;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = tid + 256 * e;
            A[(t >> 6) * LDT + (t & 63)] = c[e];
        }
        __syncthreads();
    }
    __syncthreads();
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
    launch_fill_int(flags, 0, 2, s);
    hipLaunchKernelGGL(cq_gram_kernel, dim3(q.P), dim3(256), 0, s, q);
    TTR_CHECK_LAUNCH();
    for (int pass = 1; pass <= 3; ++pass) {
        hipLaunchKernelGGL(cq_chol_kernel, dim3(1), dim3(256), 0, s, q, pass - 1);
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
