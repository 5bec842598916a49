// SVD of a small float64 matrix by one-sided (Hestenes) Jacobi, for the
// right-to-left truncation pass of Remark 2 (the "tau or l_k truncated SVD"
// of the TT-Rounding algorithm, Sec. 2.2, applied to R^T from the LQ of
// H(Y_k)).  Columns of A are rotated pairwise until mutually orthogonal:
// A V = U Sigma.  Pairs follow a recursive bipartite order: in each phase
// every 16-lane group keeps one column of A and V in registers (4 rows per
// lane) and meets a sequence of moving columns, one per round (DPP
// reductions, one barrier per round), so a round moves only half of the
// columns through LDS.
// One-sided Jacobi gives singular values to high relative accuracy, which
// the tolerance-based truncation needs.
#include <algorithm>

#include "kernels.hpp"

namespace ttr {
namespace {

// Sums over the 16 lanes of a DPP row for three values at once (the three
// butterflies interleaved so their latencies overlap).
__device__ __forceinline__ void group16_sum3(double& a, double& b, double& c) {
    a += dpp_f64<0xB1>(a);
    b += dpp_f64<0xB1>(b);
    c += dpp_f64<0xB1>(c);
    a += dpp_f64<0x4E>(a);
    b += dpp_f64<0x4E>(b);
    c += dpp_f64<0x4E>(c);
    a += dpp_f64<0x141>(a);
    b += dpp_f64<0x141>(b);
    c += dpp_f64<0x141>(c);
    a += dpp_f64<0x140>(a);
    b += dpp_f64<0x140>(b);
    c += dpp_f64<0x140>(c);
}

// Rotation (c, s) that diagonalises [[al, ga], [ga, be]] (ga != 0), the
// classical Jacobi angle tan = sign(z)/(|z| + sqrt(1 + z^2)), z = (be-al)/(2 ga),
// rewritten without divisions: with dd = be - al, g2 = 2 ga (both scaled by
// the same power of two so the larger lies in [1/2, 1)), w = |dd| +
// sqrt(dd^2 + g2^2) and h = 1/sqrt(w^2 + g2^2): c = w h, s = sign(dd) g2 h.
// c^2 + s^2 = 1 to the accuracy of h whatever the accuracy of w, so the
// rotation stays orthogonal; the scaling makes it immune to over/underflow.
__device__ __forceinline__ void jacobi_cs(double al, double be, double ga, double& c, double& s) {
    double dd = be - al, g2 = 2.0 * ga;
    int e;
    (void)frexp(fmax(fabs(dd), fabs(g2)), &e);
    dd = ldexp(dd, -e);
    g2 = ldexp(g2, -e);
    const double x = fma(dd, dd, g2 * g2);  // [1/4, 2)
    const double w = fabs(dd) + x * rsqrt_nr(x);
    const double h = rsqrt_nr(fma(w, w, g2 * g2));  // argument in [1/4, 8)
    c = w * h;
    s = copysign(1.0, dd) * g2 * h;
}

__global__ void __launch_bounds__(512) svd_jacobi_kernel(const double* A, int lda, int trans, int p, int q,
                                                         double* G, double* Vs, double* sig,
                                                         double tau, int target, int* t_out) {
    // Columns of A and V live in LDS with a fixed stride of 64 rows, zero
    // padded, so every lane handles exactly 4 rows without masks.
    constexpr int LD = 64;
    __shared__ double As[64 * LD];
    __shared__ double V[64 * LD];
    __shared__ double sg[64];
    __shared__ int perm[64];
    __shared__ int rotated;
    __shared__ int nsweeps;
    __shared__ double wmax[8];
    const int tid = threadIdx.x;
    double amax = 0.0;
    for (int t = tid; t < 64 * LD; t += 512) {
        const int c = t / LD, i = t - c * LD;
        const double a = (c < q && i < p) ? A[trans ? (size_t)i * lda + c : (size_t)c * lda + i] : 0.0;
        As[t] = a;
        amax = fmax(amax, fabs(a));
        V[t] = (c == i && c < q) ? 1.0 : 0.0;
    }
    // Scale A by a power of two (exact) so its largest entry lies in [1/2, 1):
    // squared column norms and their products then neither overflow nor
    // lose the small columns to underflow.  Undone on G and sigma at the end.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = amax;
    __syncthreads();
    amax = wmax[0];
#pragma unroll
    for (int w = 1; w < 8; ++w) amax = fmax(amax, wmax[w]);
    int sexp = 0;
    if (amax > 0.0 && amax < INFINITY) (void)frexp(amax, &sexp);
    for (int t = tid; t < 64 * LD; t += 512) As[t] = ldexp(As[t], -sexp);
    // Rotate while (x.y)^2 > tol^2 (x.x)(y.y); tol sits well above the
    // rounding error of a p-term dot product (~p u) so the sweep test can be met.
    const double tol2 = 1e-26;
    if (tid == 0) nsweeps = 0;
    // One column pair per 16-lane group; lane l16 holds rows l16, l16+16, ...
    const int g8 = tid >> 4, l8 = tid & 15;
    __syncthreads();
    for (int sweep = 0; sweep < 60 && q >= 2; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        // Recursive bipartite order on 64 column slots (columns >= q are
        // absent): phase p splits the slots into 2^p blocks of 64 >> p; group
        // g keeps column f = lo + j of its block's first half in registers
        // for the whole phase and meets the second half's columns one per
        // round, so only the moving column passes through LDS each round.
        // Every pair meets once per sweep (63 rounds of up to 32 pairs).
        for (int p = 0; p < 6; ++p) {
            const int h1 = 32 >> p, j = g8 & (h1 - 1), lo = (g8 >> (5 - p)) * 2 * h1;
            const int f = lo + j;
            double x[4], vx[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                x[t] = As[min(f, 63) * LD + l8 + 16 * t];
                vx[t] = V[min(f, 63) * LD + l8 + 16 * t];
            }
            bool fdirty = false;
            for (int r = 0; r < h1; ++r) {
                const int m = lo + h1 + ((j + r) & (h1 - 1));
                if (f < q && m < q) {  // uniform per group
                    double y[4];
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) y[t] = As[m * LD + l8 + 16 * t];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        al += x[t] * x[t];
                        be += y[t] * y[t];
                        ga += x[t] * y[t];
                    }
                    group16_sum3(al, be, ga);
                    if (ga * ga > tol2 * (al * be)) {
                        if (l8 == 0) rotated = 1;
                        fdirty = true;
                        double vy[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) vy[t] = V[m * LD + l8 + 16 * t];
                        double c, sn;
                        jacobi_cs(al, be, ga, c, sn);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int i = l8 + 16 * k;
                            const double xk = x[k], yk = y[k], uk = vx[k], wk = vy[k];
                            x[k] = c * xk - sn * yk;
                            vx[k] = c * uk - sn * wk;
                            As[m * LD + i] = sn * xk + c * yk;
                            V[m * LD + i] = sn * uk + c * wk;
                        }
                    }
                }
                __syncthreads();
            }
            if (fdirty) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    As[f * LD + l8 + 16 * t] = x[t];
                    V[f * LD + l8 + 16 * t] = vx[t];
                }
            }
            __syncthreads();
        }
        const int done = !rotated;
        if (tid == 0) nsweeps = sweep + 1;
        __syncthreads();
        if (done) break;
    }
    // Column norms, sort by decreasing norm (stable by index).
    for (int c = g8; c < q; c += 32) {
        double s = 0.0;
        for (int i = l8; i < 64; i += 16) s += As[c * 64 + i] * As[c * 64 + i];
        s = group16_sum(s);
        if (l8 == 0) sg[c] = ldexp(sqrt(s), sexp);
    }
    __syncthreads();
    if (tid < q) {
        int rank = 0;
        const double me = sg[tid];
        for (int i = 0; i < q; ++i) rank += (sg[i] > me) || (sg[i] == me && i < tid);
        perm[rank] = tid;
    }
    __syncthreads();
    for (int t = tid; t < p * q; t += 512) {
        const int r = t / p, i = t - r * p;
        G[(size_t)r * p + i] = ldexp(As[perm[r] * 64 + i], sexp);
    }
    for (int t = tid; t < q * q; t += 512) {
        const int r = t / q, i = t - r * q;
        Vs[(size_t)r * q + i] = V[perm[r] * 64 + i];
    }
    if (tid < q) sig[tid] = sg[perm[tid]];
    if (tid == 0) {
        int t = q;
        if (tau >= 0.0) {
            double acc = 0.0;
            for (int r = q - 1; r >= 1; --r) {
                const double s = sg[perm[r]];
                acc += s * s;
                if (sqrt(acc) <= tau)
                    t = r;
                else
                    break;
            }
        } else {
            t = min(max(target, 1), q);
        }
        t_out[0] = t;
        t_out[1] = nsweeps;
    }
}

}  // namespace

void launch_svd_jacobi(const double* A, int lda, int p, int q, double* G, double* Vs, double* sig,
                       double tau, int target, int* t_out, hipStream_t s, bool trans) {
    if (q < 1 || q > 64 || p < q || p > 64)
        throw Error(-6, "small SVD: need 1 <= q <= p <= 64");
    hipLaunchKernelGGL(svd_jacobi_kernel, dim3(1), dim3(512), 0, s, A, lda, trans ? 1 : 0, p, q, G, Vs, sig,
                       tau, target, t_out);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
