// SVD of a small float64 matrix by one-sided (Hestenes) Jacobi, for the
// right-to-left truncation pass of Remark 2 (the "tau or l_k truncated SVD"
// of the TT-Rounding algorithm, Sec. 2.2, applied to R^T from the LQ of
// H(Y_k)).  Columns of A are rotated pairwise until mutually orthogonal:
// A V = U Sigma.  Pairs follow a round-robin tournament, q/2 disjoint pairs
// per round, each pair owned by a 16-lane group; one barrier per round.
// One-sided Jacobi gives singular values to high relative accuracy, which
// the tolerance-based truncation needs.
#include <algorithm>

#include "kernels.hpp"

namespace ttr {
namespace {

__device__ __forceinline__ int rr_player(int pos, int r, int qq) {
    return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (qq - 1));
}

__global__ void __launch_bounds__(256) svd_jacobi_kernel(const double* A, int lda, int p, int q,
                                                         double* G, double* Vs, double* sig,
                                                         double tau, int target, int* t_out) {
    extern __shared__ double lds[];
    __shared__ double sg[64];
    __shared__ int perm[64];
    __shared__ int rotated;
    double* As = lds;          // p x q, ld p
    double* V = lds + p * q;   // q x q, ld q
    const int tid = threadIdx.x, g = tid >> 4, l16 = tid & 15;
    for (int t = tid; t < p * q; t += 256) {
        const int c = t / p, i = t - c * p;
        As[t] = A[(size_t)c * lda + i];
    }
    for (int t = tid; t < q * q; t += 256) V[t] = ((t / q) == (t % q)) ? 1.0 : 0.0;
    const int qq = q + (q & 1);
    const double tol = fmax(1e-15, 2.3e-16 * (double)p);
    __syncthreads();
    for (int sweep = 0; sweep < 60 && qq >= 2; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < qq - 1; ++r) {
            for (int ps = g; ps < qq / 2; ps += 16) {
                int i1 = rr_player(ps, r, qq), i2 = rr_player(qq - 1 - ps, r, qq);
                if (i1 > i2) {
                    const int tmp = i1;
                    i1 = i2;
                    i2 = tmp;
                }
                if (i2 >= q) continue;  // bye
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = l16; i < p; i += 16) {
                    const double x = As[i1 * p + i], y = As[i2 * p + i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = group16_sum(al);
                be = group16_sum(be);
                ga = group16_sum(ga);
                if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                    if (l16 == 0) rotated = 1;
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                    for (int i = l16; i < p; i += 16) {
                        const double x = As[i1 * p + i], y = As[i2 * p + i];
                        As[i1 * p + i] = c * x - s * y;
                        As[i2 * p + i] = s * x + c * y;
                    }
                    for (int i = l16; i < q; i += 16) {
                        const double x = V[i1 * q + i], y = V[i2 * q + i];
                        V[i1 * q + i] = c * x - s * y;
                        V[i2 * q + i] = s * x + c * y;
                    }
                }
            }
            __syncthreads();
        }
        const int done = !rotated;
        __syncthreads();
        if (done) break;
    }
    // Column norms, sort by decreasing norm (stable by index).
    for (int c = g; c < q; c += 16) {
        double s = 0.0;
        for (int i = l16; i < p; i += 16) s += As[c * p + i] * As[c * p + i];
        s = group16_sum(s);
        if (l16 == 0) sg[c] = sqrt(s);
    }
    __syncthreads();
    if (tid < q) {
        int rank = 0;
        const double me = sg[tid];
        for (int i = 0; i < q; ++i) rank += (sg[i] > me) || (sg[i] == me && i < tid);
        perm[rank] = tid;
    }
    __syncthreads();
    for (int t = tid; t < p * q; t += 256) {
        const int r = t / p, i = t - r * p;
        G[(size_t)r * p + i] = As[perm[r] * p + i];
    }
    for (int t = tid; t < q * q; t += 256) {
        const int r = t / q, i = t - r * q;
        Vs[(size_t)r * q + i] = V[perm[r] * q + i];
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
        *t_out = t;
    }
}

}  // namespace

void launch_svd_jacobi(const double* A, int lda, int p, int q, double* G, double* Vs, double* sig,
                       double tau, int target, int* t_out, hipStream_t s) {
    if (q < 1 || q > 64 || p < q)
        throw Error(-6, "small SVD: need 1 <= q <= 64 and p >= q");
    const size_t bytes = (size_t)(p * q + q * q) * sizeof(double);
    if ((int)bytes > device_lds_limit() - 4096)
        throw Error(-6, "small SVD: matrix too large for LDS");
    static bool attr = false;
    if (!attr) {
        TTR_HIP(hipFuncSetAttribute((const void*)svd_jacobi_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    device_lds_limit() - 4096));
        attr = true;
    }
    hipLaunchKernelGGL(svd_jacobi_kernel, dim3(1), dim3(256), bytes, s, A, lda, p, q, G, Vs, sig,
                       tau, target, t_out);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
