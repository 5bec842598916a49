// Thin QR of a tall-skinny float64 panel (the "reduced QR decomposition"
// of the sketches in Sec. 3.2-3.3 and of H(Y_k)^T in Remark 2), as TSQR
// with Householder reflectors:
//   factor: each workgroup factors a block of <= hmax rows in LDS; blocks
//           are combined pairwise up a binary tree, each combine done by the
//           last of the two children to finish (integer arrival counters,
//           self-resetting), so the whole R is produced in one launch;
//   formQ:  each leaf walks its root-to-leaf path applying the node
//           reflectors to [C; 0] (C starts as diag(sign(R_jj))), then its
//           own reflectors, writing its rows of the explicit Q.
// diag(R) >= 0 after the sign fix, so Q is the unique thin-QR factor of a
// full-rank panel; rank-deficient panels still get orthonormal columns.
#include <algorithm>
#include <mutex>

#include "kernels.hpp"

namespace ttr {
namespace {

// In-LDS Householder QR of an h x b column-major matrix L (ld), 256 threads.
// On return L holds R on/above the diagonal and the reflector tails below
// (unit diagonal implied); tau[j] is written to LDS array `tau`.
__device__ void hh_factor(double* L, int h, int b, int ld, double* tau, double* red) {
    const int tid = threadIdx.x, g = tid >> 4, l16 = tid & 15;
    for (int j = 0; j < b; ++j) {
        double s = 0.0;
        for (int i = j + 1 + tid; i < h; i += 256) {
            const double v = L[j * ld + i];
            s += v * v;
        }
        s = block_sum256(s, red);
        const double alpha = L[j * ld + j];
        double tj = 0.0, beta = alpha;
        if (s > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + s), alpha);
            tj = (beta - alpha) / beta;
            const double scal = 1.0 / (alpha - beta);
            for (int i = j + 1 + tid; i < h; i += 256) L[j * ld + i] *= scal;
        }
        __syncthreads();
        if (tid == 0) {
            L[j * ld + j] = beta;
            tau[j] = tj;
        }
        if (tj != 0.0) {
            for (int c = j + 1 + g; c < b; c += 16) {
                double p = (l16 == 0) ? L[c * ld + j] : 0.0;
                for (int i = j + 1 + l16; i < h; i += 16) p += L[j * ld + i] * L[c * ld + i];
                p = group16_sum(p);
                const double f = tj * p;
                if (l16 == 0) L[c * ld + j] -= f;
                for (int i = j + 1 + l16; i < h; i += 16) L[c * ld + i] -= f * L[j * ld + i];
            }
        }
        __syncthreads();
    }
}

// B (h x b, ldb) <- H_0 H_1 ... H_{b-1} B for reflectors stored in V (ldv,
// tails below the diagonal) with taus tau[].  Columns of B are owned by
// 16-lane groups for the whole sweep, so no barrier is needed inside.
__device__ void hh_apply(const double* V, int ldv, const double* tau, double* B, int ldb, int h,
                         int b) {
    const int tid = threadIdx.x, g = tid >> 4, l16 = tid & 15;
    for (int j = b - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        for (int c = g; c < b; c += 16) {
            double p = (l16 == 0) ? B[c * ldb + j] : 0.0;
            for (int i = j + 1 + l16; i < h; i += 16) p += V[j * ldv + i] * B[c * ldb + i];
            p = group16_sum(p);
            const double f = tj * p;
            if (l16 == 0) B[c * ldb + j] -= f;
            for (int i = j + 1 + l16; i < h; i += 16) B[c * ldb + i] -= f * V[j * ldv + i];
        }
    }
}

struct QrDev {
    int m, b, lda, hmax, P, levels;
    double* a;
    double* r_out;
    double* tau;    // nodes x b
    double* rbuf;   // nodes x b x b (column-major)
    double* vnode;  // (nodes - P) x (2b x b)
    int* cnt;       // nodes
    const int* only_if;  // if set, run only when *only_if != 0
};

__device__ __forceinline__ int level_count(int P, int level) {
    int n = P;
    for (int l = 0; l < level; ++l) n = (n + 1) / 2;
    return n;
}
__device__ __forceinline__ int level_offset(int P, int level) {
    int off = 0, n = P;
    for (int l = 0; l < level; ++l) {
        off += n;
        n = (n + 1) / 2;
    }
    return off;
}

__device__ void write_r(const QrDev& q, const double* L, int ld, int node) {
    const int b = q.b;
    double* R = q.rbuf + (size_t)node * b * b;
    for (int t = threadIdx.x; t < b * b; t += blockDim.x) {
        const int c = t / b, j = t - c * b;
        R[t] = (j <= c) ? L[c * ld + j] : 0.0;
    }
}

__global__ void __launch_bounds__(256) qr_factor_kernel(QrDev q) {
    if (q.only_if != nullptr && *q.only_if == 0) return;
    extern __shared__ double lds[];
    __shared__ double red[4];
    __shared__ double tau_s[64];
    __shared__ int s_last;
    const int b = q.b, leaf = blockIdx.x;
    const int r0 = (int)(((int64_t)leaf * q.m) / q.P);
    const int r1 = (int)(((int64_t)(leaf + 1) * q.m) / q.P);
    const int h = r1 - r0;
    double* L = lds;  // h x b, ld h
    for (int t = threadIdx.x; t < h * b; t += 256) {
        const int c = t / h, i = t - c * h;
        L[t] = q.a[(size_t)c * q.lda + r0 + i];
    }
    __syncthreads();
    hh_factor(L, h, b, h, tau_s, red);
    __syncthreads();
    for (int t = threadIdx.x; t < h * b; t += 256) {
        const int c = t / h, i = t - c * h;
        q.a[(size_t)c * q.lda + r0 + i] = L[t];
    }
    for (int j = threadIdx.x; j < b; j += 256) q.tau[(size_t)leaf * b + j] = tau_s[j];
    write_r(q, L, h, leaf);

    int idx = leaf;
    int node = leaf;
    for (int level = 0; level < q.levels; ++level) {
        const int nlev = level_count(q.P, level);
        const int pidx = idx >> 1;
        const int nchild = (2 * pidx + 1 < nlev) ? 2 : 1;
        const int parent = level_offset(q.P, level + 1) + pidx;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const int old = atomicAdd(&q.cnt[parent], 1);
            s_last = (old == nchild - 1);
        }
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        if (threadIdx.x == 0) q.cnt[parent] = 0;
        const int child0 = level_offset(q.P, level) + 2 * pidx;
        if (nchild == 2) {
            const int ld = 2 * b;
            for (int t = threadIdx.x; t < ld * b; t += 256) {
                const int c = t / ld, i = t - c * ld;
                const int ch = (i < b) ? child0 : child0 + 1;
                const int j = (i < b) ? i : i - b;
                L[t] = __builtin_nontemporal_load(&q.rbuf[(size_t)ch * b * b + (size_t)c * b + j]);
            }
            __syncthreads();
            hh_factor(L, ld, b, ld, tau_s, red);
            __syncthreads();
            double* V = q.vnode + (size_t)(parent - q.P) * ld * b;
            for (int t = threadIdx.x; t < ld * b; t += 256) V[t] = L[t];
            for (int j = threadIdx.x; j < b; j += 256) q.tau[(size_t)parent * b + j] = tau_s[j];
            write_r(q, L, ld, parent);
        } else {
            for (int t = threadIdx.x; t < b * b; t += 256)
                q.rbuf[(size_t)parent * b * b + t] =
                    __builtin_nontemporal_load(&q.rbuf[(size_t)child0 * b * b + t]);
            for (int j = threadIdx.x; j < b; j += 256) q.tau[(size_t)parent * b + j] = 0.0;
        }
        node = parent;
        idx = pidx;
    }
    // Only the root's workgroup reaches here.
    if (q.r_out != nullptr) {
        __threadfence();
        __syncthreads();
        const double* R = q.rbuf + (size_t)node * b * b;
        for (int t = threadIdx.x; t < b * b; t += 256) {
            const int c = t / b, j = t - c * b;
            const double d = __builtin_nontemporal_load(&R[(size_t)j * b + j]);
            const double sg = (d < 0.0) ? -1.0 : 1.0;
            q.r_out[t] = sg * __builtin_nontemporal_load(&R[t]);
        }
    }
}

__global__ void __launch_bounds__(256) qr_formq_kernel(QrDev q, int nodes) {
    if (q.only_if != nullptr && *q.only_if == 0) return;
    extern __shared__ double lds[];
    __shared__ double tau_s[64];
    const int b = q.b, leaf = blockIdx.x, hm = q.hmax;
    double* Vs = lds;             // hmax x b
    double* Bs = lds + hm * b;    // hmax x b, ld hmax
    const double* Rroot = q.rbuf + (size_t)(nodes - 1) * b * b;
    for (int t = threadIdx.x; t < b * b; t += 256) {
        const int c = t / b, j = t - c * b;
        const double sg = (Rroot[(size_t)c * b + c] < 0.0) ? -1.0 : 1.0;
        Bs[c * hm + j] = (j == c) ? sg : 0.0;
    }
    __syncthreads();
    for (int level = q.levels; level >= 1; --level) {
        const int pidx = leaf >> level;
        const int nprev = level_count(q.P, level - 1);
        if (2 * pidx + 1 >= nprev) continue;  // single child: identity
        const int node = level_offset(q.P, level) + pidx;
        const int ld = 2 * b;
        const double* V = q.vnode + (size_t)(node - q.P) * ld * b;
        for (int t = threadIdx.x; t < ld * b; t += 256) Vs[t] = V[t];
        for (int j = threadIdx.x; j < b; j += 256) tau_s[j] = q.tau[(size_t)node * b + j];
        for (int t = threadIdx.x; t < b * b; t += 256) {
            const int c = t / b, i = t - c * b;
            Bs[c * hm + b + i] = 0.0;
        }
        __syncthreads();
        hh_apply(Vs, ld, tau_s, Bs, hm, ld, b);
        __syncthreads();
        const int right = (leaf >> (level - 1)) & 1;
        if (right) {
            for (int t = threadIdx.x; t < b * b; t += 256) {
                const int c = t / b, i = t - c * b;
                Bs[c * hm + i] = Bs[c * hm + b + i];
            }
        }
        __syncthreads();
    }
    const int r0 = (int)(((int64_t)leaf * q.m) / q.P);
    const int r1 = (int)(((int64_t)(leaf + 1) * q.m) / q.P);
    const int h = r1 - r0;
    for (int t = threadIdx.x; t < h * b; t += 256) {
        const int c = t / h, i = t - c * h;
        Vs[c * h + i] = q.a[(size_t)c * q.lda + r0 + i];
        if (i >= b) Bs[c * hm + i] = 0.0;
    }
    for (int j = threadIdx.x; j < b; j += 256) tau_s[j] = q.tau[(size_t)leaf * b + j];
    __syncthreads();
    hh_apply(Vs, h, tau_s, Bs, hm, h, b);
    __syncthreads();
    for (int t = threadIdx.x; t < h * b; t += 256) {
        const int c = t / h, i = t - c * h;
        q.a[(size_t)c * q.lda + r0 + i] = Bs[c * hm + i];
    }
}

}  // namespace

int device_lds_limit() {
    static int cached = -1;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (cached < 0) {
        int dev = 0, v = 0;
        TTR_HIP(hipGetDevice(&dev));
        TTR_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        cached = v;
    }
    return cached;
}

QrPlan plan_qr(int m, int b, int lda) {
    if (b < 1 || b > 64 || m < b)
        throw Error(-6, "tt_qr: need 1 <= b <= 64 and m >= b (m=" + std::to_string(m) +
                            ", b=" + std::to_string(b) + ")");
    QrPlan p{};
    p.m = m;
    p.b = b;
    p.lda = lda;
    const int budget = device_lds_limit() / 8 - 1024;  // doubles, minus static LDS
    p.hmax = budget / (2 * b);
    if (p.hmax < 2 * b)
        throw Error(-6, "tt_qr: LDS too small for panel width " + std::to_string(b));
    p.hmax = std::min(p.hmax, 4096);
    p.P = std::max(1, ceil_div(m, p.hmax));
    int n = p.P;
    p.nodes = n;
    p.levels = 0;
    while (n > 1) {
        n = (n + 1) / 2;
        p.nodes += n;
        ++p.levels;
    }
    p.lds_bytes = (size_t)2 * p.hmax * b * sizeof(double);
    return p;
}

size_t qr_workspace_doubles(const QrPlan& p) {
    const size_t b = p.b;
    return (size_t)p.nodes * b + (size_t)p.nodes * b * b + (size_t)(p.nodes - p.P) * 2 * b * b;
}

void launch_qr(const QrPlan& p, double* a, double* r_out, double* ws, int* counters,
               hipStream_t s, const int* only_if) {
    static std::once_flag once;
    std::call_once(once, [] {
        const int lim = device_lds_limit() - 2048;
        TTR_HIP(hipFuncSetAttribute((const void*)qr_factor_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        TTR_HIP(hipFuncSetAttribute((const void*)qr_formq_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    });
    QrDev q{};
    q.m = p.m;
    q.b = p.b;
    q.lda = p.lda;
    q.hmax = p.hmax;
    q.P = p.P;
    q.levels = p.levels;
    q.a = a;
    q.r_out = r_out;
    const size_t b = p.b;
    q.tau = ws;
    q.rbuf = ws + (size_t)p.nodes * b;
    q.vnode = q.rbuf + (size_t)p.nodes * b * b;
    q.cnt = counters;
    q.only_if = only_if;
    const size_t lds_factor = (size_t)p.hmax * b * sizeof(double);
    hipLaunchKernelGGL(qr_factor_kernel, dim3(p.P), dim3(256), lds_factor, s, q);
    TTR_CHECK_LAUNCH();
    hipLaunchKernelGGL(qr_formq_kernel, dim3(p.P), dim3(256), p.lds_bytes, s, q, p.nodes);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
