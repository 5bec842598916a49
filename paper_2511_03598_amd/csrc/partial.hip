// Right-to-left KRP partial contraction of one TT core (Sec. 3.1, Eq. 7-8):
//   W_k(a, c) = sum_i Omega_k(i, c) * sum_b X_k(a, i, b) * W_{k+1}(b, c).
// The b-contraction is a GEMM of the vertical unfolding V(X_k) (rows (a,i),
// contiguous in b) with W_{k+1}; it runs on MFMA (f64 16x16x4 or f32
// 16x16x4) and its epilogue folds the Omega-weighted sum over i, so the
// r_{k-1} x r_k x ell intermediate never leaves registers and each core is
// read from HBM exactly once.
//
// Work decomposition: one workgroup (4 wave64) per output row a and 64-wide
// column block; the four waves split the b (K) range, each lane streams 4
// consecutive doubles of a core row per 16-wide K chunk, and the partial
// sums are combined across lane groups by shuffles and across waves in LDS
// (fixed order, deterministic).
#include <climits>

#include "kernels.hpp"

namespace ttr {
namespace {

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    typedef double4_t type;
    static __device__ __forceinline__ type mma(double a, double b, type c) {
        return mfma_f64_16x16x4(a, b, c);
    }
    static __device__ __forceinline__ int row(int g, int v) { return mfma_row_f64(g, v); }
};
template <>
struct Acc<float> {
    typedef float4_t type;
    static __device__ __forceinline__ type mma(float a, float b, type c) {
        return mfma_f32_16x16x4(a, b, c);
    }
    static __device__ __forceinline__ int row(int g, int v) { return mfma_row_f32(g, v); }
};

template <typename T, bool SCALED>
__global__ void __launch_bounds__(256) pc_kernel(PcArgs p) {
    typedef typename Acc<T>::type acc_t;
    const int a = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int colbase = p.c0 + blockIdx.y * 64;
    const int ncb = min(64, p.c0 + p.nc - colbase);
    const int K = p.r1, n = p.n;
    const T* Wn = static_cast<const T*>(p.Wn);

    T in_scale = T(1);
    int in_e = 0;
    if (SCALED && p.in_maxexp != nullptr) {
        int e = *p.in_maxexp;
        in_e = (e == INT_MIN) ? 0 : e;
        in_scale = (T)ldexp(1.0, -in_e);
    }

    const int nkc = (K + 15) / 16;
    const int per = (nkc + 3) / 4;
    const int kc_beg = w * per, kc_end = min(nkc, kc_beg + per);
    const double* Xa = p.X + (size_t)a * n * K;

    T part[4] = {T(0), T(0), T(0), T(0)};
    for (int rc = 0; rc < n; rc += 64) {
        acc_t acc[4][4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = acc_t{0, 0, 0, 0};

        for (int kc = kc_beg; kc < kc_end; ++kc) {
            const int kb = kc * 16 + 4 * lg;
            T av[4][4], bv[4][4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int i = rc + mb * 16 + li;
                const double* row = Xa + (size_t)i * K;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = kb + s;
                    av[mb][s] = (i < n && k < K) ? (T)row[k] : T(0);
                }
            }
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int col = nb * 16 + li;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = kb + s;
                    T v = T(0);
                    if (k < K && col < ncb) {
                        if (Wn == nullptr)
                            v = T(1);  // W_{d+1} = 1 (K == 1)
                        else
                            v = Wn[(size_t)k * p.ldw + colbase + col];
                        if (SCALED) v *= in_scale;
                    }
                    bv[nb][s] = v;
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[mb][nb] = Acc<T>::mma(av[mb][s], bv[nb][s], acc[mb][nb]);
        }
        // Omega-weighted fold over the rows i held by this lane.
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = rc + mb * 16 + Acc<T>::row(lg, v);
                if (i < n) {
                    const double* orow = p.Om + (size_t)i * p.ldo + colbase;
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        const int col = nb * 16 + li;
                        const T om = (col < ncb) ? (T)orow[col] : T(0);
                        part[nb] += acc[mb][nb][v] * om;
                    }
                }
            }
        }
    }
    // Sum over the four lane groups, then over the four waves.
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        part[nb] += __shfl_xor(part[nb], 16, 64);
        part[nb] += __shfl_xor(part[nb], 32, 64);
    }
    __shared__ T red[4][64];
    if (lg == 0) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) red[w][nb * 16 + li] = part[nb];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        const T v = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
        T* Wo = static_cast<T*>(p.Wout);
        if (c < ncb) Wo[(size_t)a * p.ldw + colbase + c] = v;
        if (SCALED) {
            int e = INT_MIN;
            if (c < ncb && v != T(0)) {
                int ex;
                frexp((double)v, &ex);
                e = ex;
            }
            e = wave_max_int(e);
            if (c == 0 && e != INT_MIN) atomicMax(p.out_maxexp, e);
            if (a == 0 && c < ncb) {
                const int base = (p.in_colexp != nullptr) ? p.in_colexp[colbase + c] : 0;
                p.out_colexp[colbase + c] = base + in_e;
            }
        }
    }
}

__global__ void fill_int_kernel(int* p, int value, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = value;
}

__global__ void w_to_f64_kernel(const float* w, const int* colexp, int64_t ldw, int rows, int c0,
                                int nc, double* out, int64_t ldo) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * nc) return;
    const int r = (int)(t / nc), c = (int)(t - (int64_t)r * nc);
    out[(size_t)r * ldo + c] = ldexp((double)w[(size_t)r * ldw + c0 + c], colexp[c0 + c]);
}

}  // namespace

void launch_pc_f64(const PcArgs& a, hipStream_t s) {
    dim3 grid(a.r0, ceil_div(a.nc, 64));
    hipLaunchKernelGGL((pc_kernel<double, false>), grid, dim3(256), 0, s, a);
    TTR_CHECK_LAUNCH();
}

void launch_pc_f32(const PcArgs& a, hipStream_t s) {
    dim3 grid(a.r0, ceil_div(a.nc, 64));
    hipLaunchKernelGGL((pc_kernel<float, true>), grid, dim3(256), 0, s, a);
    TTR_CHECK_LAUNCH();
}

void launch_fill_int(int* p, int value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(fill_int_kernel, dim3(ceil_div(count, 256)), dim3(256), 0, s, p, value,
                       count);
    TTR_CHECK_LAUNCH();
}

void launch_w_to_f64(const float* w, const int* colexp, int64_t ldw, int rows, int c0, int nc,
                     double* out, int64_t ldo, hipStream_t s) {
    const int64_t work = (int64_t)rows * nc;
    if (work <= 0) return;
    hipLaunchKernelGGL(w_to_f64_kernel, dim3(ceil_div(work, 256)), dim3(256), 0, s, w, colexp,
                       ldw, rows, c0, nc, out, ldo);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
