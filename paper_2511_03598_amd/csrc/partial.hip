// Right-to-left KRP partial contraction of one TT core (Sec. 3.1, Eq. 7-8):
//   W_k(a, c) = sum_i Omega_k(i, c) * sum_b X_k(a, i, b) * W_{k+1}(b, c).
// The b-contraction is a GEMM of the vertical unfolding V(X_k) (rows (a,i),
// contiguous in b) with W_{k+1}; it runs on MFMA (f64 16x16x4 or f32
// 16x16x4) and its epilogue folds the Omega-weighted sum over i, so the
// r_{k-1} x r_k x ell intermediate never leaves registers and each core is
// read from HBM exactly once.
//
// Work decomposition: one workgroup (4 wave64) per output row a and 64-wide
// column block; each wave owns 16 of the n rows (i) over the whole b (K)
// range.  Each lane streams 4 consecutive doubles of its core row per 16-wide
// K chunk, prefetched one 128-deep slab ahead; the matching block of W_{k+1}
// is staged once per slab in LDS and feeds the MFMA B operand.  Partial sums
// are combined across lane groups by shuffles and across waves in LDS (fixed
// order, deterministic).
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

constexpr int SLAB = 128;   // K rows of W staged per pass
constexpr int WPAD = 80;    // LDS row stride of the staged W block (bank spread)
constexpr int NCH = SLAB / 16;

// This lane's A operands for one K slab: 8 chunks of 16 K, 4 consecutive k
// per lane (k = k0 + 16c + 4*lg + s).  Loads are unconditional from a
// clamped address and masked afterwards, so the compiler issues them all
// back to back; with even K they are 16-byte aligned pairs.
template <bool KEVEN>
__device__ __forceinline__ void load_slab(const double* __restrict__ xr, bool row_ok, int K, int k0,
                                          int lg, double (&buf)[4 * NCH]) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int kb = k0 + 16 * c + 4 * lg;
        if (KEVEN) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = kb + 2 * h;
                const double2_t v =
                    *reinterpret_cast<const double2_t*>(xr + min(k, K - 2));
                const bool ok = row_ok && k < K;
                buf[4 * c + 2 * h] = ok ? v[0] : 0.0;
                buf[4 * c + 2 * h + 1] = ok ? v[1] : 0.0;
            }
        } else {
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const int k = kb + s2;
                const double v = xr[min(k, K - 1)];
                buf[4 * c + s2] = (row_ok && k < K) ? v : 0.0;
            }
        }
    }
}

template <typename T, bool SCALED, bool KEVEN>
__global__ void __launch_bounds__(256) pc_kernel(PcArgs p) {
    typedef typename Acc<T>::type acc_t;
    __shared__ T Ws[SLAB * WPAD];
    __shared__ T red[4][64];
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int colbase = p.c0 + blockIdx.y * 64;
    const int ncb = min(64, p.c0 + p.nc - colbase);
    const int K = p.r1, n = p.n;
    const T* Wn = static_cast<const T*>(p.Wn);

    T in_scale = T(1);
    int in_e = 0;
    if (SCALED && p.in_maxexp != nullptr) {
        const int e = *p.in_maxexp;
        in_e = (e == INT_MIN) ? 0 : e;
        in_scale = (T)ldexp(1.0, -in_e);
    }
    const double* Xa = p.X + (size_t)a * n * K;

    auto stage = [&](int k0) {
        __syncthreads();
        for (int t = tid; t < SLAB * 64; t += 256) {
            const int kk = t >> 6, c = t & 63, k = k0 + kk;
            T v = T(0);
            if (k < K && c < ncb) {
                v = (Wn == nullptr) ? T(k == 0 ? 1 : 0) : Wn[(size_t)k * p.ldw + colbase + c];
                if (SCALED) v *= in_scale;
            }
            Ws[kk * WPAD + c] = v;
        }
        __syncthreads();
    };
    auto compute = [&](const double (&buf)[4 * NCH], int k0, acc_t (&acc)[4]) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (k0 + 16 * c < K) {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    const T av = (T)buf[4 * c + s2];
                    const T* wr = Ws + (16 * c + 4 * lg + s2) * WPAD + li;
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) acc[nb] = Acc<T>::mma(av, wr[16 * nb], acc[nb]);
                }
            }
        }
    };

    T part[4] = {T(0), T(0), T(0), T(0)};
    for (int rc = 0; rc < n; rc += 64) {
        const int row = rc + 16 * w + li;
        const bool row_ok = row < n;
        const double* xr = Xa + (size_t)min(row, n - 1) * K;
        acc_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = acc_t{0, 0, 0, 0};
        double A0[4 * NCH], A1[4 * NCH];
        load_slab<KEVEN>(xr, row_ok, K, 0, lg, A0);
        for (int k0 = 0; k0 < K; k0 += 2 * SLAB) {
            if (k0 + SLAB < K) load_slab<KEVEN>(xr, row_ok, K, k0 + SLAB, lg, A1);
            stage(k0);
            compute(A0, k0, acc);
            if (k0 + SLAB >= K) break;
            if (k0 + 2 * SLAB < K) load_slab<KEVEN>(xr, row_ok, K, k0 + 2 * SLAB, lg, A0);
            stage(k0 + SLAB);
            compute(A1, k0 + SLAB, acc);
        }
        // Omega-weighted fold over this wave's rows.
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = rc + 16 * w + Acc<T>::row(lg, v);
            if (i < n) {
                const double* orow = p.Om + (size_t)i * p.ldo + colbase;
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const int col = nb * 16 + li;
                    const T om = (col < ncb) ? (T)orow[col] : T(0);
                    part[nb] += acc[nb][v] * om;
                }
            }
        }
    }
    // Sum over the four lane groups, then over the four waves (fixed order).
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        part[nb] += __shfl_xor(part[nb], 16, 64);
        part[nb] += __shfl_xor(part[nb], 32, 64);
    }
    if (lg == 0) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) red[w][nb * 16 + li] = part[nb];
    }
    __syncthreads();
    if (tid < 64) {
        const int c = tid;
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
    if (a.r1 % 2 == 0)
        hipLaunchKernelGGL((pc_kernel<double, false, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((pc_kernel<double, false, false>), grid, dim3(256), 0, s, a);
    TTR_CHECK_LAUNCH();
}

void launch_pc_f32(const PcArgs& a, hipStream_t s) {
    dim3 grid(a.r0, ceil_div(a.nc, 64));
    if (a.r1 % 2 == 0)
        hipLaunchKernelGGL((pc_kernel<float, true, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((pc_kernel<float, true, false>), grid, dim3(256), 0, s, a);
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
