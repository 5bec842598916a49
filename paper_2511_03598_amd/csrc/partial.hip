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
template <bool KEVEN, int NC = NCH>
__device__ __forceinline__ void load_slab(const double* __restrict__ xr, bool row_ok, int K, int k0,
                                          int lg, double (&buf)[4 * NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
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

    // W_{k+1}(k0 .. k0+SLAB, block columns) -> LDS.  All loads of a thread
    // are issued unconditionally from clamped addresses and masked after
    // (a guarded load would wait on each one in turn).
    auto stage = [&](int k0) {
        constexpr int PER = SLAB * 64 / 256;
        const int c = tid & 63, kk0 = tid >> 6;
        const int cc = colbase + min(c, ncb - 1);
        T v[PER];
        if (Wn != nullptr) {
#pragma unroll
            for (int e = 0; e < PER; ++e) v[e] = Wn[(size_t)min(k0 + kk0 + 4 * e, K - 1) * p.ldw + cc];
        } else {
#pragma unroll
            for (int e = 0; e < PER; ++e) v[e] = T(k0 + kk0 + 4 * e == 0 ? 1 : 0);
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int kk = kk0 + 4 * e;
            T x = (k0 + kk < K && c < ncb) ? v[e] : T(0);
            if (SCALED) x *= in_scale;
            Ws[kk * WPAD + c] = x;
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
        {
            double om[4][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = min(rc + 16 * w + Acc<T>::row(lg, v), n - 1);
                const double* orow = p.Om + (size_t)i * p.ldo + colbase;
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) om[v][nb] = orow[min(nb * 16 + li, ncb - 1)];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const bool iok = rc + 16 * w + Acc<T>::row(lg, v) < n;
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const T o = (iok && nb * 16 + li < ncb) ? (T)om[v][nb] : T(0);
                    part[nb] += acc[nb][v] * o;
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


// ---------------------------------------------------------------------------
// Wide variant: one workgroup of KG x 4 waves (KG = 2) per output row a and 64-wide
// column block.  The whole W_{k+1} block (K x 64, zero-padded to whole
// 16-row chunks) is staged in LDS once; the K range is cut into KG slices,
// one per group of 4 waves (each wave 16 of the 64 rows i of a row chunk),
// and the KG x 4 partial column sums are added in LDS in a fixed order.
// Every X load of a slab and every staging load are issued before the first
// wait, so a workgroup has its whole row of the core (n x K doubles for
// n <= 64) in flight at once.  Used when the staged block fits in LDS.
// ---------------------------------------------------------------------------
constexpr int WPW = 68;  // LDS row stride of the staged W (2-way bank split)

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    typedef float4_t type;
};
template <>
struct Vec4<double> {
    typedef double4_t type;
};

// KG wave groups of 4 waves; WSCH 16-wide K chunks per slab and wave; VEC4:
// W_{k+1} rows and the column block start are 16-byte aligned (and W is not
// the implicit W_{d+1} = 1), so the staging uses 16-byte loads.
template <typename T, bool SCALED, bool KEVEN, int KG, int WSCH, bool VEC4>
__global__ void __launch_bounds__(KG * 256) pc_wide_kernel(PcArgs p) {
    typedef typename Acc<T>::type acc_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = p.r1, n = p.n;
    const int chunks = (K + 15) / 16;
    const int K16 = 16 * chunks;
    T* Ws = reinterpret_cast<T*>(smem_raw);  // K16 x WPW
    T* red = Ws + (size_t)K16 * WPW;         // [KG*4][64]
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wg = wv >> 2, wr = wv & 3;
    const int li = lane & 15, lg = lane >> 4;
    const int colbase = p.c0 + blockIdx.y * 64;
    const int ncb = min(64, p.c0 + p.nc - colbase);
    const T* Wn = static_cast<const T*>(p.Wn);
    const int kbeg = 16 * ((wg * chunks) / KG);
    const int kend = min(K, 16 * (((wg + 1) * chunks) / KG));
    const bool has_k = kend > kbeg;  // uniform per wave group
    const double* Xa = p.X + (size_t)a * n * K;

    T in_scale = T(1);
    int in_e = 0;
    if (SCALED && p.in_maxexp != nullptr) {
        const int e = *p.in_maxexp;
        in_e = (e == INT_MIN) ? 0 : e;
        in_scale = (T)ldexp(1.0, -in_e);
    }

    // Raw (unmasked) X values of one slab: this lane's row, 4 consecutive k
    // per 16-wide chunk from clamped addresses; the mask is applied where the
    // values are consumed, so no load has to be waited for before then.
    double buf[4 * WSCH];
    auto load = [&](int rc, int k0) {
        const double* xr = Xa + (size_t)min(rc + 16 * wr + li, n - 1) * K;
#pragma unroll
        for (int c = 0; c < WSCH; ++c) {
            const int kb = k0 + 16 * c + 4 * lg;
            if (KEVEN) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double2_t v =
                        *reinterpret_cast<const double2_t*>(xr + min(kb + 2 * h, kend - 2));
                    buf[4 * c + 2 * h] = v[0];
                    buf[4 * c + 2 * h + 1] = v[1];
                }
            } else {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) buf[4 * c + s2] = xr[min(kb + s2, kend - 1)];
            }
        }
    };
    // Stage W_{k+1} rows 0..K16 (zero beyond K and beyond ncb).  The first
    // round's loads are issued before the X loads, so waiting for them
    // (vector memory counters retire in order) does not wait for X.
    const int total = K16 * 64, nthr = KG * 256;
    if (VEC4) {
        // 16-byte loads: thread -> (row, 4 columns); rows 16-byte aligned
        constexpr int SR = (sizeof(T) == 4) ? 8 : 4;
        const int cq = (tid & 15) * 4, rr = tid >> 4;   // 16 column quads per row
        const int rows_per_pass = nthr / 16;
        const int cqc = min(cq, ((ncb + 3) & ~3) - 4);
        typedef typename Vec4<T>::type v4;
        auto ld = [&](int r) -> v4 {
            return *reinterpret_cast<const v4*>(Wn + (size_t)min(r, K - 1) * p.ldw + colbase + cqc);
        };
        auto st = [&](int r, v4 v) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                T x = (r < K && cq + j < ncb) ? v[j] : T(0);
                if (SCALED) x *= in_scale;
                v[j] = x;
            }
            if (r < K16) *reinterpret_cast<v4*>(Ws + r * WPW + cq) = v;
        };
        v4 sv[SR];
#pragma unroll
        for (int e = 0; e < SR; ++e) sv[e] = ld(rr + e * rows_per_pass);
        if (has_k) load(0, kbeg);
#pragma unroll
        for (int e = 0; e < SR; ++e) st(rr + e * rows_per_pass, sv[e]);
        for (int r0 = SR * rows_per_pass; r0 < K16; r0 += SR * rows_per_pass) {
#pragma unroll
            for (int e = 0; e < SR; ++e) sv[e] = ld(r0 + rr + e * rows_per_pass);
#pragma unroll
            for (int e = 0; e < SR; ++e) st(r0 + rr + e * rows_per_pass, sv[e]);
        }
    } else {
        constexpr int SR = (sizeof(T) == 4) ? 32 : 16;
        auto stage_load = [&](int round, T (&v)[SR]) {
            if (Wn) {
#pragma unroll
                for (int e = 0; e < SR; ++e) {
                    const int idx = min(round * nthr * SR + e * nthr + tid, total - 1);
                    const int k = min(idx >> 6, K - 1), c = min(idx & 63, ncb - 1);
                    v[e] = Wn[(size_t)k * p.ldw + colbase + c];
                }
            } else {
#pragma unroll
                for (int e = 0; e < SR; ++e) {
                    const int idx = round * nthr * SR + e * nthr + tid;
                    v[e] = T((idx >> 6) == 0 ? 1 : 0);
                }
            }
        };
        auto stage_store = [&](int round, const T (&v)[SR]) {
#pragma unroll
            for (int e = 0; e < SR; ++e) {
                const int idx = round * nthr * SR + e * nthr + tid;
                const int k = idx >> 6, c = idx & 63;
                T x = (k < K && c < ncb) ? v[e] : T(0);
                if (SCALED) x *= in_scale;
                if (idx < total) Ws[k * WPW + c] = x;
            }
        };
        const int rounds = (total + nthr * SR - 1) / (nthr * SR);
        T sv[SR];
        stage_load(0, sv);
        if (has_k) load(0, kbeg);
        stage_store(0, sv);
        for (int r = 1; r < rounds; ++r) {
            stage_load(r, sv);
            stage_store(r, sv);
        }
    }
    __syncthreads();

    T part[4] = {T(0), T(0), T(0), T(0)};
    for (int rc = 0; rc < n; rc += 64) {
        // Omega rows of this wave, issued before the MFMAs that precede their use
        T om[4][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = min(rc + 16 * wr + Acc<T>::row(lg, v), n - 1);
            const double* orow = p.Om + (size_t)i * p.ldo + colbase;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) om[v][nb] = (T)orow[min(nb * 16 + li, ncb - 1)];
        }
        acc_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = acc_t{0, 0, 0, 0};
        if (has_k) {
            for (int k0 = kbeg; k0 < kend; k0 += 16 * WSCH) {
#pragma unroll
                for (int c = 0; c < WSCH; ++c) {
                    const int kc = k0 + 16 * c;
                    if (kc < kend) {
                        const bool rok = rc + 16 * wr + li < n;
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) {
                            const bool ok = rok && kc + 4 * lg + s2 < kend;
                            const T av = ok ? (T)buf[4 * c + s2] : T(0);
                            const T* wrow = Ws + (kc + 4 * lg + s2) * WPW + li;
#pragma unroll
                            for (int nb = 0; nb < 4; ++nb)
                                acc[nb] = Acc<T>::mma(av, wrow[16 * nb], acc[nb]);
                        }
                    }
                }
                const int nk0 = k0 + 16 * WSCH;
                if (nk0 < kend)
                    load(rc, nk0);
                else if (rc + 64 < n)
                    load(rc + 64, kbeg);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool iok = rc + 16 * wr + Acc<T>::row(lg, v) < n;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const T o = (iok && nb * 16 + li < ncb) ? om[v][nb] : T(0);
                part[nb] += acc[nb][v] * o;
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        part[nb] += __shfl_xor(part[nb], 16, 64);
        part[nb] += __shfl_xor(part[nb], 32, 64);
    }
    if (lg == 0) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) red[wv * 64 + nb * 16 + li] = part[nb];
    }
    __syncthreads();
    if (tid < 64) {
        const int c = tid;
        T v = T(0);
#pragma unroll
        for (int w = 0; w < KG * 4; ++w) v += red[w * 64 + c];
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

template <typename T, int KG>
size_t wide_lds_bytes(int K) {
    return ((size_t)16 * ((K + 15) / 16) * WPW + (size_t)KG * 4 * 64) * sizeof(T);
}

constexpr size_t kWideLdsMax = 150 * 1024;

template <typename T, bool SCALED, bool KEVEN, int KG, int WSCH, bool VEC4>
void launch_wide(const PcArgs& a, size_t lds, hipStream_t s) {
    auto kern = pc_wide_kernel<T, SCALED, KEVEN, KG, WSCH, VEC4>;
    static const hipError_t attr = hipFuncSetAttribute(
        (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWideLdsMax);
    (void)attr;
    dim3 grid(a.r0, ceil_div(a.nc, 64));
    hipLaunchKernelGGL(kern, grid, dim3(KG * 256), lds, s, a);
    TTR_CHECK_LAUNCH();
}

template <typename T, bool SCALED, int KG, int WSCH>
bool try_launch_wide(const PcArgs& a, hipStream_t s) {
    const size_t lds = wide_lds_bytes<T, KG>(a.r1);
    if (lds > kWideLdsMax) return false;
    // 16-byte staging needs 4-element aligned rows and block start
    const bool vec4 = a.Wn != nullptr && (a.ldw % 4) == 0 && (a.c0 % 4) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.Wn) % (4 * sizeof(T))) == 0;
    if (a.r1 % 2 == 0) {
        if (vec4)
            launch_wide<T, SCALED, true, KG, WSCH, true>(a, lds, s);
        else
            launch_wide<T, SCALED, true, KG, WSCH, false>(a, lds, s);
    } else {
        launch_wide<T, SCALED, false, KG, WSCH / 2, false>(a, lds, s);
    }
    return true;
}


// ---------------------------------------------------------------------------
// BF16 variant: X is rounded to bfloat16 in registers, W_{k+1} is stored in
// bfloat16 (with the same per-column power-of-two exponents as the FP32
// path) and the b-contraction runs on v_mfma_f32_16x16x16_bf16 with FP32
// accumulation; the Omega fold and the reductions stay in FP32 and W_k is
// rounded to bfloat16 once at the end.  A lane's four consecutive k of a
// 16-wide chunk are exactly its A operand, so one MFMA covers a chunk; W
// is staged transposed (column-major in LDS) so the matching B operand is
// one 8-byte LDS read.  Same workgroup shape as the wide FP32 kernel.
// ---------------------------------------------------------------------------
typedef short bf16x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float((unsigned)h << 16);
}

template <bool KEVEN, int KG, int WSCH>
__global__ void __launch_bounds__(KG * 256) pc_bf16_kernel(PcArgs p) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = p.r1, n = p.n;
    const int chunks = (K + 15) / 16;
    const int K16 = 16 * chunks;
    const int LDK = K16 + 8;  // transposed row stride (bf16 elements)
    unsigned short* Wt = reinterpret_cast<unsigned short*>(smem_raw);  // 64 x LDK
    float* red = reinterpret_cast<float*>(Wt + (size_t)64 * LDK);       // [KG*4][64]
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wg = wv >> 2, wr = wv & 3;
    const int li = lane & 15, lg = lane >> 4;
    const int colbase = p.c0 + blockIdx.y * 64;
    const int ncb = min(64, p.c0 + p.nc - colbase);
    const unsigned short* Wn = static_cast<const unsigned short*>(p.Wn);
    const int kbeg = 16 * ((wg * chunks) / KG);
    const int kend = min(K, 16 * (((wg + 1) * chunks) / KG));
    const bool has_k = kend > kbeg;
    const double* Xa = p.X + (size_t)a * n * K;

    float in_scale = 1.f;
    int in_e = 0;
    if (p.in_maxexp != nullptr) {
        const int e = *p.in_maxexp;
        in_e = (e == INT_MIN) ? 0 : e;
        in_scale = (float)ldexp(1.0, -in_e);
    }

    double buf[4 * WSCH];
    auto load = [&](int rc, int k0) {
        const double* xr = Xa + (size_t)min(rc + 16 * wr + li, n - 1) * K;
#pragma unroll
        for (int c = 0; c < WSCH; ++c) {
            const int kb = k0 + 16 * c + 4 * lg;
            if (KEVEN) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double2_t v =
                        *reinterpret_cast<const double2_t*>(xr + min(kb + 2 * h, kend - 2));
                    buf[4 * c + 2 * h] = v[0];
                    buf[4 * c + 2 * h + 1] = v[1];
                }
            } else {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) buf[4 * c + s2] = xr[min(kb + s2, kend - 1)];
            }
        }
    };
    // Stage W_{k+1}: thread -> (row k, column c); element loads are 2 bytes,
    // issued in rounds of SR before the X loads of the first slab.
    {
        constexpr int SR = 16;
        const int nthr = KG * 256, total = K16 * 64;
        const int c = tid & 63, cc = colbase + min(c, ncb - 1);
        const bool cok = c < ncb;
        for (int base = 0; base < total; base += nthr * SR) {
            unsigned short v[SR];
#pragma unroll
            for (int e = 0; e < SR; ++e) {
                const int k = min((base + e * nthr + tid) >> 6, K - 1);
                v[e] = Wn ? Wn[(size_t)k * p.ldw + cc] : (unsigned short)(k == 0 ? 0x3F80 : 0);
            }
            if (base == 0 && has_k) load(0, kbeg);
#pragma unroll
            for (int e = 0; e < SR; ++e) {
                const int idx = base + e * nthr + tid;
                const int k = idx >> 6;
                const float x = (k < K && cok) ? bf16_to_f32(v[e]) * in_scale : 0.f;
                if (idx < total) Wt[c * LDK + k] = bf16_rne(x);
            }
        }
        if (total == 0 && has_k) load(0, kbeg);
    }
    __syncthreads();

    float part[4] = {0.f, 0.f, 0.f, 0.f};
    for (int rc = 0; rc < n; rc += 64) {
        float om[4][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = min(rc + 16 * wr + mfma_row_f32(lg, v), n - 1);
            const double* orow = p.Om + (size_t)i * p.ldo + colbase;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) om[v][nb] = (float)orow[min(nb * 16 + li, ncb - 1)];
        }
        float4_t acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = float4_t{0.f, 0.f, 0.f, 0.f};
        if (has_k) {
            const bool rok = rc + 16 * wr + li < n;
            for (int k0 = kbeg; k0 < kend; k0 += 16 * WSCH) {
#pragma unroll
                for (int c = 0; c < WSCH; ++c) {
                    const int kc = k0 + 16 * c;
                    if (kc < kend) {
                        bf16x4_t av;
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) {
                            const bool ok = rok && kc + 4 * lg + s2 < kend;
                            av[s2] = (short)bf16_rne(ok ? (float)buf[4 * c + s2] : 0.f);
                        }
#pragma unroll
                        for (int nb = 0; nb < 4; ++nb) {
                            const bf16x4_t bv = *reinterpret_cast<const bf16x4_t*>(
                                Wt + (nb * 16 + li) * LDK + kc + 4 * lg);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nb], 0, 0, 0);
                        }
                    }
                }
                const int nk0 = k0 + 16 * WSCH;
                if (nk0 < kend)
                    load(rc, nk0);
                else if (rc + 64 < n)
                    load(rc + 64, kbeg);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool iok = rc + 16 * wr + mfma_row_f32(lg, v) < n;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const float o = (iok && nb * 16 + li < ncb) ? om[v][nb] : 0.f;
                part[nb] += acc[nb][v] * o;
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        part[nb] += __shfl_xor(part[nb], 16, 64);
        part[nb] += __shfl_xor(part[nb], 32, 64);
    }
    if (lg == 0) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) red[wv * 64 + nb * 16 + li] = part[nb];
    }
    __syncthreads();
    if (tid < 64) {
        const int c = tid;
        float v = 0.f;
#pragma unroll
        for (int w = 0; w < KG * 4; ++w) v += red[w * 64 + c];
        const unsigned short hv = bf16_rne(v);
        unsigned short* Wo = static_cast<unsigned short*>(p.Wout);
        if (c < ncb) Wo[(size_t)a * p.ldw + colbase + c] = hv;
        const float vr = bf16_to_f32(hv);
        int e = INT_MIN;
        if (c < ncb && vr != 0.f) {
            int ex;
            frexp((double)vr, &ex);
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

__global__ void w_bf16_to_f64_kernel(const unsigned short* w, const int* colexp, int64_t ldw,
                                     int rows, int c0, int nc, double* out, int64_t ldo) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * nc) return;
    const int r = (int)(t / nc), c = (int)(t - (int64_t)r * nc);
    out[(size_t)r * ldo + c] =
        ldexp((double)bf16_to_f32(w[(size_t)r * ldw + c0 + c]), colexp[c0 + c]);
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
    if (try_launch_wide<double, false, 2, 8>(a, s)) return;
    dim3 grid(a.r0, ceil_div(a.nc, 64));
    if (a.r1 % 2 == 0)
        hipLaunchKernelGGL((pc_kernel<double, false, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((pc_kernel<double, false, false>), grid, dim3(256), 0, s, a);
    TTR_CHECK_LAUNCH();
}

void launch_pc_f32(const PcArgs& a, hipStream_t s) {
    if (try_launch_wide<float, true, 2, 8>(a, s)) return;
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

void launch_pc_bf16(const PcArgs& a, hipStream_t s) {
    constexpr int KG = 2;
    const size_t lds = (size_t)64 * (16 * ceil_div(a.r1, 16) + 8) * 2 + (size_t)KG * 4 * 64 * 4;
    if (lds > kWideLdsMax) throw Error(-6, "BF16 partial contraction: rank too large for LDS staging");
    dim3 grid(a.r0, ceil_div(a.nc, 64));
    if (a.r1 % 2 == 0) {
        auto kern = pc_bf16_kernel<true, KG, 8>;
        static const hipError_t attr = hipFuncSetAttribute(
            (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWideLdsMax);
        (void)attr;
        hipLaunchKernelGGL(kern, grid, dim3(KG * 256), lds, s, a);
    } else {
        auto kern = pc_bf16_kernel<false, KG, 4>;
        static const hipError_t attr = hipFuncSetAttribute(
            (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWideLdsMax);
        (void)attr;
        hipLaunchKernelGGL(kern, grid, dim3(KG * 256), lds, s, a);
    }
    TTR_CHECK_LAUNCH();
}

void launch_w_bf16_to_f64(const unsigned short* w, const int* colexp, int64_t ldw, int rows, int c0,
                          int nc, double* out, int64_t ldo, hipStream_t s) {
    const int64_t work = (int64_t)rows * nc;
    if (work <= 0) return;
    hipLaunchKernelGGL(w_bf16_to_f64_kernel, dim3(ceil_div(work, 256)), dim3(256), 0, s, w, colexp,
                       ldw, rows, c0, nc, out, ldo);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
