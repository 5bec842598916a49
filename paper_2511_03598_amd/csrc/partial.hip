// Right-to-left KRP partial contraction of one TT core (Sec. 3.1, Eq. 7-8):
//   W_k(a, c) = sum_i Omega_k(i, c) * sum_b X_k(a, i, b) * W_{k+1}(b, c).
// The b-contraction is a GEMM of the vertical unfolding V(X_k) (rows (a,i),
// contiguous in b) with W_{k+1}; it runs on MFMA and its epilogue folds the
// Omega-weighted sum over i, so the r_{k-1} x r_k x ell intermediate never
// leaves registers and each core is read from HBM exactly once.
//
// Storage: W_k is kept transposed (one row of r_{k-1} values per sketch
// column, row stride ld a multiple of 4) and, when its contraction is split
// over K, as S partial matrices that every consumer adds in slice order.
//
// Work decomposition: one workgroup per output row a, 64-wide column block
// and K slice (S = pc_slices(r_{k-1}, r_k, precision) slices of whole
// 16-wide chunks).  In the FP64/FP32 kernel every wave owns 16 RT rows i of
// each 64-row group and a share of the slice's chunks, and loads both MFMA
// operands itself: its core rows (4 consecutive b per lane and chunk) and
// the matching W_{k+1} entries (4 consecutive b of one column, one 16-byte
// load in the transposed layout).  No wave waits for another until the
// final reduction, so loads of one wave overlap the MFMAs of the others.
// Partial sums are combined across lane groups by shuffles and across waves
// in LDS in a fixed order; nothing depends on scheduling.
//
// Precisions: FP64 (f64 MFMA 16x16x4), FP32 (f32 MFMA 16x16x4, W stored in
// float32 with a power-of-two exponent per column), BF16 (cores rounded to
// bfloat16 in registers, W stored in bfloat16 with the same exponents,
// v_mfma_f32_16x16x16_bf16 with FP32 accumulation).
#include <algorithm>
#include <climits>

#include "kernels.hpp"

namespace ttr {
namespace {

constexpr size_t kSliceLds = 96 * 1024;  // LDS budget for one staged BF16 slice
constexpr size_t kLdsMax = 150 * 1024;   // dynamic LDS limit requested per kernel

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

typedef short bf16x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float((unsigned)h << 16);
}

// This workgroup's K slice: whole 16-wide chunks [c_lo, c_hi) of the K
// range, i.e. rows kb0 .. kb1 of W_{k+1}; rows16 = 16 (c_hi - c_lo) >= 16.
struct Slice {
    int kb0, kb1, rows16;
};
__device__ __forceinline__ Slice slice_of(int K, int h, int S) {
    const int chunks = (K + 15) / 16;
    const int c_lo = (h * chunks) / S, c_hi = ((h + 1) * chunks) / S;
    return Slice{16 * c_lo, min(K, 16 * c_hi), 16 * (c_hi - c_lo)};
}

// Raw (unmasked) X values of one slab: this lane's row, 4 consecutive k per
// 16-wide chunk, from addresses clamped into [.., kend); the mask is applied
// where the values are consumed, so no load is waited for before then.
template <bool KEVEN, int NC>
__device__ __forceinline__ void load_x(const double* __restrict__ xr, int kend, int k0, int lg,
                                       double (&buf)[4 * NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
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
}

// Input scale of reduced precision: 2^-e with e the largest exponent the
// producer of W_{k+1} recorded (one entry per producer workgroup).  The
// first 256 entries are loaded up front (ExpLoads) so that waiting for them
// does not wait for the operand loads issued after them.
struct ExpLoads {
    int v[4];
    int count;
};
__device__ __forceinline__ ExpLoads issue_input_exponent(const PcArgs& p) {
    ExpLoads x;
    x.count = (p.in_maxexp == nullptr) ? 0 : p.r1 * (int)gridDim.y * p.in_slices;
    // unconditional loads (from this launch's own slots when there is no
    // input; those values are not used) keep the four loads together
    const int* src = (p.in_maxexp != nullptr) ? p.in_maxexp : p.out_maxexp;
    const int last = max(x.count, 1) - 1;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 4; ++j) x.v[j] = src[min(lane + 64 * j, last)];
    return x;
}
__device__ __forceinline__ int input_exponent(const PcArgs& p, const ExpLoads& x) {
    if (x.count == 0) return 0;
    int e = max(max(x.v[0], x.v[1]), max(x.v[2], x.v[3]));
    for (int j = (threadIdx.x & 63) + 256; j < x.count; j += 64) e = max(e, p.in_maxexp[j]);
    e = wave_max_int(e);
    return e == INT_MIN ? 0 : e;
}
__device__ __forceinline__ int input_exponent(const PcArgs& p) {
    return input_exponent(p, issue_input_exponent(p));
}

// Exponent bookkeeping of a reduced-precision output row: this workgroup's
// largest exponent goes to its own entry of out_maxexp; row 0 of slice 0
// writes colexp_k.  Called by the first wave.
__device__ __forceinline__ void track_exponents(const PcArgs& p, int a, int colbase, int c, int ncb,
                                                double v, int in_e) {
    int e = INT_MIN;
    if (c < ncb && v != 0.0) {
        int ex;
        frexp(v, &ex);
        e = ex;
    }
    e = wave_max_int(e);
    if (c == 0) p.out_maxexp[((size_t)a * gridDim.y + blockIdx.y) * gridDim.z + blockIdx.z] = e;
    if (a == 0 && blockIdx.z == 0 && c < ncb) {
        const int base = (p.in_colexp != nullptr) ? p.in_colexp[colbase + c] : 0;
        p.out_colexp[colbase + c] = base + in_e;
    }
}

// ---------------------------------------------------------------------------
// FP64 / FP32 kernel.  NW waves: RG = 4 / RT row groups of 16 RT rows times
// KGN = NW / RG groups of the slice's chunks.  FP32 uses RT = 4: every wave
// covers all 64 rows of a row block for its own chunks, so each W value is
// loaded once per workgroup and feeds four MFMAs, and each core value feeds
// four; FP64 (accumulators twice as wide) uses RT = 1.  WSCH chunks per
// slab of operand loads; ONE: n <= 64 and every wave's chunks fit one slab,
// so all operands are requested before the first MFMA and nothing later.
// MS: W_{k+1} has more than one slice.  NBC: 16-column tiles of the output
// block (launches of at most 48 columns use fewer than four, so no MFMA
// works on padding columns).
//
// Omega's 64 x 64 tile for the row block is loaded once per workgroup
// (coalesced, first), converted to T and kept in LDS for the fold.
// Out-of-range operands are clamped into the arrays and made harmless: W
// entries beyond K are zeroed at use (the matching core values are finite),
// rows beyond n and columns beyond ncb meet zero Omega entries.  The
// reduced-precision input scale 2^-e is applied to the reduced row at the
// end: scaling by a power of two commutes exactly with the products and
// sums.
// ---------------------------------------------------------------------------
template <typename T, bool SCALED, bool KEVEN, int WSCH, int RT, int NW, bool MS, bool ONE, int NBC>
__global__ void __launch_bounds__(64 * NW, 8 / NW) pc_kernel(PcArgs p) {
    constexpr int RG = 4 / RT;    // row groups
    constexpr int KGN = NW / RG;  // chunk groups
    constexpr int OLD = 64 + 4;   // LDS row stride of the Omega tile
    typedef typename Acc<T>::type acc_t;
    typedef typename Vec4<T>::type v4;
    __shared__ T om_s[64 * OLD];
    __shared__ T red[NW][64];
    const int K = p.r1, n = p.n;
    // grid z: slices of one term, or (term, slice) pairs of a grouped launch
    const int nt = max(p.terms, 1), S = gridDim.z / nt;
    const int term = blockIdx.z / S, zs = blockIdx.z - term * S;
    const Slice sl = slice_of(K, zs, S);
    const int nck = sl.rows16 / 16;
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wr = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rg = wr % RG, kg = wr / RG;
    const int wk0 = sl.kb0 + 16 * ((kg * nck) / KGN);
    const int wk1 = min(sl.kb1, sl.kb0 + 16 * (((kg + 1) * nck) / KGN));
    const bool has_k = wk1 > wk0;  // uniform per wave
    const int colbase = p.c0 + blockIdx.y * 64;
    const int ncb = min(64, p.c0 + p.nc - colbase);
    const double* Xa = (nt > 1 ? p.Xt[term] : p.X) + (size_t)a * n * K;
    const T* Wn = static_cast<const T*>(nt > 1 ? p.Wnt[term] : p.Wn);

    // Omega tile rows rc..rc+63, columns colbase..colbase+63 (zero outside
    // n x ncb): thread -> one row, 8 consecutive columns
    constexpr int OT = 64 * 8 / (64 * NW);  // 8-column pieces per thread
    double od[OT][8];
    auto load_om = [&](int rc) {
#pragma unroll
        for (int j = 0; j < OT; ++j) {
            const int q = tid + j * 64 * NW, r = q >> 3, c8 = (q & 7) * 8;
            const double* orow = p.Om + (size_t)min(rc + r, n - 1) * p.ldo + colbase;
#pragma unroll
            for (int e = 0; e < 8; ++e) od[j][e] = orow[min(c8 + e, ncb - 1)];
        }
    };
    auto store_om = [&](int rc) {
#pragma unroll
        for (int j = 0; j < OT; ++j) {
            const int q = tid + j * 64 * NW, r = q >> 3, c8 = (q & 7) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                om_s[r * OLD + c8 + e] = (rc + r < n && c8 + e < ncb) ? (T)od[j][e] : T(0);
        }
    };

    // operands of one slab, loaded in chunk order (core rows of every tile,
    // then the W entries of that chunk) so the MFMAs of the first chunk wait
    // only for its own data
    double xb[RT][4 * WSCH];
    v4 wb[WSCH][4];
    auto load = [&](int rc, int k0) {
        if (Wn == nullptr) {  // the last core: W_{d+1} = 1 (K = 1)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                load_x<KEVEN, WSCH>(Xa + (size_t)min(rc + 16 * (RT * rg + t) + li, n - 1) * K, wk1, k0, lg,
                                    xb[t]);
#pragma unroll
            for (int c = 0; c < WSCH; ++c)
#pragma unroll
                for (int nb = 0; nb < NBC; ++nb) wb[c][nb] = v4{T(k0 + 16 * c + 4 * lg == 0), T(0), T(0), T(0)};
            return;
        }
        const double* xr[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) xr[t] = Xa + (size_t)min(rc + 16 * (RT * rg + t) + li, n - 1) * K;
        const T* wcol[4];
#pragma unroll
        for (int nb = 0; nb < NBC; ++nb)
            wcol[nb] = Wn + (size_t)(colbase + min(16 * nb + li, ncb - 1)) * p.in_ld;
        const int bmax = (int)p.in_ld - 4;
#pragma unroll
        for (int c = 0; c < WSCH; ++c) {
            const int kb = k0 + 16 * c + 4 * lg;  // first of this lane's 4 b
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if (KEVEN) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double2_t v = *reinterpret_cast<const double2_t*>(xr[t] + min(kb + 2 * h, wk1 - 2));
                        xb[t][4 * c + 2 * h] = v[0];
                        xb[t][4 * c + 2 * h + 1] = v[1];
                    }
                } else {
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) xb[t][4 * c + s2] = xr[t][min(kb + s2, wk1 - 1)];
                }
            }
            // 4 consecutive b of one column: one 16-byte load per chunk and
            // column tile in the transposed layout
#pragma unroll
            for (int nb = 0; nb < NBC; ++nb) wb[c][nb] = *reinterpret_cast<const v4*>(wcol[nb] + min(kb, bmax));
        }
        if (MS) {
            for (int s = 1; s < p.in_slices; ++s)
#pragma unroll
                for (int c = 0; c < WSCH; ++c)
#pragma unroll
                    for (int nb = 0; nb < NBC; ++nb)
                        wb[c][nb] += *reinterpret_cast<const v4*>(wcol[nb] + s * p.in_ss +
                                                                  min(k0 + 16 * c + 4 * lg, bmax));
        }
    };

    // issue order: input exponents and Omega first (waiting for them does
    // not wait for the operands issued after them), then the first slab
    ExpLoads ex;
    if (SCALED) ex = issue_input_exponent(p);
    load_om(0);
    if (has_k) load(0, wk0);
    store_om(0);
    const int in_e = SCALED ? input_exponent(p, ex) : 0;

    T part[4] = {T(0), T(0), T(0), T(0)};
    for (int rc = 0; ONE ? rc == 0 : rc < n; rc += 64) {
        if (!ONE && rc > 0) {
            load_om(rc);
            __syncthreads();  // every wave has folded the previous tile
            store_om(rc);
        }
        acc_t acc[RT][4];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int nb = 0; nb < NBC; ++nb) acc[t][nb] = acc_t{0, 0, 0, 0};
        if (has_k) {
            for (int k0 = wk0; ONE ? k0 == wk0 : k0 < wk1; k0 += 16 * WSCH) {
#pragma unroll
                for (int c = 0; c < WSCH; ++c) {
                    const int kc = k0 + 16 * c;
                    if (kc < wk1) {
                        // W entries beyond K (clamped loads) are zeroed; the
                        // matching core values are finite copies
                        const bool tail = kc + 16 > K;
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) {
                            const bool kok = !tail || kc + 4 * lg + s2 < K;
#pragma unroll
                            for (int t = 0; t < RT; ++t) {
                                const T av = (T)xb[t][4 * c + s2];
#pragma unroll
                                for (int nb = 0; nb < NBC; ++nb)
                                    acc[t][nb] = Acc<T>::mma(av, kok ? wb[c][nb][s2] : T(0), acc[t][nb]);
                            }
                        }
                    }
                }
                if (!ONE) {
                    const int nk0 = k0 + 16 * WSCH;
                    if (nk0 < wk1)
                        load(rc, nk0);
                    else if (rc + 64 < n)
                        load(rc + 64, wk0);
                }
            }
        }
        __syncthreads();  // the Omega tile is in LDS
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T* orow = om_s + (16 * (RT * rg + t) + Acc<T>::row(lg, v)) * OLD + li;
#pragma unroll
                for (int nb = 0; nb < NBC; ++nb) part[nb] += acc[t][nb][v] * orow[16 * nb];
            }
    }
#pragma unroll
    for (int nb = 0; nb < NBC; ++nb) {
        part[nb] += __shfl_xor(part[nb], 16, 64);
        part[nb] += __shfl_xor(part[nb], 32, 64);
    }
    if (lg == 0) {
#pragma unroll
        for (int nb = 0; nb < NBC; ++nb) red[wr][nb * 16 + li] = part[nb];
    }
    __syncthreads();
    if (tid < 64) {  // the whole first wave: track_exponents reduces over it
        const int c = tid;
        T v = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
        if (NW == 8) v += (red[4][c] + red[5][c]) + (red[6][c] + red[7][c]);
        if (SCALED) v *= (T)ldexp(1.0, -in_e);
        T* Wo = static_cast<T*>(nt > 1 ? p.Woutt[term] : p.Wout) + zs * p.out_ss;
        if (c < ncb) Wo[(size_t)(colbase + c) * p.out_ld + a] = v;
        if (SCALED) track_exponents(p, a, colbase, c, ncb, (double)v, in_e);
    }
}

// ---------------------------------------------------------------------------
// BF16 kernel: a lane's four consecutive k of a 16-wide chunk are exactly
// its A operand of v_mfma_f32_16x16x16_bf16, so one MFMA covers a chunk; the
// W slice is staged transposed (column-major in LDS) so the matching B
// operand is one 8-byte LDS read.
// ---------------------------------------------------------------------------
template <bool KEVEN, int WSCH>
__global__ void __launch_bounds__(256, 2) pc_bf16_kernel(PcArgs p) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = p.r1, n = p.n;
    const Slice sl = slice_of(K, blockIdx.z, gridDim.z);
    const int LDK = sl.rows16 + 8;  // transposed row stride (bf16 elements)
    unsigned short* Wt = reinterpret_cast<unsigned short*>(smem_raw);  // 64 x LDK
    float* red = reinterpret_cast<float*>(Wt + (size_t)64 * LDK);       // [4][64]
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wr = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int colbase = p.c0 + blockIdx.y * 64;
    const int ncb = min(64, p.c0 + p.nc - colbase);
    const unsigned short* Wn = static_cast<const unsigned short*>(p.Wn);
    const double* Xa = p.X + (size_t)a * n * K;
    const int in_e = input_exponent(p);
    const float in_scale = (float)ldexp(1.0, -in_e);

    double buf[4 * WSCH];
    auto load = [&](int rc, int k0) {
        load_x<KEVEN, WSCH>(Xa + (size_t)min(rc + 16 * wr + li, n - 1) * K, sl.kb1, k0, lg, buf);
    };
    // Stage the slice transposed (LDS row per column): thread -> (column c,
    // 8 consecutive b), slices summed in FP32 in slice order, scaled,
    // rounded once to bfloat16.
    load(0, sl.kb0);
    {
        const int total = sl.rows16 * 64 / 8;  // 8-element pieces
        for (int q = tid; q < total; q += 256) {
            const int c = q / (sl.rows16 / 8), r = (q - c * (sl.rows16 / 8)) * 8;
            const int cc = colbase + min(c, ncb - 1);
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = sl.kb0 + r + j;
                const size_t off = (size_t)cc * p.in_ld + min(k, K - 1);
                float x;
                if (Wn) {
                    x = bf16_to_f32(Wn[off]);
                    for (int s = 1; s < p.in_slices; ++s) x += bf16_to_f32(Wn[s * p.in_ss + off]);
                } else {
                    x = (k == 0) ? 1.f : 0.f;
                }
                v[j] = (k < K && c < ncb) ? x * in_scale : 0.f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) Wt[c * LDK + r + j] = bf16_rne(v[j]);
        }
    }
    __syncthreads();

    // B operands of one chunk, read from LDS one chunk ahead of their MFMAs
    auto read_b = [&](int rel, bf16x4_t (&bv)[4]) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            bv[nb] = *reinterpret_cast<const bf16x4_t*>(Wt + (nb * 16 + li) * LDK + rel + 4 * lg);
    };
    bf16x4_t bq[4];
    read_b(0, bq);
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
        const bool rok = rc + 16 * wr + li < n;
        for (int k0 = sl.kb0; k0 < sl.kb1; k0 += 16 * WSCH) {
#pragma unroll
            for (int c = 0; c < WSCH; ++c) {
                const int kc = k0 + 16 * c;
                if (kc < sl.kb1) {
                    bf16x4_t bn[4];
                    read_b(kc + 16 < sl.kb1 ? kc + 16 - sl.kb0 : 0, bn);
                    bf16x4_t av;
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) {
                        const bool ok = rok && kc + 4 * lg + s2 < sl.kb1;
                        av[s2] = (short)bf16_rne(ok ? (float)buf[4 * c + s2] : 0.f);
                    }
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bq[nb], acc[nb], 0, 0, 0);
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) bq[nb] = bn[nb];
                }
            }
            const int nk0 = k0 + 16 * WSCH;
            if (nk0 < sl.kb1)
                load(rc, nk0);
            else if (rc + 64 < n)
                load(rc + 64, sl.kb0);
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
        for (int nb = 0; nb < 4; ++nb) red[wr * 64 + nb * 16 + li] = part[nb];
    }
    __syncthreads();
    if (tid < 64) {
        const int c = tid;
        const float v = (red[c] + red[64 + c]) + (red[128 + c] + red[192 + c]);
        const unsigned short hv = bf16_rne(v);
        unsigned short* Wo = static_cast<unsigned short*>(p.Wout) + blockIdx.z * p.out_ss;
        if (c < ncb) Wo[(size_t)(colbase + c) * p.out_ld + a] = hv;
        track_exponents(p, a, colbase, c, ncb, (double)bf16_to_f32(hv), in_e);
    }
}

// W_k as float64: the sum of its slices in slice order (in the storage's
// arithmetic type: FP64, or FP32 for FP32 and bfloat16 storage), times
// 2^colexp for reduced precision.
template <typename T>
struct Stored;
template <>
struct Stored<double> {
    typedef double acc;
    static __device__ __forceinline__ double get(const double* w, size_t i) { return w[i]; }
};
template <>
struct Stored<float> {
    typedef float acc;
    static __device__ __forceinline__ float get(const float* w, size_t i) { return w[i]; }
};
template <>
struct Stored<unsigned short> {
    typedef float acc;
    static __device__ __forceinline__ float get(const unsigned short* w, size_t i) {
        return bf16_to_f32(w[i]);
    }
};

template <typename T>
__global__ void w_export_kernel(const T* w, const int* colexp, int64_t ld, int rows, int c0, int nc,
                                int slices, int64_t sstride, double* out, int64_t ldo) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * nc) return;
    const int r = (int)(t / nc), c = (int)(t - (int64_t)r * nc);
    const size_t off = (size_t)(c0 + c) * ld + r;
    typename Stored<T>::acc v = Stored<T>::get(w, off);
    for (int s = 1; s < slices; ++s) v += Stored<T>::get(w, s * sstride + off);
    out[(size_t)r * ldo + c] = colexp ? ldexp((double)v, colexp[c0 + c]) : (double)v;
}

__global__ void fill_int_kernel(int* p, int value, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = value;
}

template <typename K>
void allow_lds(K kern) {
    static const hipError_t attr = hipFuncSetAttribute(
        (const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    (void)attr;
}

template <typename T, bool SCALED, int NW, bool MS, int NBC>
void launch_mfma_nbc(const PcArgs& a, const dim3& grid, int max_wave_chunks, hipStream_t s) {
    // row tiles per wave and chunks per slab (register budget); when n <= 64
    // and every wave's chunks fit one slab of ONE_WS, all its operands are
    // requested at once
    constexpr int RT = sizeof(T) == 8 ? 1 : 4;
    constexpr int WS = 1;
    constexpr int ONE_WS = 2;
    const dim3 block(64 * NW);
    if (max_wave_chunks <= ONE_WS && a.n <= 64) {
        if (a.r1 % 2 == 0)
            hipLaunchKernelGGL((pc_kernel<T, SCALED, true, ONE_WS, RT, NW, MS, true, NBC>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pc_kernel<T, SCALED, false, ONE_WS, RT, NW, MS, true, NBC>), grid, block, 0, s, a);
    } else {
        if (a.r1 % 2 == 0)
            hipLaunchKernelGGL((pc_kernel<T, SCALED, true, WS, RT, NW, MS, false, NBC>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((pc_kernel<T, SCALED, false, WS, RT, NW, MS, false, NBC>), grid, block, 0, s, a);
    }
}

template <typename T, bool SCALED, int NW, bool MS>
void launch_mfma_nw(const PcArgs& a, const dim3& grid, int max_wave_chunks, hipStream_t s) {
    // 16-column tiles: fewer than four only when the launch has one column
    // block of at most 48 columns
    const int nbc = a.nc > 48 ? 4 : std::max(1, ceil_div(a.nc, 16));
    if (nbc == 1)
        launch_mfma_nbc<T, SCALED, NW, MS, 1>(a, grid, max_wave_chunks, s);
    else if (nbc == 2)
        launch_mfma_nbc<T, SCALED, NW, MS, 2>(a, grid, max_wave_chunks, s);
    else if (nbc == 3)
        launch_mfma_nbc<T, SCALED, NW, MS, 3>(a, grid, max_wave_chunks, s);
    else
        launch_mfma_nbc<T, SCALED, NW, MS, 4>(a, grid, max_wave_chunks, s);
}

void check_pc_args(const PcArgs& a, size_t esz) {
    if (a.Wn != nullptr) {
        if (a.in_slices < 1) throw Error(-6, "partial contraction: bad slice count");
        if (a.in_ld < 4 || a.in_ld % 4 != 0 || a.in_ld < a.r1 || a.in_ss % 4 != 0 ||
            reinterpret_cast<uintptr_t>(a.Wn) % (4 * esz) != 0)
            throw Error(-6, "partial contraction: W_{k+1} storage must be 4-element aligned");
    }
    if (a.out_ld < a.r0) throw Error(-6, "partial contraction: W_k row stride too small");
}

template <typename T, bool SCALED>
void launch_mfma(const PcArgs& a, hipStream_t s) {
    check_pc_args(a, sizeof(T));
    const int terms = std::max(a.terms, 1);
    if (terms > 1 && (SCALED || !a.Xt || !a.Woutt || !a.Wnt))
        throw Error(-6, "partial contraction: grouped terms need FP64 and pointer tables");
    const int S = pc_slices((int64_t)a.r0 * terms, a.r1, sizeof(T) == 8 ? 0 : 1);
    const int rows16 = 16 * ceil_div(ceil_div(a.r1, 16), S);  // largest slice
    const dim3 grid(a.r0, ceil_div(a.nc, 64), S * terms);
    // eight waves when the slices are long enough to give every chunk group work
    const bool ms = a.Wn != nullptr && a.in_slices > 1;
    const int nck = rows16 / 16;
    constexpr int RG = sizeof(T) == 8 ? 4 : 1;  // row groups per workgroup
    if (rows16 >= 16 * 8) {
        const int wc = ceil_div(nck, 8 / RG);
        if (ms)
            launch_mfma_nw<T, SCALED, 8, true>(a, grid, wc, s);
        else
            launch_mfma_nw<T, SCALED, 8, false>(a, grid, wc, s);
    } else {
        const int wc = ceil_div(nck, 4 / RG);
        if (ms)
            launch_mfma_nw<T, SCALED, 4, true>(a, grid, wc, s);
        else
            launch_mfma_nw<T, SCALED, 4, false>(a, grid, wc, s);
    }
    TTR_CHECK_LAUNCH();
}

}  // namespace

int pc_slices(int64_t r0, int64_t r1, int prec) {
    const int chunks = ceil_div(std::max<int64_t>(r1, 1), 16);
    // with 160 or more rows one workgroup per row keeps most CUs busy and
    // every consumer reads W_k once; fewer rows are sliced up to four ways
    // toward one workgroup per CU
    const int64_t rr = std::max<int64_t>(r0, 1);
    const int s_occ = rr >= 160 ? 1 : (int)std::min<int64_t>(4, (256 + rr - 1) / rr);
    // and, for BF16, a staged slice within the LDS budget
    const int s_lds = prec == 2 ? ceil_div(chunks, (int)(kSliceLds / ((size_t)64 * 16 * 2))) : 1;
    return std::max(1, std::min(chunks, std::max(s_occ, s_lds)));
}

void launch_pc_f64(const PcArgs& a, hipStream_t s) { launch_mfma<double, false>(a, s); }

void launch_pc_f32(const PcArgs& a, hipStream_t s) { launch_mfma<float, true>(a, s); }

void launch_pc_bf16(const PcArgs& a, hipStream_t s) {
    check_pc_args(a, 2);
    if (a.terms > 1) throw Error(-6, "partial contraction: grouped terms need FP64");
    const int S = pc_slices(a.r0, a.r1, 2);
    const int rows16 = 16 * ceil_div(ceil_div(a.r1, 16), S);
    const size_t lds = (size_t)64 * (rows16 + 8) * 2 + (size_t)4 * 64 * 4;
    if (lds > kLdsMax) throw Error(-6, "partial contraction: W slice does not fit in LDS");
    const dim3 grid(a.r0, ceil_div(a.nc, 64), S);
    if (a.r1 % 2 == 0) {
        auto kern = pc_bf16_kernel<true, 8>;
        allow_lds(kern);
        hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, a);
    } else {
        auto kern = pc_bf16_kernel<false, 4>;
        allow_lds(kern);
        hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, a);
    }
    TTR_CHECK_LAUNCH();
}

void launch_fill_int(int* p, int value, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(fill_int_kernel, dim3(ceil_div(count, 256)), dim3(256), 0, s, p, value,
                       count);
    TTR_CHECK_LAUNCH();
}

void launch_w_export(int prec, const void* w, const int* colexp, int64_t ld, int rows, int c0,
                     int nc, int slices, int64_t sstride, double* out, int64_t ldo, hipStream_t s) {
    const int64_t work = (int64_t)rows * nc;
    if (work <= 0) return;
    const dim3 g(ceil_div(work, 256));
    if (prec == 0)
        hipLaunchKernelGGL(w_export_kernel<double>, g, dim3(256), 0, s, static_cast<const double*>(w),
                           nullptr, ld, rows, c0, nc, slices, sstride, out, ldo);
    else if (prec == 1)
        hipLaunchKernelGGL(w_export_kernel<float>, g, dim3(256), 0, s, static_cast<const float*>(w),
                           colexp, ld, rows, c0, nc, slices, sstride, out, ldo);
    else
        hipLaunchKernelGGL(w_export_kernel<unsigned short>, g, dim3(256), 0, s,
                           static_cast<const unsigned short*>(w), colexp, ld, rows, c0, nc, slices,
                           sstride, out, ldo);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
