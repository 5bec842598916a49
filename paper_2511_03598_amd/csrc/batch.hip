// Batched adaptive KRP TT-rounding in one persistent launch (the adaptive
// rank algorithm of Sec. 3.3 with the right-to-left partial contractions of
// Sec. 3.1, applied to many independent tensors).
//
// The whole rounding of a tensor -- Gaussian factors, partial
// contractions, the Remark 1 norm estimate, and for every mode the sketch,
// the thin QR, the residual sketch and estimator, the basis growth with
// regenerated sketch columns, the projection and the next core -- runs as
// device code, so the adaptive decisions (est > tau, regeneration) are
// taken on the device and the launch needs no host round trip: it can be
// recorded in a HIP graph.
//
// Workgroups (256 threads, four waves) take tickets from a device counter.
// Ticket s belongs to tensor order[t] with prefix[t] <= s < prefix[t+1]; the
// T = prefix[t+1] - prefix[t] workgroups holding that tensor's tickets form
// its team and split each step's work: rows of tall panels by member,
// output tiles of products over the team's workgroups.  Members meet at
// team barriers (an arrival counter and a generation word in device
// memory); small reduced results (Gram matrices, Q^T S, the estimate) are
// summed by every member from per-member partial slots in member order, so
// every member takes the same decisions.  Tensors are handed out largest
// first, so a team waits only for workgroups that are finishing earlier
// tensors: with the grid no larger than the resident workgroups and T at
// most half of them, every team completes.  Every barrier wait is bounded;
// a wait that times out sets the tensor's status bit and the kernel still
// ends.
//
// Products stream the tall operand straight into MFMA layout, each wave
// through two register stages (the next step's loads in flight during the
// current MFMAs), with K steps paired so that an operand contiguous along K
// is one 16-byte load per lane: tall panels times small matrices
// (sketches, residual updates, R^{-1} applications) run over 16-row blocks
// per wave with the small matrix staged in LDS; long-K reductions with
// small outputs (Gram matrices, Q^T S, the projection) stream K per wave
// and add the four wave partials in wave order; the partial contractions
// stream (row, 16-row block, K step) per wave with W_{k+1}'s column block
// in LDS; the next core streams the columns of H(X_{k+1}) with 64 rows of
// the projection in LDS.  The last core's contraction (and products with
// more than 128 rows of K) use 64 x 64 tiles staged through LDS.  The steps
// are out-of-line functions so that each gets its own register budget.
//
// All reductions run in an order fixed by the tensor's shape and team size,
// and the team size depends on the tensor alone, so a tensor's result is
// bitwise the same whatever else is in the batch.
#include "batch.hpp"

#include <algorithm>

#include "kernels.hpp"
#include "philox.hpp"

namespace ttr {
namespace {

// LDS (71 KB of the CU's 160 KB; one workgroup per CU): the b x b Gram /
// Cholesky factor G, or the double-buffered GEMM slabs, or a 64-column
// block of W_{k+1} (never live at the same time), then misc scratch.
constexpr int kLD = kBatchMaxBlock + 1;                        // LDS stride of b x b matrices
constexpr int kSlab = 16;                                      // K depth of a staged GEMM slab
constexpr int kSP = 68;                                        // LDS stride of a staged slab row
constexpr int kSlabDoubles = kSlab * kSP;                      // one 64 x 16 panel slab
constexpr int kStageDoubles = 4 * kSlabDoubles;                // A and B slabs, double-buffered
constexpr int kWRows = 128, kWLD = 68;                          // W_{k+1} column block held in LDS
constexpr int kWDoubles = kWRows * kWLD;
constexpr int kMisc = std::max({kBatchMaxBlock * kLD, kStageDoubles, kWDoubles});
constexpr int kLdsDoubles = kMisc + 2 * kBatchMaxBlock + 16;  // G, misc
static_assert(kLdsDoubles * 8 + 16 <= 80 * 1024, "LDS layout must stay below 80 KiB");
static_assert(4 * 256 <= kMisc, "atb's wave partial tiles must fit below misc");
constexpr double kUnit = 1.1102230246251565e-16;               // 2^-53
constexpr uint64_t kSpinTicks = 500000000ull;                  // 5 s of the 100 MHz wall clock

// Global-memory views of device pointers: loads and stores through them
// compile to global_* instructions (counted by vmcnt alone) instead of
// flat_* ones, which the compiler must also count as LDS accesses.
typedef __attribute__((address_space(1))) double gdouble;
// two doubles at an 8-byte aligned address (one 16-byte global load)
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef __attribute__((address_space(1))) d2u gd2u;
__device__ __forceinline__ const gdouble* gptr(const double* p) { return (const gdouble*)p; }
__device__ __forceinline__ gdouble* gptr(double* p) { return (gdouble*)p; }

// LDS pointer: functions that take one address LDS with ds_* instructions
// even when they are not inlined.
typedef __attribute__((address_space(3))) double ldouble;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// ---------------------------------------------------------------------------
// Team barrier
// ---------------------------------------------------------------------------
// Agent-scope fences on gfx950 act on the whole L2 of the calling XCD (a
// release writes its dirty lines back, an acquire invalidates it), and that
// L2 is shared with the other workgroups of the XCD.  So the barrier takes
// one release fence before arriving and one acquire fence after leaving,
// and thread 0 polls the generation word with relaxed loads: an acquiring
// poll would invalidate the L2 once per poll for as long as the member waits.
// The arrival is a release read-modify-write, which also keeps the read of
// the old generation before the arrival.  Thread 0's own acquire fences
// complete the chain: the last member to arrive acquires the others'
// releases on the counter before it releases the generation, and a waiting
// member acquires that release before the workgroup barrier passes it on.
__device__ __forceinline__ void team_sync(const BatchTT& t) {
    if (t.T == 1) {
        __syncthreads();
        return;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0 && !(__hip_atomic_load(t.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1)) {
        unsigned* cnt = t.bar;
        unsigned* gen = t.bar + 1;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == (unsigned)t.T - 1u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > kSpinTicks) {
                    __hip_atomic_fetch_or(t.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Rows [rb, re) of member m of T for a matrix of `rows` rows, in 16-row blocks.
__device__ __forceinline__ void member_rows(int rows, int T, int m, int& rb, int& re) {
    const int64_t blocks = (rows + 15) >> 4;
    rb = (int)min<int64_t>(rows, (blocks * m / T) * 16);
    re = (int)min<int64_t>(rows, (blocks * (m + 1) / T) * 16);
}

// ---------------------------------------------------------------------------
// Workgroup-level MFMA tiles (v_mfma_f64_16x16x4_f64) staged through LDS
// ---------------------------------------------------------------------------
// An operand panel is viewed as P(r, k) = p[r*rs + k*cs]: for the left
// factor r is the output row, for the right factor r is the output column
// (B(k, c) = P(c, k) with rs = B's column stride, cs = its row stride).
// Each K slab (kSlab deep) of a 64-row panel is loaded by the workgroup's
// 256 threads, four elements each, along whichever index is contiguous,
// and stored k-major in LDS (stride kSP) so that the 16 lanes of an MFMA
// operand read 16 consecutive r at one k.  Out-of-range elements are read
// at a clamped index (every load is issued unconditionally) and zeroed.
static_assert(kStageDoubles <= kMisc, "GEMM staging must fit below the misc area");

struct Panel {
    const double* p;
    int64_t rs, cs;
    int R;  // valid rows (r < R)
};

struct Slab4 {
    double v[4];
};

__device__ __forceinline__ void slab_load(const Panel& P, int r0, int k, int k1, Slab4& s) {
    const int tid = threadIdx.x;
    const gdouble* g = gptr(P.p);
    if (P.cs == 1) {
        const int r = tid >> 2, kq = (tid & 3) * 4;
        const int gr = r0 + r;
        const int64_t base = (int64_t)min(gr, P.R - 1) * P.rs;
        const int gk0 = k + kq;
        if (gr < P.R && gk0 + 4 <= k1) {  // four in-range neighbours: two 16-byte loads
            const d2u v0 = *(const gd2u*)(g + base + gk0), v1 = *(const gd2u*)(g + base + gk0 + 2);
            s.v[0] = v0[0];
            s.v[1] = v0[1];
            s.v[2] = v1[0];
            s.v[3] = v1[1];
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gk = gk0 + q;
            const double v = g[base + min(gk, k1 - 1)];
            s.v[q] = (gr < P.R && gk < k1) ? v : 0.0;
        }
    } else {
        const int kk = tid >> 4, rq = (tid & 15) * 4;
        const int gk = k + kk;
        const int64_t kb = (int64_t)min(gk, k1 - 1) * P.cs;
        const int gr0 = r0 + rq;
        if (P.rs == 1 && gk < k1 && gr0 + 4 <= P.R) {  // four consecutive rows in one column
            const d2u v0 = *(const gd2u*)(g + gr0 + kb), v1 = *(const gd2u*)(g + gr0 + 2 + kb);
            s.v[0] = v0[0];
            s.v[1] = v0[1];
            s.v[2] = v1[0];
            s.v[3] = v1[1];
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gr = gr0 + q;
            const double v = g[(int64_t)min(gr, P.R - 1) * P.rs + kb];
            s.v[q] = (gr < P.R && gk < k1) ? v : 0.0;
        }
    }
}

__device__ __forceinline__ void slab_store(const Panel& P, const Slab4& s, ldouble* L) {
    const int tid = threadIdx.x;
    if (P.cs == 1) {
        const int r = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) L[(kq + q) * kSP + r] = s.v[q];
    } else {
        const int kk = tid >> 4, rq = (tid & 15) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) L[kk * kSP + rq + q] = s.v[q];
    }
}

template <int TN>
__device__ __forceinline__ void zero_acc(double4_t (&acc)[TN]) {
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
}

// acc += A[m0:m0+64, k0:k1] B[k0:k1, n0:n0+16TN] for this wave's 16 rows
// (m0+16w .. +16) and all TN column blocks.  Every thread of the
// workgroup must call it (it stages through LDS and synchronises); lds
// holds kStageDoubles.  Accumulator element v of lane l in block j is row
// m0 + 16w + l/16 + 4v, column n0 + 16j + l%16.
template <int TN>
__device__ __forceinline__ void wg_tile(const Panel& A, const Panel& B, int m0, int n0, int k0, int k1,
                                        double4_t (&acc)[TN], ldouble* lds) {
    const int l = lane_id(), li = l & 15, lg = l >> 4, w = wave_id();
    const int nslab = (k1 - k0 + kSlab - 1) / kSlab;
    if (nslab <= 0) return;
    Slab4 ra, rb;
    slab_load(A, m0, k0, k1, ra);
    slab_load(B, n0, k0, k1, rb);
    slab_store(A, ra, lds);
    slab_store(B, rb, lds + kSlabDoubles);
    __syncthreads();
    for (int s = 0; s < nslab; ++s) {
        const bool more = s + 1 < nslab;
        if (more) {
            slab_load(A, m0, k0 + (s + 1) * kSlab, k1, ra);
            slab_load(B, n0, k0 + (s + 1) * kSlab, k1, rb);
        }
        const ldouble* As = lds + (s & 1) * 2 * kSlabDoubles;
        const ldouble* Bs = As + kSlabDoubles;
#pragma unroll
        for (int q = 0; q < kSlab / 4; ++q) {
            const double a = As[(4 * q + lg) * kSP + 16 * w + li];
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[j] = mfma_f64_16x16x4(a, Bs[(4 * q + lg) * kSP + 16 * j + li], acc[j]);
        }
        if (more) {
            ldouble* An = lds + ((s + 1) & 1) * 2 * kSlabDoubles;
            slab_store(A, ra, An);
            slab_store(B, rb, An + kSlabDoubles);
        }
        __syncthreads();
    }
}

// C(r, c) = alpha * acc + beta * C(r, c) for r < M, c < N.
template <int TN>
__device__ __forceinline__ void tile_store(double* C, int64_t crs, int64_t ccs, int M, int N, int m0, int n0,
                                           const double4_t (&acc)[TN], double alpha, double beta) {
    const int l = lane_id(), li = l & 15, lg = l >> 4, w = wave_id();
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = m0 + 16 * w + lg + 4 * v, c = n0 + 16 * j + li;
            if (r < M && c < N) {
                gdouble* p = gptr(C) + (int64_t)r * crs + (int64_t)c * ccs;
                double x = alpha * acc[j][v];
                if (beta != 0.0) x += beta * *p;
                *p = x;
            }
        }
}

// C[rb:re, 0:N] = alpha A[rb:re, 0:K] B[0:K, 0:N] + beta C, A(r, k) =
// A[r*ars + k*acs], B(k, c) = B[k*brs + c*bcs]; tiles of 64 x 16TN handed to
// workgroups g, g+G, ... of the team.  With N <= 16TN one tile spans every
// column, so C may be A itself (each tile reads all of its A rows before
// any store).
template <int TN>
__device__ __forceinline__ void wg_gemm_t(const double* A, int64_t ars, int64_t acs, const double* B, int64_t brs,
                                          int64_t bcs, double* C, int64_t crs, int64_t ccs, int rb, int re, int N,
                                          int K, double alpha, double beta, int g, int G, ldouble* lds) {
    if (re <= rb || N <= 0) return;
    constexpr int tw = 16 * TN;
    const int nrt = (re - rb + 63) / 64, nct = (N + tw - 1) / tw;
    const Panel PA{A, ars, acs, re};
    const Panel PB{B, bcs, brs, N};
    for (int t = g; t < nrt * nct; t += G) {
        const int m0 = rb + (t / nct) * 64, n0 = (t % nct) * tw;
        double4_t acc[TN];
        zero_acc(acc);
        wg_tile<TN>(PA, PB, m0, n0, 0, K, acc, lds);
        tile_store<TN>(C, crs, ccs, re, N, m0, n0, acc, alpha, beta);
    }
}

__device__ __noinline__ void wg_gemm(const double* A, int64_t ars, int64_t acs, const double* B, int64_t brs,
                                     int64_t bcs, double* C, int64_t crs, int64_t ccs, int rb, int re, int N, int K,
                                     double alpha, double beta, int g, int G, ldouble* lds) {
    if (N <= 16)
        wg_gemm_t<1>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, g, G, lds);
    else if (N <= 32)
        wg_gemm_t<2>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, g, G, lds);
    else
        wg_gemm_t<4>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, g, G, lds);
}

// C[r0:r0+16, 0:N] = alpha A[r0:r0+16, 0:K] B[0:K, 0:N] + beta C for each of
// a wave's 16-row blocks of a tall panel (N <= 16 NB): A rows and B are
// loaded straight into MFMA layout, KS 4-deep K steps of loads at a time;
// every load of a block precedes its stores and other blocks' rows are
// disjoint, so C may be A.
// With GRAM the block's stored values X (16 rows x N, zero outside the
// panel) are also accumulated into gram[] = the upper blocks (j1 <= j2) of
// X^T X: a 16-row output tile in accumulator layout (lane l holds rows
// l/16 + 4v of column l%16) is exactly the A and the B operand of its own
// Gram product, four 4-deep steps over its rows.
template <int NB>
struct GramAcc {
    double4_t g[NB * (NB + 1) / 2];
};

// B(k, c) (K <= kWRows, N <= 64) into LDS at k kWLD + c, zero past N; every
// thread of the workgroup calls it, and a barrier must follow.
__device__ __forceinline__ void stage_b(const double* B, int64_t brs, int64_t bcs, int K, int N, ldouble* lds) {
    const gdouble* g = gptr(B);
    for (int e = threadIdx.x; e < K * 64; e += 256) {
        const int k = e >> 6, c = e & 63;
        lds[k * kWLD + c] = c < N ? g[(int64_t)k * brs + (int64_t)c * bcs] : 0.0;
    }
}

template <int NB, int KS, bool LB, bool GRAM = false>
__device__ __forceinline__ void rows_stream(const double* A, int64_t ars, int64_t acs, const double* B, int64_t brs,
                                            int64_t bcs, double* C, int64_t crs, int64_t ccs, int rb, int re, int N,
                                            int K, double alpha, double beta, const ldouble* wl,
                                            GramAcc<NB>* gram = nullptr) {
    // This wave's 16-row blocks r0 = rb + 16 w + 64 u in turn; each block's
    // K range in steps of 4 KS.  The (block, step) sequence runs through two
    // register stages, so the loads of the next step (possibly the next
    // block's first) are in flight during the MFMAs of the current one; the
    // per-block MFMA order and stores are those of one stage.
    const int l = lane_id(), li = l & 15, lg = l >> 4;
    const int rfirst = rb + 16 * wave_id();
    const int kit = (K + 4 * KS - 1) / (4 * KS);
    const int nblk = (rfirst < re && K > 0) ? (re - rfirst + 63) / 64 : 0;
    const int steps = nblk * kit;
    const gdouble* pb[NB];
    bool vb[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int c = 16 * j + li;
        vb[j] = c < N;
        pb[j] = gptr(B) + (int64_t)min(c, N - 1) * bcs;
    }
    // K steps in pairs as in atb_stream: lane group lg holds rows base +
    // 2 lg and base + 2 lg + 1 of the pair at base, so an A contiguous along
    // K (a row-major panel) is one 16-byte load per lane and pair
    static_assert(KS % 2 == 0, "K steps come in pairs");
    typedef double StageA[KS];
    typedef double StageB[KS][NB];
    typedef double StageC[NB][4];
    const bool acont = acs == 1;
    // with beta != 0 a block's last step also loads the C entries its
    // stores update, so no store waits for a load of its own
    auto load = [&](int st, StageA& a, StageB& b, StageC& cv) {
        const int blk = st / kit, ki = st - blk * kit, k = ki * 4 * KS;
        if (beta != 0.0 && ki == kit - 1) {  // uniform
            const int r0 = rfirst + 64 * blk;
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = min(r0 + lg + 4 * v, re - 1), c = min(16 * j + li, N - 1);
                    cv[j][v] = gptr(C)[(int64_t)rr * crs + (int64_t)c * ccs];
                }
        }
        const int r = rfirst + 64 * blk + li;
        const bool vr = r < re;
        const bool whole = k + 4 * KS <= K;  // uniform
        const gdouble* pa = gptr(A) + (int64_t)min(r, re - 1) * ars;
#pragma unroll
        for (int q = 0; q < KS / 2; ++q) {
            const int kk = k + 8 * q + 2 * lg;
            const bool ok0 = kk < K, ok1 = kk + 1 < K;
            const int64_t kc0 = min(kk, K - 1), kc1 = min(kk + 1, K - 1);
            double v0, v1;
            if (acont && whole) {
                const d2u v = *(const gd2u*)(pa + kk);
                v0 = v[0];
                v1 = v[1];
            } else {
                v0 = pa[kc0 * acs];
                v1 = pa[kc1 * acs];
            }
            a[2 * q] = (ok0 && vr) ? v0 : 0.0;
            a[2 * q + 1] = (ok1 && vr) ? v1 : 0.0;
            if (!LB) {
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double u0 = pb[j][kc0 * brs], u1 = pb[j][kc1 * brs];
                    b[2 * q][j] = (ok0 && vb[j]) ? u0 : 0.0;
                    b[2 * q + 1][j] = (ok1 && vb[j]) ? u1 : 0.0;
                }
            }
        }
    };
    double4_t acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
    // with B staged in LDS (LB) its entries are read just before their
    // MFMAs, so a register stage holds only A's rows
    auto mma = [&](int st, const StageA& a, const StageB& b) {
        if (LB) {
            const int k = (st % kit) * 4 * KS;
#pragma unroll
            for (int q = 0; q < KS / 2; ++q) {
                const int kk = k + 8 * q + 2 * lg;
                const bool ok0 = kk < K, ok1 = kk + 1 < K;
                const int kc0 = min(kk, K - 1), kc1 = min(kk + 1, K - 1);
                double u0[NB], u1[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double w0 = wl[kc0 * kWLD + 16 * j + li], w1 = wl[kc1 * kWLD + 16 * j + li];
                    u0[j] = (ok0 && vb[j]) ? w0 : 0.0;
                    u1[j] = (ok1 && vb[j]) ? w1 : 0.0;
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = mfma_f64_16x16x4(a[2 * q], u0[j], acc[j]);
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = mfma_f64_16x16x4(a[2 * q + 1], u1[j], acc[j]);
            }
        } else {
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = mfma_f64_16x16x4(a[s2], b[s2][j], acc[j]);
        }
    };
    // after the last step of a block: its stores (and Gram products)
    auto finish = [&](int blk, const StageC& cv) {
        const int r0 = rfirst + 64 * blk;
        double xs[NB][4];
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = r0 + lg + 4 * v, c = 16 * j + li;
                xs[j][v] = 0.0;
                if (rr < re && c < N) {
                    double x = alpha * acc[j][v];
                    if (beta != 0.0) x += beta * cv[j][v];
                    gptr(C)[(int64_t)rr * crs + (int64_t)c * ccs] = x;
                    xs[j][v] = x;
                }
            }
        if (GRAM) {
            int e = 0;
#pragma unroll
            for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
                for (int j2 = j1; j2 < NB; ++j2, ++e)
#pragma unroll
                    for (int v = 0; v < 4; ++v) gram->g[e] = mfma_f64_16x16x4(xs[j1][v], xs[j2][v], gram->g[e]);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
    };
    if (steps == 0) return;
    StageA a0, a1;
    StageB b0, b1;
    StageC c0, c1;
    load(0, a0, b0, c0);
    for (int st = 0; st < steps; st += 2) {  // uniform per wave
        const bool more1 = st + 1 < steps, more2 = st + 2 < steps;
        if (more1) load(st + 1, a1, b1, c1);
        mma(st, a0, b0);
        if ((st + 1) % kit == 0) finish(st / kit, c0);
        if (more2) load(st + 2, a0, b0, c0);
        if (more1) {
            mma(st + 1, a1, b1);
            if ((st + 2) % kit == 0) finish((st + 1) / kit, c1);
        }
    }
}

// Row-split product of one member: its rows [rb, re) of a panel of N <= 64
// columns, 16-row blocks handed to the four waves in turn (C may be A).
__device__ __noinline__ void gemm_rows(const double* A, int64_t ars, int64_t acs, const double* B, int64_t brs,
                                       int64_t bcs, double* C, int64_t crs, int64_t ccs, int rb, int re, int N, int K,
                                       double alpha, double beta, ldouble* lds) {
    if (re <= rb || N <= 0) return;
    // B (at most kWRows x 64) is read by every row block: staged in LDS
    const bool staged = K <= kWRows && N <= 64;
    if (staged) {
        stage_b(B, brs, bcs, K, N, lds);
        __syncthreads();
    }
    if (staged) {
        if (N <= 16 && K <= 16)  // one 16-deep step per block
            rows_stream<1, 4, true>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, lds);
        else if (N <= 16)
            rows_stream<1, 8, true>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, lds);
        else if (N <= 32)
            rows_stream<2, 8, true>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, lds);
        else
            rows_stream<4, 8, true>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, lds);
    } else {
        if (N <= 16)
            rows_stream<1, 8, false>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, nullptr);
        else if (N <= 32)
            rows_stream<2, 4, false>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, nullptr);
        else
            rows_stream<4, 4, false>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, nullptr);
    }
    if (staged) __syncthreads();  // the caller may reuse the LDS
}

// gemm_rows that also writes this member's partial Gram matrix of the
// stored block, P (N x N, row-major) = sum over its rows [rb, re) of
// C(r, i) C(r, j), the four wave partials added in wave order through LDS
// (a member without rows writes zeros).  This replaces the Gram pass that
// would otherwise read the block back.
template <int NB, int KS>
__device__ __forceinline__ void gemm_rows_gram_t(const double* A, int64_t ars, int64_t acs, const double* B,
                                                 int64_t brs, int64_t bcs, double* C, int64_t crs, int64_t ccs, int rb,
                                                 int re, int N, int K, double alpha, double beta, double* P,
                                                 ldouble* lds) {
    GramAcc<NB> ga;
#pragma unroll
    for (int e = 0; e < NB * (NB + 1) / 2; ++e) ga.g[e] = double4_t{0.0, 0.0, 0.0, 0.0};
    const bool staged = K <= kWRows && N <= 64;
    if (staged) {
        stage_b(B, brs, bcs, K, N, lds);
        __syncthreads();
    }
    if (staged)
        rows_stream<NB, KS, true, true>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, lds, &ga);
    else
        rows_stream<NB, KS, false, true>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, nullptr,
                                         &ga);
    const int l = lane_id(), li = l & 15, lg = l >> 4, w = wave_id(), tid = threadIdx.x;
    __syncthreads();  // the staged B and the caller's LDS contents are no longer needed
    int e = 0;
#pragma unroll
    for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
        for (int j2 = j1; j2 < NB; ++j2, ++e) {
#pragma unroll
            for (int v = 0; v < 4; ++v) lds[w * 256 + (lg + 4 * v) * 16 + li] = ga.g[e][v];
            __syncthreads();
            {
                const int r = tid >> 4, c = tid & 15;
                const int gi = 16 * j1 + r, gj = 16 * j2 + c;
                const double x = ((lds[tid] + lds[256 + tid]) + lds[512 + tid]) + lds[768 + tid];
                if (gi < N && gj < N) {
                    gptr(P)[(int64_t)gi * N + gj] = x;
                    if (j1 != j2) gptr(P)[(int64_t)gj * N + gi] = x;
                }
            }
            __syncthreads();
        }
}

__device__ __noinline__ void gemm_rows_gram(const double* A, int64_t ars, int64_t acs, const double* B, int64_t brs,
                                            int64_t bcs, double* C, int64_t crs, int64_t ccs, int rb, int re, int N,
                                            int K, double alpha, double beta, double* P, ldouble* lds) {
    if (N <= 16 && K <= 16)  // one 16-deep step per block
        gemm_rows_gram_t<1, 4>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, P, lds);
    else if (N <= 16)
        gemm_rows_gram_t<1, 8>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, P, lds);
    else if (N <= 32)
        gemm_rows_gram_t<2, 4>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, P, lds);
    else
        gemm_rows_gram_t<4, 2>(A, ars, acs, B, brs, bcs, C, crs, ccs, rb, re, N, K, alpha, beta, P, lds);
}

// P (Mo x No, row-major) = sum over k in [kb, ke) of A(i, k) B(k, j) for
// A(i, k) = A[i*ars + k*acs], B(k, j) = B[k*brs + j*bcs] and a long K (the
// rows of tall panels): each wave streams a contiguous quarter of K (16-row
// units) with its operands loaded straight into MFMA layout, 16 rows of
// loads issued before their MFMAs, and holds every 16 x 16 output block
// of the MB x NB block group; the four wave partials are then added in
// wave order through LDS.  Output block groups are done one after the
// other.
template <int MB, int NB, int KS = 4>
__device__ __forceinline__ void atb_stream(const double* A, int64_t ars, int64_t acs, int Mo, const double* B,
                                           int64_t brs, int64_t bcs, int No, int kb, int ke, int i0, int j0, double* P,
                                           ldouble* lds) {
    const int l = lane_id(), li = l & 15, lg = l >> 4, w = wave_id(), tid = threadIdx.x;
    const int blocks = (ke - kb + 15) / 16;
    const int k0 = kb + min(ke - kb, (blocks * w / 4) * 16);
    const int k1 = kb + min(ke - kb, (blocks * (w + 1) / 4) * 16);
    const gdouble* pa[MB];
    bool va[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int r = i0 + 16 * i + li;
        va[i] = r < Mo;
        pa[i] = gptr(A) + (int64_t)min(r, Mo - 1) * ars;
    }
    const gdouble* pb[NB];
    bool vb[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int c = j0 + 16 * j + li;
        vb[j] = c < No;
        pb[j] = gptr(B) + (int64_t)min(c, No - 1) * bcs;
    }
    double4_t acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    // Two register stages: the loads of the next 4 KS rows of K are issued
    // before the MFMAs of the current ones.  K steps go in pairs: in the
    // pair at base, lane group lg holds rows base + 2 lg (first step) and
    // base + 2 lg + 1 (second), so an operand contiguous along K (a
    // column-major panel) is one 16-byte load per lane and pair.
    static_assert(KS % 2 == 0, "K steps come in pairs");
    typedef double StageA[KS][MB];
    typedef double StageB[KS][NB];
    const bool acont = acs == 1, bcont = brs == 1;
    auto load = [&](int k, StageA& a, StageB& b) {
        const bool whole = k + 4 * KS <= k1;  // uniform: no row of the step past k1
#pragma unroll
        for (int q = 0; q < KS / 2; ++q) {
            const int kk = k + 8 * q + 2 * lg;
            const bool ok0 = kk < k1, ok1 = kk + 1 < k1;
            const int64_t kc0 = min(kk, k1 - 1), kc1 = min(kk + 1, k1 - 1);
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                double v0, v1;
                if (acont && whole) {
                    const d2u v = *(const gd2u*)(pa[i] + kk);
                    v0 = v[0];
                    v1 = v[1];
                } else {
                    v0 = pa[i][kc0 * acs];
                    v1 = pa[i][kc1 * acs];
                }
                a[2 * q][i] = (ok0 && va[i]) ? v0 : 0.0;
                a[2 * q + 1][i] = (ok1 && va[i]) ? v1 : 0.0;
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                double v0, v1;
                if (bcont && whole) {
                    const d2u v = *(const gd2u*)(pb[j] + kk);
                    v0 = v[0];
                    v1 = v[1];
                } else {
                    v0 = pb[j][kc0 * brs];
                    v1 = pb[j][kc1 * brs];
                }
                b[2 * q][j] = (ok0 && vb[j]) ? v0 : 0.0;
                b[2 * q + 1][j] = (ok1 && vb[j]) ? v1 : 0.0;
            }
        }
    };
    auto mma = [&](const StageA& a, const StageB& b) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[i][j] = mfma_f64_16x16x4(a[s][i], b[s][j], acc[i][j]);
    };
    StageA a0, a1;
    StageB b0, b1;
    if (k0 < k1) load(k0, a0, b0);
    for (int k = k0; k < k1; k += 8 * KS) {
        const bool more1 = k + 4 * KS < k1, more2 = k + 8 * KS < k1;  // uniform
        if (more1) load(k + 4 * KS, a1, b1);
        mma(a0, b0);
        if (more2) load(k + 8 * KS, a0, b0);
        if (more1) mma(a1, b1);
    }
    // wave partials of each block through LDS, added in wave order
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) lds[w * 256 + (lg + 4 * v) * 16 + li] = acc[i][j][v];
            __syncthreads();
            {
                const int r = tid >> 4, c = tid & 15;
                const int gr = i0 + 16 * i + r, gc = j0 + 16 * j + c;
                if (gr < Mo && gc < No)
                    gptr(P)[(int64_t)gr * No + gc] =
                        ((lds[tid] + lds[256 + tid]) + lds[512 + tid]) + lds[768 + tid];
            }
            __syncthreads();
        }
}

// P = A^T-style product over a long K (see atb_stream), in block groups of
// at most 8 output blocks of 16 x 16.
__device__ __noinline__ void atb(const double* A, int64_t ars, int64_t acs, int Mo, const double* B, int64_t brs,
                                 int64_t bcs, int No, int kb, int ke, double* P, ldouble* lds) {
    if (No <= 16) {
        for (int i0 = 0; i0 < Mo; i0 += 128) {
            const int mb = (min(Mo - i0, 128) + 15) / 16;
            if (mb <= 1)
                atb_stream<1, 1, 8>(A, ars, acs, Mo, B, brs, bcs, No, kb, ke, i0, 0, P, lds);
            else if (mb <= 2)
                atb_stream<2, 1, 8>(A, ars, acs, Mo, B, brs, bcs, No, kb, ke, i0, 0, P, lds);
            else if (mb <= 4)
                atb_stream<4, 1, 4>(A, ars, acs, Mo, B, brs, bcs, No, kb, ke, i0, 0, P, lds);
            else if (mb <= 6)
                atb_stream<6, 1, 2>(A, ars, acs, Mo, B, brs, bcs, No, kb, ke, i0, 0, P, lds);
            else
                atb_stream<8, 1, 2>(A, ars, acs, Mo, B, brs, bcs, No, kb, ke, i0, 0, P, lds);
        }
        return;
    }
    for (int i0 = 0; i0 < Mo; i0 += 32)
        for (int j0 = 0; j0 < No; j0 += 64) atb_stream<2, 4, 2>(A, ars, acs, Mo, B, brs, bcs, No, kb, ke, i0, j0, P, lds);
}

// Workgroup sum (256 threads) through LDS; every thread gets the sum.
__device__ __forceinline__ double block_sum_lds(double v, ldouble* red) {
    v = wave_sum(v);
    const int lane = lane_id(), w = wave_id();
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Sum of squares of rows [rb, re) of a column-major rows x cols block
// (fixed traversal, then a fixed-order workgroup sum); same value in every
// thread.
__device__ __forceinline__ double sumsq_rows(const double* S, int rows, int cols, int rb, int re, ldouble* red) {
    const int nr = re - rb;
    double s = 0.0;
    if (nr > 0)
        for (int64_t e = threadIdx.x; e < (int64_t)nr * cols; e += 256) {
            const int64_t c = e / nr, r = rb + (e - c * nr);
            const double v = gptr(S)[c * rows + r];
            s += v * v;
        }
    return block_sum_lds(s, red);
}

// dst[(e / cols) * ldd + e % cols] = sum over members of slots[m*ps + e], for
// e in [e0, e1), in member order.
template <class DST>
__device__ __forceinline__ void reduce_slots(const double* slots, int64_t ps, int T, int e0, int e1, int cols, DST* dst,
                                             int64_t ldd) {
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
        const gdouble* sl = gptr(slots);
        double v = sl[e];
        for (int m = 1; m < T; ++m) v += sl[(int64_t)m * ps + e];
        dst[(int64_t)(e / cols) * ldd + e % cols] = v;
    }
}

// ---------------------------------------------------------------------------
// Small dense factorizations in LDS (b <= 64)
// ---------------------------------------------------------------------------
// Upper Cholesky in place: R^T R = G + shift I (upper triangle of G, LDS
// stride kLD).  Returns true when every pivot (before its square root) is
// positive and finite and, with cert, keeps more than 1e-10 of the diagonal
// entry it started from -- the CholeskyQR breakdown certificate.
__device__ __forceinline__ bool chol_lds(ldouble* G, int b, double shift, bool cert, ldouble* misc) {
    const int tid = threadIdx.x;
    if (tid < b) misc[2 + tid] = G[tid * kLD + tid];
    if (tid == 0) misc[1] = 0.0;
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        if (tid == 0) {
            const double p = G[j * kLD + j] + shift;
            const bool ok = (p > 0.0) && isfinite(p) && (!cert || p > 1e-10 * misc[2 + j]);
            if (!ok) misc[1] = 1.0;
            const double dj = ok ? sqrt(p) : 1.0;
            G[j * kLD + j] = dj;
            misc[0] = 1.0 / dj;
        }
        __syncthreads();
        const double inv = misc[0];
        for (int c = j + 1 + tid; c < b; c += 256) G[j * kLD + c] *= inv;
        __syncthreads();
        const int nt = b - j - 1;
        for (int e = tid; e < nt * nt; e += 256) {
            const int r = j + 1 + e / nt, c = j + 1 + e % nt;
            if (c >= r) G[r * kLD + c] -= G[j * kLD + r] * G[j * kLD + c];
        }
        __syncthreads();
    }
    return misc[1] == 0.0;
}

// X = R^{-1} (upper triangular) by back substitution, one column per
// thread, in LDS after G (the chain of each column reads only LDS), then
// copied to dst (b x b row-major, zeros below the diagonal).
__device__ __forceinline__ void rinv_lds(ldouble* G, int b, double* dst) {
    const int tid = threadIdx.x;
    ldouble* X = G + kBatchMaxBlock * kLD;
    if (tid < b) {
        const int c = tid;
        X[c * kLD + c] = 1.0 / G[c * kLD + c];
        for (int i = c - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= c; ++k) s += G[i * kLD + k] * X[k * kLD + c];
            X[i * kLD + c] = -s / G[i * kLD + i];
        }
    }
    __syncthreads();
    for (int e = tid; e < b * b; e += 256) {
        const int i = e / b, c = e - i * b;
        gptr(dst)[e] = i > c ? 0.0 : X[i * kLD + c];
    }
    __syncthreads();
}
static_assert(2 * kBatchMaxBlock * kLD <= kMisc, "R^{-1} must fit between G and the misc area");

// Householder QR of a rows x b column-major panel by one workgroup,
// overwritten by the explicit Q with diag(R) >= 0; V (rows x b) holds the
// reflectors.  The fallback when CholeskyQR breaks down.
__device__ __noinline__ void householder_wg(double* A, int rows, int b, double* V, ldouble* lds) {
    ldouble* tau = lds;
    ldouble* bet = lds + kBatchMaxBlock;
    ldouble* red = lds + 2 * kBatchMaxBlock;
    const int tid = threadIdx.x, w = wave_id(), l = lane_id();
    for (int j = 0; j < b; ++j) {
        const int64_t cj = (int64_t)j * rows;
        double s = 0.0;
        for (int r = j + 1 + tid; r < rows; r += 256) s += A[cj + r] * A[cj + r];
        s = block_sum_lds(s, red);
        const double alpha = A[cj + j];
        double beta, tj, scale;
        if (s == 0.0 && alpha >= 0.0) {
            beta = alpha;
            tj = 0.0;
            scale = 0.0;
        } else {
            const double nx = sqrt(alpha * alpha + s);
            beta = -copysign(nx, alpha);
            tj = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int r = j + 1 + tid; r < rows; r += 256) V[cj + r] = A[cj + r] * scale;
        for (int r = tid; r < j; r += 256) V[cj + r] = 0.0;
        if (tid == 0) {
            V[cj + j] = 1.0;
            tau[j] = tj;
            bet[j] = beta;
        }
        __syncthreads();
        for (int c = j + 1 + w; c < b; c += 4) {
            const int64_t cc = (int64_t)c * rows;
            double p = 0.0;
            for (int r = j + l; r < rows; r += 64) p += V[cj + r] * A[cc + r];
            p = wave_sum(p);
            const double f = tj * p;
            for (int r = j + l; r < rows; r += 64) A[cc + r] -= f * V[cj + r];
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)rows * b; e += 256) {
        const int64_t c = e / rows, r = e - c * rows;
        A[e] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = b - 1; j >= 0; --j) {
        const int64_t cj = (int64_t)j * rows;
        const double tj = tau[j];
        for (int c = j + w; c < b; c += 4) {
            const int64_t cc = (int64_t)c * rows;
            double p = 0.0;
            for (int r = j + l; r < rows; r += 64) p += V[cj + r] * A[cc + r];
            p = wave_sum(p);
            const double f = tj * p;
            for (int r = j + l; r < rows; r += 64) A[cc + r] -= f * V[cj + r];
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)rows * b; e += 256) {
        const int c = (int)(e / rows);
        if (bet[c] < 0.0) A[e] = -A[e];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Team-level steps.  Each is out of line with a small signature, so that
// register allocation is local to the step; LDS is passed as an
// address-space-3 pointer.  `par` is the member's partial-slot parity
// (alternating per reduction); steps that reduce return the new parity.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double* slot_of(const BatchTT* t, int par, int m) {
    return t->slots + ((int64_t)par * t->T + m) * t->pslot;
}
__device__ __forceinline__ const double* slots_base(const BatchTT* t, int par) {
    return t->slots + (int64_t)par * t->T * t->pslot;
}
__device__ __forceinline__ bool team_failed(const BatchTT* t) {
    return __hip_atomic_load(t->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1;
}
// Adds one to entry e of the tensor's run record (first member only).
__device__ __forceinline__ void count_event(const BatchTT* t, int m, int e) {
    if (m == 0 && threadIdx.x == 0) t->info[e] += 1.0;
}

// Thin QR of the rows x b column-major panel S (b <= 64): CholeskyQR with the
// breakdown certificate until two certified passes in a row, a shifted pass
// (shift 11 (rows b + b(b+1)) u trace(G), Fukaya et al. 2020) after a
// certificate failure (at most two), and a Householder QR by the first
// member when a shifted factorization fails too or after six passes.  Each
// member applies R^{-1} to its own rows [rb, re); the Householder route
// ends with a team barrier, the others do not.  need_ok: plain (certified,
// unshifted) passes that end the loop -- two for a general block, one for a
// block that is already orthonormal to rounding error (after the
// reorthogonalisation its Gram matrix is I + O(u), and one pass leaves it
// orthonormal to O(u)).  have_gram: every member's
// partial Gram matrix of S is already in its slot of parity par (written
// with the block, see gemm_rows_gram); each R^{-1} application that a
// further pass will factor writes the next Gram the same way.  synced: a
// team barrier has already passed since those slots were written, so the
// first pass reads them without one.
__device__ __noinline__ int qr_team(const BatchTT* t, int m, int par, double* S, int rows, int b, int rb, int re,
                                    ldouble* lds, bool have_gram, int need_ok = 2, bool synced = false) {
    ldouble* G = lds;
    ldouble* misc = lds + kMisc;
    double* rinv = t->priv + (int64_t)m * t->privs;
    int plain_ok = 0, shifts = 0, passes = 0;
    for (;;) {
        if (!have_gram) atb(S, rows, 1, b, S, 1, rows, b, rb, re, slot_of(t, par, m), lds);
        if (!(have_gram && synced)) team_sync(*t);
        have_gram = false;
        synced = false;
        const double* base = slots_base(t, par);
        par ^= 1;
        reduce_slots(base, t->pslot, t->T, 0, b * b, b, G, kLD);
        __syncthreads();
        bool ok = chol_lds(G, b, 0.0, true, misc);
        if (ok) {
            ++plain_ok;
        } else if (shifts < 2) {
            reduce_slots(base, t->pslot, t->T, 0, b * b, b, G, kLD);
            __syncthreads();
            if (threadIdx.x == 0) {
                double tr = 0.0;
                for (int j = 0; j < b; ++j) tr += G[j * kLD + j];
                misc[kBatchMaxBlock + 8] = 11.0 * ((double)rows * b + (double)b * (b + 1)) * kUnit * tr;
            }
            __syncthreads();
            const double shift = misc[kBatchMaxBlock + 8];
            ok = chol_lds(G, b, shift, false, misc);
            if (ok) {
                ++shifts;
                count_event(t, m, 6);
                plain_ok = 0;
            }
        }
        if (!ok || ++passes > 6) {
            team_sync(*t);
            if (m == 0) householder_wg(S, rows, b, t->hh, lds);
            count_event(t, m, 5);
            team_sync(*t);
            return par;
        }
        rinv_lds(G, b, rinv);
        if (plain_ok >= need_ok) {
            gemm_rows(S, 1, rows, rinv, b, 1, S, 1, rows, rb, re, b, b, 1.0, 0.0, lds);
            __syncthreads();
            return par;
        }
        // another pass follows: its Gram is formed while S is written
        gemm_rows_gram(S, 1, rows, rinv, b, 1, S, 1, rows, rb, re, b, b, 1.0, 0.0, slot_of(t, par, m), lds);
        __syncthreads();
        have_gram = true;
    }
}

// S[own rows] -= Q[:, 0:ncq] (Q^T S), with Q^T S reduced over the team; S is
// the rows x nb block that follows Q's ncq columns.  The update also writes
// each member's partial Gram matrix of the new S into its slot of the
// returned parity (for qr_team with have_gram).  With want_sumsq the
// team-reduced ||S||_F^2, the trace of that Gram matrix, is returned in *ss
// after a team barrier; a caller that does not go on to qr_team must then
// flip the parity before the slots are written again.
__device__ __noinline__ int project_out(const BatchTT* t, int m, int par, double* Q, int rows, int ncq, int nb,
                                        int rb, int re, int want_sumsq, double* ss, ldouble* lds) {
    double* S = Q + (int64_t)ncq * rows;
    double* tm = t->priv + (int64_t)m * t->privs + kBatchPrivRinv;
    atb(Q, rows, 1, ncq, S, 1, rows, nb, rb, re, slot_of(t, par, m), lds);
    team_sync(*t);
    reduce_slots(slots_base(t, par), t->pslot, t->T, 0, ncq * nb, nb, tm, nb);
    par ^= 1;
    __syncthreads();
    gemm_rows_gram(Q, 1, rows, tm, nb, 1, S, 1, rows, rb, re, nb, ncq, -1.0, 1.0, slot_of(t, par, m), lds);
    __syncthreads();
    if (!want_sumsq) return par;
    team_sync(*t);
    double tot = 0.0;
    const gdouble* base = gptr(slots_base(t, par));
    for (int mm = 0; mm < t->T; ++mm) {
        double tr = 0.0;
        for (int i = 0; i < nb; ++i) tr += base[(int64_t)mm * t->pslot + (int64_t)i * nb + i];
        tot += tr;
    }
    *ss = tot;
    return par;
}

// Omega_j(:, c0:c0+nc) for modes j = j0..d, split over the team's threads.
__device__ __noinline__ void gen_omega(const BatchTT* t, int m, int j0, int c0, int nc) {
    const int64_t gt = (int64_t)m * 256 + threadIdx.x, stride = (int64_t)t->T * 256;
    for (int j = j0; j <= t->d; ++j) {
        const int64_t n = t->n[j - 1], np = (n + 1) / 2;
        gdouble* om = gptr(t->om + t->ooff[j]);
        for (int64_t e = gt; e < np * nc; e += stride) {
            const int64_t p = e / nc, c = e - p * nc;
            double g0, g1;
            omega_pair(t->seed, p, (uint64_t)(c0 + c), j, g0, g1);
            om[(2 * p) * t->lcap + c0 + c] = g0;
            if (2 * p + 1 < n) om[(2 * p + 1) * t->lcap + c0 + c] = g1;
        }
    }
}

// W_k(a, c0:c0+nc) = sum_i Omega_k(i, c) sum_b X_k(a, i, b) W_{k+1}(b, c) for
// one row a, by the workgroup: the core row times W_{k+1} as MFMA tiles,
// each folded with Omega_k in registers (fixed order over i), then the
// lane groups by two butterflies and the waves in wave order through LDS.
// Rows a = a0, a0 + astep, ... of W_k for one wave (Sec. 3.1, Eq. 8):
// W_k(a, c) = sum_i Omega_k(i, c) sum_b X_k(a, i, b) W_{k+1}(b, c).  For
// each row, 16-row blocks i0 of X_k(a) (n x r1, rows contiguous in b) are
// multiplied by W_{k+1} (r1 x nc, row stride lcap) over K = r1 in steps of
// 4 KS, and each finished block is folded with Omega_k(i0.., c) into the
// lane's partial sums; a row's sums are reduced over the lane groups and
// stored.  The wave's (row, block, step) sequence runs through two
// register stages, and a block's last step also loads its Omega entries,
// so no MFMA or fold waits for a load issued just before it.  K steps are
// paired as in atb_stream (16-byte loads of a core row).
template <int NB, int KS, bool LB>
__device__ __forceinline__ void pc_stream(const double* X, int r0, int n, int r1, const double* Wn, int lcap,
                                          const double* Om, int nc, double* W, int a0, int astep,
                                          const ldouble* wl) {
    static_assert(KS % 2 == 0, "K steps come in pairs");
    const int l = lane_id(), li = l & 15, lg = l >> 4;
    const int nrow = a0 < r0 ? (r0 - a0 + astep - 1) / astep : 0;
    const int nbk = (n + 15) / 16, kit = (r1 + 4 * KS - 1) / (4 * KS), per_row = nbk * kit;
    const int steps = nrow * per_row;
    if (steps == 0) return;
    const gdouble* pb[NB];
    bool vb[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int c = 16 * j + li;
        vb[j] = c < nc;
        pb[j] = gptr(Wn) + min(c, nc - 1);
    }
    typedef double StageA[KS];
    typedef double StageB[KS][NB];
    typedef double StageO[NB][4];
    auto load = [&](int st, StageA& a, StageB& b, StageO& o) {
        const int u = st / per_row, rem = st - u * per_row, bk = rem / kit, ki = rem - bk * kit;
        const int row = a0 + astep * u, i = 16 * bk + li, k = 4 * KS * ki;
        const bool vi = i < n, whole = k + 4 * KS <= r1;  // whole: uniform
        const gdouble* pa = gptr(X) + ((int64_t)row * n + min(i, n - 1)) * r1;
#pragma unroll
        for (int q = 0; q < KS / 2; ++q) {
            const int kk = k + 8 * q + 2 * lg;
            const bool ok0 = kk < r1, ok1 = kk + 1 < r1;
            const int kc0 = min(kk, r1 - 1), kc1 = min(kk + 1, r1 - 1);
            double v0, v1;
            if (whole) {
                const d2u v = *(const gd2u*)(pa + kk);
                v0 = v[0];
                v1 = v[1];
            } else {
                v0 = pa[kc0];
                v1 = pa[kc1];
            }
            a[2 * q] = (ok0 && vi) ? v0 : 0.0;
            a[2 * q + 1] = (ok1 && vi) ? v1 : 0.0;
            if (!LB) {
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double w0 = pb[j][(int64_t)kc0 * lcap], w1 = pb[j][(int64_t)kc1 * lcap];
                    b[2 * q][j] = (ok0 && vb[j]) ? w0 : 0.0;
                    b[2 * q + 1][j] = (ok1 && vb[j]) ? w1 : 0.0;
                }
            }
        }
        if (ki == kit - 1) {  // uniform: the block's Omega entries for its fold
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ii = 16 * bk + lg + 4 * v, c = 16 * j + li;
                    const double om = gptr(Om)[(int64_t)min(ii, n - 1) * lcap + min(c, nc - 1)];
                    o[j][v] = (ii < n && c < nc) ? om : 0.0;
                }
        }
    };
    double4_t acc[NB];
    double part[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
        part[j] = 0.0;
    }
    // with W_{k+1}'s block in LDS (LB) its entries are read just before
    // their MFMAs, so a register stage holds only the core's rows
    auto mma = [&](int st, const StageA& a, const StageB& b) {
        if (LB) {
            const int k = ((st % per_row) % kit) * 4 * KS;
#pragma unroll
            for (int q = 0; q < KS / 2; ++q) {
                const int kk = k + 8 * q + 2 * lg;
                const bool ok0 = kk < r1, ok1 = kk + 1 < r1;
                const int kc0 = min(kk, r1 - 1), kc1 = min(kk + 1, r1 - 1);
                double u0[NB], u1[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const double w0 = wl[kc0 * kWLD + 16 * j + li], w1 = wl[kc1 * kWLD + 16 * j + li];
                    u0[j] = (ok0 && vb[j]) ? w0 : 0.0;
                    u1[j] = (ok1 && vb[j]) ? w1 : 0.0;
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = mfma_f64_16x16x4(a[2 * q], u0[j], acc[j]);
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = mfma_f64_16x16x4(a[2 * q + 1], u1[j], acc[j]);
            }
        } else {
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = mfma_f64_16x16x4(a[s2], b[s2][j], acc[j]);
        }
    };
    // after step st: fold a finished block, store a finished row
    auto after = [&](int st, const StageO& o) {
        const int rem = st % per_row;
        if ((rem + 1) % kit != 0) return;  // uniform
#pragma unroll
        for (int j = 0; j < NB; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) part[j] += o[j][v] * acc[j][v];
            acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
        }
        if (rem + 1 != per_row) return;  // uniform
        const int row = a0 + astep * (st / per_row);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double sj = part[j];
            sj += __shfl_xor(sj, 16, 64);
            sj += __shfl_xor(sj, 32, 64);
            if (lg == 0 && vb[j]) gptr(W)[(int64_t)row * lcap + 16 * j + li] = sj;
            part[j] = 0.0;
        }
    };
    StageA sa0, sa1;
    StageB sb0, sb1;
    StageO so0, so1;
    load(0, sa0, sb0, so0);
    for (int st = 0; st < steps; st += 2) {  // uniform per wave
        const bool more1 = st + 1 < steps, more2 = st + 2 < steps;
        if (more1) load(st + 1, sa1, sb1, so1);
        mma(st, sa0, sb0);
        after(st, so0);
        if (more2) load(st + 2, sa0, sb0, so0);
        if (more1) {
            mma(st + 1, sa1, sb1);
            after(st + 1, so1);
        }
    }
}

// Core k of a right-to-left pass over columns [c0, c0+nc) (Sec. 3.1):
// W_d = H(X_d) Omega_d at k = d, else W_k from W_{k+1}; rows (or tiles)
// split over the team's workgroups.
__device__ __noinline__ void pc_core(const BatchTT* t, int m, int k, int c0, int nc, ldouble* lds) {
    const int d = t->d, lcap = t->lcap;
    const int r0 = (int)t->r[k - 1], n = (int)t->n[k - 1], r1 = (int)t->r[k];
    const double* X = t->X[k - 1];
    const double* Om = t->om + t->ooff[k] + c0;
    double* W = t->w + t->woff[k] + c0;
    if (k == d) {
        wg_gemm(X, n, 1, Om, lcap, 1, W, lcap, 1, 0, r0, nc, n, 1.0, 0.0, m, t->T, lds);
        return;
    }
    const double* Wn = t->w + t->woff[k + 1] + c0;
    // rows a = m + T (w + 4 u) for wave w of member m, 64 columns at a time;
    // with r1 <= kWRows the block of W_{k+1} is staged in LDS first (every
    // row of the core multiplies all of it)
    const int a0 = m + t->T * wave_id(), astep = 4 * t->T;
    const bool staged = r1 <= kWRows;
    for (int n0 = 0; n0 < nc; n0 += 64) {
        const int nb = min(64, nc - n0);
        if (staged) {
            const gdouble* wg = gptr(Wn) + n0;
            for (int e = threadIdx.x; e < r1 * 64; e += 256) {
                const int kq = e >> 6, c = e & 63;
                lds[kq * kWLD + c] = c < nb ? wg[(int64_t)kq * lcap + c] : 0.0;
            }
            __syncthreads();
        }
        if (staged) {
            if (nb <= 16)
                pc_stream<1, 8, true>(X, r0, n, r1, Wn + n0, lcap, Om + n0, nb, W + n0, a0, astep, lds);
            else if (nb <= 32)
                pc_stream<2, 8, true>(X, r0, n, r1, Wn + n0, lcap, Om + n0, nb, W + n0, a0, astep, lds);
            else
                pc_stream<4, 8, true>(X, r0, n, r1, Wn + n0, lcap, Om + n0, nb, W + n0, a0, astep, lds);
        } else {
            if (nb <= 16)
                pc_stream<1, 8, false>(X, r0, n, r1, Wn + n0, lcap, Om + n0, nb, W + n0, a0, astep, nullptr);
            else if (nb <= 32)
                pc_stream<2, 8, false>(X, r0, n, r1, Wn + n0, lcap, Om + n0, nb, W + n0, a0, astep, nullptr);
            else
                pc_stream<4, 4, false>(X, r0, n, r1, Wn + n0, lcap, Om + n0, nb, W + n0, a0, astep, nullptr);
        }
        __syncthreads();  // the staged block is replaced by the next one
    }
}

// One right-to-left pass: Omega and W for columns [c0, c0+nc) of modes k1..d.
__device__ __forceinline__ void pc_pass(const BatchTT* t, int m, int k1, int c0, int nc, int& passes,
                                        ldouble* lds) {
    gen_omega(t, m, k1, c0, nc);
    team_sync(*t);
    for (int k = t->d; k >= k1; --k) {
        pc_core(t, m, k, c0, nc, lds);
        team_sync(*t);
    }
    if (m == 0 && threadIdx.x == 0 && passes < kBatchMaxPasses) {
        t->info[8 + 2 * passes] = (double)k1;
        t->info[9 + 2 * passes] = (double)nc;
    }
    ++passes;
}

// Remark 1: ||X|| ~ ||V(X_1) W_2(:, 0:r0)||_F / sqrt(r0), squared norm
// reduced over the team (the product goes through the Q buffer).
__device__ __noinline__ int norm_estimate(const BatchTT* t, int m, int par, double* nrmx, ldouble* lds) {
    const int rows = (int)t->n[0], r1 = (int)t->r[1];
    int rb, re;
    member_rows(rows, t->T, m, rb, re);
    gemm_rows(t->X[0], r1, 1, t->w + t->woff[2], t->lcap, 1, t->q, 1, rows, rb, re, t->r0, r1, 1.0, 0.0, lds);
    __syncthreads();
    const double s = sumsq_rows(t->q, rows, t->r0, rb, re, lds + kMisc + kBatchMaxBlock + 12);
    if (threadIdx.x == 0) slot_of(t, par, m)[0] = s;
    team_sync(*t);
    double tot = 0.0;
    const double* base = slots_base(t, par);
    for (int mm = 0; mm < t->T; ++mm) tot += base[(int64_t)mm * t->pslot];
    *nrmx = sqrt(tot / (double)t->r0);
    return par ^ 1;
}

// Projection M = Q^T V(Y_k) (lk x R) reduced over the team by entry
// ranges, this member's rows of the output core V(Y_k) <- Q, and the next
// core H(Y_{k+1}) = M H(X_{k+1}) (lk x n_{k+1} r_{k+1}) by output tiles.
// C[0:Mg, cb:ce] = A B for A (Mg <= 64 rows, K <= kWRows) staged in LDS as
// Al[k kWLD + m] (rows past Mg zero) and B (K x ncols, row stride ldb)
// streamed from global memory: wave w takes the 16-column blocks cb +
// 16 (w + 4 u) < ce, each over K in steps of 4 KS, the (block, step)
// sequence through two register stages of B values.  The MFMA order per
// output tile is that of a K loop in steps of 4, as in wg_tile.
template <int MB, int KS>
__device__ __forceinline__ void cols_stream(const ldouble* Al, int Mg, int K, const double* B, int64_t ldb, double* C,
                                            int64_t ldc, int cb, int ce) {
    const int l = lane_id(), li = l & 15, lg = l >> 4;
    const int cfirst = cb + 16 * wave_id();
    const int kit = (K + 4 * KS - 1) / (4 * KS);
    const int nblk = cfirst < ce ? (ce - cfirst + 63) / 64 : 0;
    const int steps = nblk * kit;
    if (steps == 0) return;
    typedef double StageB[KS];
    auto load = [&](int st, StageB& b) {
        const int blk = st / kit, k = (st - blk * kit) * 4 * KS;
        const int c = cfirst + 64 * blk + li;
        const bool vc = c < ce;
        const gdouble* pb = gptr(B) + min(c, ce - 1);
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
            const int kk = k + 4 * s2 + lg;
            const double v = pb[(int64_t)min(kk, K - 1) * ldb];
            b[s2] = (kk < K && vc) ? v : 0.0;
        }
    };
    double4_t acc[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) acc[i] = double4_t{0.0, 0.0, 0.0, 0.0};
    auto mma = [&](int st, const StageB& b) {
        const int k = (st % kit) * 4 * KS;
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
            const int kc = min(k + 4 * s2 + lg, K - 1);
#pragma unroll
            for (int i = 0; i < MB; ++i) acc[i] = mfma_f64_16x16x4(Al[kc * kWLD + 16 * i + li], b[s2], acc[i]);
        }
    };
    auto finish = [&](int blk) {
        const int c = cfirst + 64 * blk + li;
#pragma unroll
        for (int i = 0; i < MB; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * i + lg + 4 * v;
                if (r < Mg && c < ce) gptr(C)[(int64_t)r * ldc + c] = acc[i][v];
            }
            acc[i] = double4_t{0.0, 0.0, 0.0, 0.0};
        }
    };
    StageB b0, b1;
    load(0, b0);
    for (int st = 0; st < steps; st += 2) {  // uniform per wave
        const bool more1 = st + 1 < steps, more2 = st + 2 < steps;
        if (more1) load(st + 1, b1);
        mma(st, b0);
        if ((st + 1) % kit == 0) finish(st / kit);
        if (more2) load(st + 2, b0);
        if (more1) {
            mma(st + 1, b1);
            if ((st + 2) % kit == 0) finish((st + 1) / kit);
        }
    }
}

// dst (lk x ncols, row-major) = M (lk x R, row-major) X (R x ncols, row
// stride ncols) for this member's share of the columns: 64 rows of M at a
// time staged in LDS (R <= kWRows), X streamed (cols_stream); larger R
// goes through the LDS-staged tiles of wg_gemm.
__device__ __noinline__ void next_core(const double* M, int lk, int R, const double* X, int ncols, double* dst, int m,
                                       int T, ldouble* lds) {
    if (R > kWRows) {
        wg_gemm(M, R, 1, X, ncols, 1, dst, ncols, 1, 0, lk, ncols, R, 1.0, 0.0, m, T, lds);
        return;
    }
    int cb, ce;
    member_rows(ncols, T, m, cb, ce);
    const gdouble* Mg = gptr(M);
    for (int m0 = 0; m0 < lk; m0 += 64) {
        const int rows = min(64, lk - m0);
        for (int e = threadIdx.x; e < R * 64; e += 256) {
            const int kq = e >> 6, r = e & 63;
            lds[kq * kWLD + r] = r < rows ? Mg[(int64_t)(m0 + r) * R + kq] : 0.0;
        }
        __syncthreads();
        double* C = dst + (int64_t)m0 * ncols;
        if (rows <= 16)
            cols_stream<1, 8>(lds, rows, R, X, ncols, C, ncols, cb, ce);
        else if (rows <= 32)
            cols_stream<2, 8>(lds, rows, R, X, ncols, C, ncols, cb, ce);
        else
            cols_stream<4, 8>(lds, rows, R, X, ncols, C, ncols, cb, ce);
        __syncthreads();  // the staged rows are replaced by the next ones
    }
}

__device__ __noinline__ int project_and_next(const BatchTT* t, int m, int par, int k, const double* ycur, int rows,
                                             int R, int lk, int rb, int re, double* dst, ldouble* lds) {
    const int T = t->T;
    double* Q = t->q;
    atb(Q, rows, 1, lk, ycur, R, 1, R, rb, re, slot_of(t, par, m), lds);
    // this member's rows of Q (column-major) into the output core
    // (row-major), through LDS in 64 x 64 tiles so that both the reads and
    // the writes are contiguous; the next tile's reads are in flight while
    // the current one is written
    gdouble* Yk = gptr(t->Y[k - 1]);
    const gdouble* Qg = gptr(Q);
    {
        const int nct = (lk + 63) / 64, ntile = ((re - rb + 63) / 64) * nct;
        double buf[16];
        auto read_tile = [&](int tile) {  // thread -> row tid % 64, column tid / 64 + 4 u
            const int r0 = rb + (tile / nct) * 64, c0 = (tile % nct) * 64;
            const int r = min(r0 + (int)(threadIdx.x & 63), re - 1);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int c = min(c0 + (int)(threadIdx.x >> 6) + 4 * u, lk - 1);
                buf[u] = Qg[(int64_t)c * rows + r];
            }
        };
        if (ntile > 0 && rb < re) read_tile(0);
        for (int tile = 0; tile < ntile && rb < re; ++tile) {
#pragma unroll
            for (int u = 0; u < 16; ++u) lds[((threadIdx.x >> 6) + 4 * u) * 65 + (threadIdx.x & 63)] = buf[u];
            __syncthreads();
            if (tile + 1 < ntile) read_tile(tile + 1);
            const int r0 = rb + (tile / nct) * 64, c0 = (tile % nct) * 64;
            const int nr = min(64, re - r0), ncc = min(64, lk - c0);
#pragma unroll
            for (int u = 0; u < 16; ++u) {  // write: thread -> column tid % 64, row tid / 64 + 4 u
                const int c = threadIdx.x & 63, r = (threadIdx.x >> 6) + 4 * u;
                if (r < nr && c < ncc) Yk[(int64_t)(r0 + r) * lk + c0 + c] = lds[c * 65 + r];
            }
            __syncthreads();
        }
    }
    team_sync(*t);
    const int E = lk * R;
    reduce_slots(slots_base(t, par), t->pslot, T, (int)((int64_t)E * m / T), (int)((int64_t)E * (m + 1) / T), R,
                 t->m, R);
    par ^= 1;
    team_sync(*t);
    const int nr1 = (int)(t->n[k] * t->r[k + 1]);
    next_core(t->m, lk, R, t->X[k], nr1, dst, m, T, lds);
    team_sync(*t);
    return par;
}

// The adaptive rounding of one tensor as member m of its team.
__device__ __forceinline__ void round_tensor(const BatchTT* t, int m, ldouble* lds) {
    const int d = t->d, lcap = t->lcap, T = t->T;
    if (m == 0 && threadIdx.x == 0) {
        t->info[kBatchInfoClock] = (double)wall_clock64();
        t->info[5] = 0.0;
        t->info[6] = 0.0;
    }
    uint64_t phase[kBatchPhases] = {0, 0, 0, 0, 0};
    uint64_t clk = wall_clock64();
    auto tock = [&](int p) {
        const uint64_t now = wall_clock64();
        phase[p] += now - clk;
        clk = now;
    };
    int par = 0, passes = 0, iterations = 0;
    double min_margin = INFINITY;

    int ncols = t->init_cols;
    pc_pass(t, m, 2, 0, ncols, passes, lds);
    tock(0);

    double nrmx = t->nrmx;
    if (!t->has_nrmx) par = norm_estimate(t, m, par, &nrmx, lds);
    const double tau = t->tol * nrmx / sqrt((double)(d - 1));

    const double* ycur = t->X[0];
    int lprev = 1;
    double* Q = t->q;
    for (int k = 1; k < d; ++k) {
        if (team_failed(t)) break;
        const int rows = (int)(lprev * t->n[k - 1]);
        const int R = (int)t->r[k];
        const int rbar = min(rows, R);
        const int binit = max(1, min(rbar, (int)ceil(t->f_init * (double)rbar)));
        int rb, re;
        member_rows(rows, T, m, rb, re);
        const double* Wk1 = t->w + t->woff[k + 1];
        tock(4);
        // sketch of the first binit columns (with its Gram matrix) and its QR
        gemm_rows_gram(ycur, R, 1, Wk1, lcap, 1, Q, 1, rows, rb, re, binit, R, 1.0, 0.0, slot_of(t, par, m), lds);
        __syncthreads();
        tock(1);
        par = qr_team(t, m, par, Q, rows, binit, rb, re, lds, true);
        __syncthreads();
        tock(2);
        int ncq = binit;
        int sketched = binit;  // columns of Q's buffer that already hold V(Y_k) W_{k+1}
        const int blk = t->ell_block > 0 ? t->ell_block : max(1, (int)ceil(0.05 * (double)rbar));
        while (ncq < rbar) {
            const int bb = min(blk, rbar - ncq);
            const int need = ncq + bb;
            if (ncols < need) {
                const int grow = min(lcap - ncols, max(need - ncols, ncols));
                pc_pass(t, m, k + 1, ncols, grow, passes, lds);
                ncols += grow;
                tock(0);
            }
            double* S = Q + (int64_t)ncq * rows;
            if (sketched < need) {
                // sketch up to 64 columns ahead in one pass over V(Y_k): a
                // column's sketch does not depend on the basis, so the later
                // blocks find theirs in place (unused ones are dropped)
                const int nsk = max(bb, min(min(kBatchMaxBlock, rbar - ncq), ncols - ncq));
                gemm_rows(ycur, R, 1, Wk1 + ncq, lcap, 1, S, 1, rows, rb, re, nsk, R, 1.0, 0.0, lds);
                __syncthreads();
                sketched = ncq + nsk;
            }
            tock(1);
            double ss = 0.0;
            par = project_out(t, m, par, Q, rows, ncq, bb, rb, re, 1, &ss, lds);
            tock(3);
            const double est = sqrt(ss / (double)bb);
            ++iterations;
            if (tau > 0.0) min_margin = fmin(min_margin, fabs(est - tau) / tau);
            if (!(est > tau)) {
                par ^= 1;  // the block's Gram slots are not consumed
                break;
            }
            // the estimate's barrier in project_out already published the Gram slots
            par = qr_team(t, m, par, S, rows, bb, rb, re, lds, true, 2, true);
            __syncthreads();
            tock(2);
            par = project_out(t, m, par, Q, rows, ncq, bb, rb, re, 0, &ss, lds);
            tock(3);
            par = qr_team(t, m, par, S, rows, bb, rb, re, lds, true, 1);
            __syncthreads();
            tock(2);
            ncq += bb;
        }
        const int lk = ncq;
        double* dst = (k + 1 == d) ? t->Y[d - 1] : t->yb[k & 1];
        par = project_and_next(t, m, par, k, ycur, rows, R, lk, rb, re, dst, lds);
        tock(4);
        if (m == 0 && threadIdx.x == 0) t->ranks[k] = lk;
        ycur = dst;
        lprev = lk;
    }
    if (m == 0 && threadIdx.x == 0) {
        t->ranks[0] = 1;
        t->ranks[d] = 1;
        t->info[0] = tau;
        t->info[1] = nrmx;
        t->info[2] = iterations;
        t->info[3] = passes;
        t->info[4] = ncols;
        t->info[7] = min_margin;
        t->info[kBatchInfoClock + 1] = (double)wall_clock64();
        for (int p = 0; p < kBatchPhases; ++p) t->info[kBatchInfoClock + 2 + p] = (double)phase[p];
    }
}

// The ticket loop of one workgroup (lds: kLdsDoubles of LDS, s_ticket one
// int of LDS).
__device__ __forceinline__ void batch_body(const BatchTT* __restrict__ tts, const int* __restrict__ order,
                                           const int* __restrict__ prefix, int count, unsigned* ticket, ldouble* lds,
                                           int* s_ticket) {
    const int total = prefix[count];
    for (;;) {
        if (threadIdx.x == 0) *s_ticket = (int)atomicAdd(ticket, 1u);
        __syncthreads();
        const int s = *s_ticket;
        __syncthreads();
        if (s >= total) break;
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= s) lo = mid;
            else hi = mid - 1;
        }
        round_tensor(&tts[order[lo]], s - prefix[lo], lds);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) batch_kernel(const BatchTT* __restrict__ tts, const int* __restrict__ order,
                                                    const int* __restrict__ prefix, int count,
                                                    unsigned* ticket) {
    __shared__ double lds[kLdsDoubles];
    __shared__ int s_ticket;
    batch_body(tts, order, prefix, count, ticket, (ldouble*)lds, &s_ticket);
}

__global__ void zero_words_kernel(unsigned* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

void launch_batch(const BatchTT* tts, const int* order, const int* prefix, int count, unsigned* ticket,
                  unsigned* zero, int64_t zwords, int grid, hipStream_t s) {
    if (count <= 0) return;
    if (zwords > 0) {
        hipLaunchKernelGGL(zero_words_kernel, dim3(ceil_div(zwords, 256)), dim3(256), 0, s, zero, zwords);
        TTR_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(256), 0, s, tts, order, prefix, count, ticket);
    TTR_CHECK_LAUNCH();
}

int batch_resident_workgroups() {
    int dev = 0, cus = 0, per = 0;
    TTR_HIP(hipGetDevice(&dev));
    TTR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    TTR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel, 256, 0));
    return std::max(1, cus * std::max(per, 1));
}

}  // namespace ttr
