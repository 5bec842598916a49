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
// the tolerance-based truncation needs.  A truncation to a fixed rank only
// needs the best rank-t subspaces, so in that mode sweeping stops as soon
// as split_certified proves the kept/dropped split (the kept columns are
// then not diagonalised among themselves).
// t_out: [0] kept rank, [1] sweeps, [2] Cholesky tests run by the split
// certificate, [3] pivots those that failed got through.
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

// Tile e of the ten 16x16 tiles on and above the diagonal of a 64x64
// matrix: e < 4 the diagonal, then (0,1) (0,2) (0,3) (1,2) (1,3) (2,3).
__device__ __forceinline__ int tile_i(int e) { return e < 4 ? e : (e < 7 ? 0 : (e < 9 ? 1 : 2)); }
__device__ __forceinline__ int tile_j(int e) { return e < 4 ? e : (e < 7 ? e - 3 : (e < 9 ? e - 5 : 3)); }

// Maximum over the 16 lanes of a DPP row (the butterflies of group16_sum).
__device__ __forceinline__ double group16_max(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return v;
}

constexpr int GLD = 65;  // row stride of the Gram matrix in LDS
// Column stride (doubles) of A and V in LDS: 64 rows plus 2 of padding, so
// that 16 lanes reading row k of 16 consecutive columns (the MFMA operand
// pattern of the Gram matrix) hit 16 different bank pairs.
constexpr int CLD = 66;

// Rank-t split certificate for a truncation that only needs the kept
// subspace.  With B = A V the current columns (stride CLD in As), K the t
// columns of largest norm and D the rest, the truncation B_K V_K^T is the
// best rank-t approximation of A up to sin(theta) ||A|| once
//   sin(theta) <= ||B_K^T B_D||_F / (lambda_min(B_K^T B_K) - lambda_max(B_D^T B_D)) <= 1e-13
// (Davis-Kahan for the block split of A^T A).  Bounds used: lambda_max of
// the D block <= its largest diagonal entry + the Frobenius norm of its
// off-diagonal part (Weyl); lambda_min of the K block > mu, mu = that
// bound + ||G_KD||_F / 1e-13 + a rounding margin, when its smallest diagonal
// entry minus the Frobenius norm of its off-diagonal part exceeds mu
// (Weyl), else when the Cholesky of G_KK - mu I keeps every pivot
// positive.  Columns are ranked by the same squared norms (16-lane sums)
// and rule as the final sort, so K is
// exactly the set the caller keeps.  The Gram matrix comes from MFMA in
// rank order (eight waves, the ten 16x16 tiles on and above the diagonal),
// so K is its leading t x t block.  Returns true when certified; uniform
// over the block, every thread of the 512-thread block must call it.
__device__ bool split_certified(const double* As, int q, int t, double* Gs, double* nd, int* ord,
                                double (*red)[7], int* stats, bool& skip_next) {
    constexpr int LD = CLD;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, li = l & 15, lg = l >> 4;
    const int g16 = tid >> 4, l16 = tid & 15;
    for (int c = g16; c < q; c += 32) {
        double s = 0.0;
        for (int i = l16; i < 64; i += 16) s += As[c * LD + i] * As[c * LD + i];
        s = group16_sum(s);
        if (l16 == 0) nd[c] = s;
    }
    __syncthreads();
    // ord[rank] = column, by decreasing squared norm, ties by index: thread
    // (column tid/8, part tid%8) counts the larger norms among columns
    // part + 8u, summed over the 8 lanes of the column; slots >= q keep their
    // own (zero) columns
    {
        const int c = tid >> 3, part = tid & 7;
        const double me = c < q ? nd[c] : 0.0;
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = part + 8 * u;
            if (i < q) {
                const double o = nd[i];
                cnt += (o > me) || (o == me && i < c);
            }
        }
        cnt += __builtin_amdgcn_mov_dpp(cnt, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
        cnt += __builtin_amdgcn_mov_dpp(cnt, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
        cnt += __builtin_amdgcn_mov_dpp(cnt, 0x141, 0xF, 0xF, true);  // row_half_mirror
        if (part == 0) ord[c] = c;  // a valid column in every slot even if a NaN norm broke the ranking
        __syncthreads();
        if (part == 0 && c < q) ord[cnt] = c;
    }
    __syncthreads();
    for (int s = 0; s < 2; ++s) {
        const int e = w + 8 * s;
        if (e < 10) {  // uniform per wave
            const int I = tile_i(e), J = tile_j(e);
            const double* ca = As + ord[I * 16 + li] * LD + lg;
            const double* cb = As + ord[J * 16 + li] * LD + lg;
            // all operands are loaded first; two accumulators (even and odd
            // k-steps) halve the dependent MFMA chain
            double av[16], bv[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                av[k] = ca[4 * k];
                bv[k] = cb[4 * k];
            }
            double4_t acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 16; k += 2) {
                acc = mfma_f64_16x16x4(av[k], bv[k], acc);
                acc2 = mfma_f64_16x16x4(av[k + 1], bv[k + 1], acc2);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += acc2[v];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = I * 16 + lg + 4 * v, c = J * 16 + li;
                Gs[r * GLD + c] = acc[v];
                if (I != J) Gs[c * GLD + r] = acc[v];
            }
        }
    }
    __syncthreads();
    // ||G_KD||^2, ||offdiag G_DD||^2, ||offdiag G_KK||^2, max diag D, min
    // and max diag K, finiteness; thread: row tid/8, columns tid%8 + 8u
    double cross = 0.0, offd = 0.0, offk = 0.0, maxd = 0.0, mink = INFINITY, maxk = 0.0, fin = 1.0;
    const int r = tid >> 3;
    for (int c = tid & 7; c < q && r < q; c += 8) {
        const double g = Gs[r * GLD + c];
        if (!(fabs(g) < INFINITY)) fin = 0.0;
        if (r < t && c >= t) cross += g * g;
        if (r >= t && c >= t && r != c) offd += g * g;
        if (r < t && c < t && r != c) offk += g * g;
        if (r == c) {
            if (r < t) {
                mink = fmin(mink, g);
                maxk = fmax(maxk, g);
            } else {
                maxd = fmax(maxd, g);
            }
        }
    }
    // within each 16-lane row by DPP, then across the four rows
    cross = group16_sum(cross);
    offd = group16_sum(offd);
    offk = group16_sum(offk);
    maxd = group16_max(maxd);
    maxk = group16_max(maxk);
    mink = -group16_max(-mink);
    fin = -group16_max(-fin);
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
        cross += __shfl_xor(cross, off, 64);
        offd += __shfl_xor(offd, off, 64);
        offk += __shfl_xor(offk, off, 64);
        maxd = fmax(maxd, __shfl_xor(maxd, off, 64));
        maxk = fmax(maxk, __shfl_xor(maxk, off, 64));
        mink = fmin(mink, __shfl_xor(mink, off, 64));
        fin = fmin(fin, __shfl_xor(fin, off, 64));
    }
    if (l == 0) {
        red[w][0] = cross;
        red[w][1] = offd;
        red[w][2] = maxd;
        red[w][3] = mink;
        red[w][4] = maxk;
        red[w][5] = fin;
        red[w][6] = offk;
    }
    __syncthreads();
    cross = red[0][0], offd = red[0][1], maxd = red[0][2], mink = red[0][3], maxk = red[0][4], fin = red[0][5];
    offk = red[0][6];
    for (int v = 1; v < 8; ++v) {
        cross += red[v][0];
        offd += red[v][1];
        maxd = fmax(maxd, red[v][2]);
        mink = fmin(mink, red[v][3]);
        maxk = fmax(maxk, red[v][4]);
        fin = fmin(fin, red[v][5]);
        offk += red[v][6];
    }
    const double mu = maxd + sqrt(offd) + sqrt(cross) * 1e13 + 64.0 * t * 2.3e-16 * maxk;
    // Coupling x = ||G_KD||_F / gap above 1e-4: even at Jacobi's quadratic
    // rate the next sweep leaves it above the 1e-13 this test needs, so the
    // caller skips the next test.
    skip_next = !(mink - maxd - sqrt(offd) > 1e4 * sqrt(cross));
    if (!(fin > 0.0) || !(mink > mu) || !(mu < INFINITY)) return false;  // block-uniform
    // lambda_min(G_KK) >= min diag - ||offdiag G_KK||_F (Weyl) often suffices
    if (mink - sqrt(offk) > mu) return true;
    if (tid == 0) ++stats[0];
    // Cholesky (LDL^T) of the leading t x t block minus mu I, in place on its
    // lower triangle: step a subtracts G_ia G_ja / G_aa from a < j <= i
    // (thread: row a+1 + tid/8, columns a+1 + tid%8 + 8u); no entry a step
    // writes is read in that step.
    if (tid < t) Gs[tid * GLD + tid] -= mu;
    __syncthreads();
    for (int a = 0; a < t; ++a) {
        const double piv = Gs[a * GLD + a];
        if (!(piv > 0.0)) {  // every thread reads the same pivot
            if (tid == 0) stats[1] += a;
            return false;
        }
        const double ip = 1.0 / piv;
        const int i = a + 1 + (tid >> 3);
        if (i < t) {
            const double gi = Gs[i * GLD + a] * ip;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = a + 1 + (tid & 7) + 8 * u;
                if (j <= i) Gs[i * GLD + j] -= gi * Gs[j * GLD + a];
            }
        }
        __syncthreads();
    }
    return true;
}

__global__ void __launch_bounds__(512) svd_jacobi_kernel(const double* A, int lda, int trans, int p, int q,
                                                         double* G, double* Vs, double* sig,
                                                         double tau, int target, int* t_out,
                                                         int split_only) {
    // Columns of A and V live in LDS, 64 rows zero padded so every lane
    // handles exactly 4 rows without masks, at the stride CLD.
    constexpr int LD = CLD;
    __shared__ double As[64 * LD];
    __shared__ double V[64 * LD];
    __shared__ double sg[64];
    __shared__ int perm[64];
    __shared__ int rotated;
    __shared__ int nsweeps;
    __shared__ double wmax[8];
    // rank-t split certificate (split_only): Gram matrix, ranks, reductions
    __shared__ double Gs[64 * GLD];
    __shared__ double nd[64];
    __shared__ int ord[64];
    __shared__ double red[8][7];
    __shared__ int cstats[2];  // Cholesky attempts, pivots done in failed ones
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
    if (tid == 0) {
        nsweeps = 0;
        cstats[0] = cstats[1] = 0;
    }
    // One column pair per 16-lane group; lane l16 holds rows l16, l16+16, ...
    const int g8 = tid >> 4, l8 = tid & 15;
    __syncthreads();
    // A truncation to a fixed rank tt only needs the kept subspace: with
    // nothing to drop, any V will do (no sweep); otherwise sweeping stops
    // once split_certified holds.  The kept columns are then orthogonal to
    // the dropped ones but not necessarily to each other.
    const int tt = min(max(target, 1), q);
    const bool split = split_only && tau < 0.0;
    bool skip_test = false;  // uniform: the last test found the split far off
    for (int sweep = 0; sweep < 60 && q >= 2 && !(split && tt >= q); ++sweep) {
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
        if (split) {
            if (skip_test)
                skip_test = false;
            else if (split_certified(As, q, tt, Gs, nd, ord, red, cstats, skip_test))
                break;
        }
    }
    // Column norms; order by decreasing squared norm, ties by index (the
    // order split_certified uses): thread (column tid/8, part tid%8) counts
    // the larger norms among columns part + 8u, summed over its 8 lanes.
    for (int c = g8; c < q; c += 32) {
        double s = 0.0;
        for (int i = l8; i < 64; i += 16) s += As[c * LD + i] * As[c * LD + i];
        s = group16_sum(s);
        if (l8 == 0) {
            nd[c] = s;
            sg[c] = ldexp(sqrt(s), sexp);
        }
    }
    __syncthreads();
    {
        const int c = tid >> 3, part = tid & 7;
        const double me = c < q ? nd[c] : 0.0;
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = part + 8 * u;
            if (i < q) {
                const double o = nd[i];
                cnt += (o > me) || (o == me && i < c);
            }
        }
        cnt += __builtin_amdgcn_mov_dpp(cnt, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
        cnt += __builtin_amdgcn_mov_dpp(cnt, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
        cnt += __builtin_amdgcn_mov_dpp(cnt, 0x141, 0xF, 0xF, true);  // row_half_mirror
        if (part == 0) perm[c] = c;  // a valid column in every slot even if a NaN norm broke the ranking
        __syncthreads();
        if (part == 0 && c < q) perm[cnt] = c;
    }
    __syncthreads();
    // column r of G and Vs from column perm[r]: thread (r = tid/8, rows tid%8 + 8u)
    {
        const int r = tid >> 3, i0 = tid & 7;
        if (r < q) {
            const int pc = perm[r];
            for (int i = i0; i < p; i += 8) G[(size_t)r * p + i] = ldexp(As[pc * LD + i], sexp);
            for (int i = i0; i < q; i += 8) Vs[(size_t)r * q + i] = V[pc * LD + i];
        }
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
            t = tt;
        }
        t_out[0] = t;
        t_out[1] = nsweeps;
        t_out[2] = cstats[0];
        t_out[3] = cstats[1];
    }
}

// ---------------------------------------------------------------------------
// Wide one-sided Jacobi (q <= kSvdWideMax columns, p >= q rows).  One
// workgroup on one CU cannot sweep hundreds of columns quickly: every round
// moves the whole of A and V through that CU's L2 port.  Here a round of
// the circle-method tournament (column Q-1 fixed, the others rotating; Q = q
// rounded up to even, the extra column absent) is one launch with one
// workgroup per column pair, so a round costs about one launch whatever q
// is.  A and V are column-major in global memory.  The host runs Q - 1
// rounds per sweep and reads the sweep's rotation count.
// ---------------------------------------------------------------------------
constexpr int kWideThreads = 256;

__device__ __forceinline__ double wide_elem(const double* A, int lda, int trans, int i, int c) {
    return trans ? A[(size_t)i * lda + c] : A[(size_t)c * lda + i];
}

// The exponent e of max |A| (2^e > max |A| >= 2^(e-1)): columns are scaled
// by 2^-e so squared norms neither overflow nor lose small columns.
__global__ void __launch_bounds__(1024) wide_amax_kernel(const double* A, int lda, int trans, int p, int q,
                                                         int* sexp) {
    __shared__ double wmax[16];
    double m = 0.0;
    const int64_t total = (int64_t)p * q;
    for (int64_t t = threadIdx.x; t < total; t += 1024) {
        const int c = (int)(t / p), i = (int)(t - (int64_t)c * p);
        m = fmax(m, fabs(wide_elem(A, lda, trans, i, c)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = wmax[0];
        for (int w = 1; w < 16; ++w) a = fmax(a, wmax[w]);
        int e = 0;
        if (a > 0.0 && a < INFINITY) (void)frexp(a, &e);
        sexp[0] = e;
    }
}

// Aw = 2^-e A (column-major, ld p), Vw = I (q x q).
__global__ void __launch_bounds__(256) wide_init_kernel(const double* A, int lda, int trans, int p, int q,
                                                        const int* sexp, double* Aw, double* Vw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t na = (int64_t)p * q, nv = (int64_t)q * q;
    const int e = sexp[0];
    if (t < na) {
        const int c = (int)(t / p), i = (int)(t - (int64_t)c * p);
        Aw[t] = ldexp(wide_elem(A, lda, trans, i, c), -e);
    } else if (t < na + nv) {
        const int64_t u = t - na;
        const int c = (int)(u / q), i = (int)(u - (int64_t)c * q);
        Vw[u] = (i == c) ? 1.0 : 0.0;
    }
}

// Pair blockIdx.x of round r: (r, Q-1) for the first pair, else the columns
// (r + k) and (r - k) modulo Q - 1.  Each thread sums its rows of the three
// inner products; the waves' partials are added in wave order.
__global__ void __launch_bounds__(kWideThreads) wide_round_kernel(double* Aw, double* Vw, int p, int q, int Q,
                                                                  int r, double tol2, unsigned* rotated) {
    __shared__ double part[3][kWideThreads / 64];
    const int k = blockIdx.x, m = Q - 1;
    int i, j;
    if (k == 0) {
        i = r;
        j = m;
    } else {
        i = (r + k) % m;
        j = (r - k + m) % m;
    }
    if (i >= q || j >= q) return;  // the absent column of an odd q (uniform per workgroup)
    double* x = Aw + (size_t)i * p;
    double* y = Aw + (size_t)j * p;
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int t = threadIdx.x; t < p; t += kWideThreads) {
        const double a = x[t], b = y[t];
        al = fma(a, a, al);
        be = fma(b, b, be);
        ga = fma(a, b, ga);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        al += __shfl_xor(al, off, 64);
        be += __shfl_xor(be, off, 64);
        ga += __shfl_xor(ga, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][w] = al;
        part[1][w] = be;
        part[2][w] = ga;
    }
    __syncthreads();
    al = part[0][0];
    be = part[1][0];
    ga = part[2][0];
#pragma unroll
    for (int u = 1; u < kWideThreads / 64; ++u) {
        al += part[0][u];
        be += part[1][u];
        ga += part[2][u];
    }
    if (!(ga * ga > tol2 * (al * be))) return;  // uniform: already orthogonal to the tolerance
    if (threadIdx.x == 0) atomicAdd(rotated, 1u);
    double c, sn;
    jacobi_cs(al, be, ga, c, sn);
    for (int t = threadIdx.x; t < p; t += kWideThreads) {
        const double a = x[t], b = y[t];
        x[t] = c * a - sn * b;
        y[t] = sn * a + c * b;
    }
    double* vx = Vw + (size_t)i * q;
    double* vy = Vw + (size_t)j * q;
    for (int t = threadIdx.x; t < q; t += kWideThreads) {
        const double a = vx[t], b = vy[t];
        vx[t] = c * a - sn * b;
        vy[t] = sn * a + c * b;
    }
}

// Column norms, order by decreasing norm (ties by index), G = A V sorted and
// rescaled, Vs, sig and the kept rank by the tail rule (tau >= 0) or the
// target, as the one-workgroup kernel reports them.
__global__ void __launch_bounds__(1024) wide_finish_kernel(const double* Aw, const double* Vw, const int* sexp,
                                                           int p, int q, double* G, double* Vs, double* sig,
                                                           double tau, int target, int sweeps, int* t_out) {
    __shared__ double nd[kSvdWideMax], sg[kSvdWideMax];
    __shared__ int perm[kSvdWideMax];
    const int e = sexp[0];
    for (int c = threadIdx.x; c < q; c += 1024) {
        const double* col = Aw + (size_t)c * p;
        double s = 0.0;
        for (int i = 0; i < p; ++i) s = fma(col[i], col[i], s);
        nd[c] = s;
        sg[c] = ldexp(sqrt(s), e);
        perm[c] = c;  // a valid column in every slot even if a NaN norm breaks the ranking
    }
    __syncthreads();
    int rank_of[(kSvdWideMax + 1023) / 1024];
#pragma unroll
    for (int u = 0; u < (kSvdWideMax + 1023) / 1024; ++u) {
        const int c = threadIdx.x + 1024 * u;
        int cnt = -1;
        if (c < q) {
            const double me = nd[c];
            cnt = 0;
            for (int o = 0; o < q; ++o) cnt += (nd[o] > me) || (nd[o] == me && o < c);
        }
        rank_of[u] = cnt;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (kSvdWideMax + 1023) / 1024; ++u)
        if (rank_of[u] >= 0 && rank_of[u] < q) perm[rank_of[u]] = threadIdx.x + 1024 * u;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < (int64_t)p * q; t += 1024) {
        const int rr = (int)(t / p), i = (int)(t - (int64_t)rr * p);
        G[t] = ldexp(Aw[(size_t)perm[rr] * p + i], e);
    }
    for (int64_t t = threadIdx.x; t < (int64_t)q * q; t += 1024) {
        const int rr = (int)(t / q), i = (int)(t - (int64_t)rr * q);
        Vs[t] = Vw[(size_t)perm[rr] * q + i];
    }
    for (int c = threadIdx.x; c < q; c += 1024) sig[c] = sg[perm[c]];
    if (threadIdx.x == 0) {
        int t = q;
        if (tau >= 0.0) {
            double acc = 0.0;
            for (int rr = q - 1; rr >= 1; --rr) {
                const double sv = sg[perm[rr]];
                acc += sv * sv;
                if (sqrt(acc) <= tau)
                    t = rr;
                else
                    break;
            }
        } else {
            t = min(max(target, 1), q);
        }
        t_out[0] = t;
        t_out[1] = sweeps;
        t_out[2] = 0;
        t_out[3] = 0;
    }
}

}  // namespace

void launch_svd_jacobi(const double* A, int lda, int p, int q, double* G, double* Vs, double* sig,
                       double tau, int target, int* t_out, hipStream_t s, bool trans,
                       bool split_only) {
    if (q < 1 || q > 64 || p < q || p > 64)
        throw Error(-6, "small SVD: need 1 <= q <= p <= 64");
    hipLaunchKernelGGL(svd_jacobi_kernel, dim3(1), dim3(512), 0, s, A, lda, trans ? 1 : 0, p, q, G, Vs, sig,
                       tau, target, t_out, split_only ? 1 : 0);
    TTR_CHECK_LAUNCH();
}

int svd_wide_max() { return kSvdWideMax; }

double svd_wide_tol2(int p) {
    // rotate while (x.y)^2 > tol^2 (x.x)(y.y), tol well above the rounding
    // error of a p-term inner product so that a sweep can end without one
    const double tol = 1e-13 * std::max(1.0, (double)p / 64.0);
    return tol * tol;
}

void launch_svd_wide_init(const double* A, int lda, int p, int q, bool trans, double* Aw, double* Vw, int* sexp,
                          hipStream_t s) {
    if (q < 1 || q > kSvdWideMax || p < q) throw Error(-6, "wide SVD: need 1 <= q <= p, q <= 512");
    hipLaunchKernelGGL(wide_amax_kernel, dim3(1), dim3(1024), 0, s, A, lda, trans ? 1 : 0, p, q, sexp);
    TTR_CHECK_LAUNCH();
    const int64_t work = (int64_t)p * q + (int64_t)q * q;
    hipLaunchKernelGGL(wide_init_kernel, dim3(ceil_div(work, 256)), dim3(256), 0, s, A, lda, trans ? 1 : 0, p, q,
                       sexp, Aw, Vw);
    TTR_CHECK_LAUNCH();
}

void launch_svd_wide_round(double* Aw, double* Vw, int p, int q, int round, unsigned* rotated, hipStream_t s) {
    const int Q = q + (q & 1);
    if (Q < 2 || round < 0 || round >= Q - 1) throw Error(-1, "wide SVD: bad round");
    hipLaunchKernelGGL(wide_round_kernel, dim3(Q / 2), dim3(kWideThreads), 0, s, Aw, Vw, p, q, Q, round,
                       svd_wide_tol2(p), rotated);
    TTR_CHECK_LAUNCH();
}

void launch_svd_wide_finish(const double* Aw, const double* Vw, const int* sexp, int p, int q, double* G,
                            double* Vs, double* sig, double tau, int target, int sweeps, int* t_out,
                            hipStream_t s) {
    if (q < 1 || q > kSvdWideMax || p < q) throw Error(-6, "wide SVD: need 1 <= q <= p, q <= 512");
    hipLaunchKernelGGL(wide_finish_kernel, dim3(1), dim3(1024), 0, s, Aw, Vw, sexp, p, q, G, Vs, sig, tau, target,
                       sweeps, t_out);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr
