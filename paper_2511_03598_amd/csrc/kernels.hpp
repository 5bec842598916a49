// Launch interfaces of the device kernels of libttround (gfx950).
#pragma once

#include "common.hpp"

namespace ttr {

// ---- Gaussian mode factors (omega.hip) ------------------------------------
struct OmegaArgs {
    uint64_t seed;
    int first_mode;      // 1-based first mode of the launch
    const int64_t* n;    // device [nmodes] sizes of modes first_mode, first_mode+1, ...
    const int64_t* off;  // device [nmodes] element offsets of those Omega_j in `base`
    double* base;        // storage: Omega_j(i, col) at base[off[j-first_mode] + i*ld + col]
    int64_t ld;          // row stride (column capacity)
    int64_t col0;        // first global sketch column generated
    int64_t store_col0;  // storage column where global column col0 goes
    int64_t ncols;
};
void launch_omega(const OmegaArgs& a, int nmodes, int64_t max_n, hipStream_t s);
void launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                   hipStream_t s);

// ---- KRP partial contraction of one core (partial.hip) --------------------
// W_k(a, c) = sum_i Omega_k(i, c) sum_b X_k(a, i, b) W_{k+1}(b, c) for
// storage columns c in [c0, c0+nc).  W is stored transposed: entry (a, c)
// of a slice at c * ld + a, ld a multiple of 4 (at least the row count),
// and split into slices: W_k is stored as pc_slices(r_{k-1}, r_k, prec)
// partial matrices (ss elements apart) whose sum, in slice order, is W_k.
// For reduced precision W is float32 or bfloat16 with a per-column int
// exponent: true W_k(:, c) = sum of slices(:, c) * 2^colexp_k[c].
struct PcArgs {
    const double* X;     // core k (r0 x n x r1), float64
    int r0, n, r1;
    const void* Wn;      // W_{k+1} storage (nullptr: the last core, W_{d+1} = 1)
    int64_t in_ld, in_ss;
    int in_slices;
    const double* Om;    // Omega_k storage, row stride ldo
    int64_t ldo;
    void* Wout;          // W_k storage (room for pc_slices(r0, r1, prec) slices)
    int64_t out_ld, out_ss;
    int c0, nc;
    // reduced precision only:
    const int* in_maxexp;   // per-workgroup max exponents written by the launch that made
                            // W_{k+1} in this pass (r1 x ceil(nc/64) x in_slices; nullptr at k=d)
    int* out_maxexp;        // this launch's entries (r0 x ceil(nc/64) x slices)
    const int* in_colexp;   // colexp_{k+1} (nullptr at k=d)
    int* out_colexp;        // colexp_k
    // FP64 only: terms > 1 contracts core k of `terms` TTs of the same shape
    // in one launch; the cores, W_{k+1} and W_k of term i are Xt[i], Wnt[i]
    // and Woutt[i] (device pointer tables; X, Wn and Wout then name term 0's
    // for the argument checks), every term with the same strides.
    int terms;
    const double* const* Xt;
    const void* const* Wnt;
    void* const* Woutt;
};
// Number of K slices of the contraction of an r0 x n x r1 core (prec 0 FP64,
// 1 FP32, 2 BF16); depends on the shape only, so every column block of W_k
// is split the same way.  A grouped launch of t terms uses
// pc_slices(t r0, r1, 0).
int pc_slices(int64_t r0, int64_t r1, int prec);
void launch_pc_f64(const PcArgs& a, hipStream_t s);
void launch_pc_f32(const PcArgs& a, hipStream_t s);
// BF16: W storage is bfloat16 (uint16 bits) with per-column exponents.
void launch_pc_bf16(const PcArgs& a, hipStream_t s);
void launch_fill_int(int* p, int value, int64_t count, hipStream_t s);
// out(r, c) = W(r, c0 + c) as float64 for r < rows, c < nc, W transposed
// with row stride ld: the sum of `slices` slices (sstride elements apart)
// times 2^colexp[c0 + c] when colexp is given; w is double (prec 0), float
// (1) or bfloat16 bits (2).
void launch_w_export(int prec, const void* w, const int* colexp, int64_t ld, int rows, int c0,
                     int nc, int slices, int64_t sstride, double* out, int64_t ldo, hipStream_t s);

// ---- left-to-right KRP partial contraction of one core (lr.hip) ----------
// W(b, c) = sum_{a, i} X(a, i, b) Wp(a, c) Om(i, c) for b < r1, c < nc; X is
// an r0 x n x r1 core (b fastest); Wp == nullptr stands for W^L_0 = 1 (then
// r0 must be 1).  Split-K slices write partials (splits x r1 x nc doubles).
struct LrArgs {
    const double* X;
    int r0, n, r1;
    const double* Wp;  // Wp(a, c) at Wp[a * ldw + c]
    int64_t ldw;
    const double* Om;  // Om(i, c) at Om[i * ldo + c]
    int64_t ldo;
    double* W;         // W(b, c) at W[b * ldwo + c]
    int64_t ldwo;
    int nc;
};
// K slices launch_lr uses for one core; the caller provides
// splits * r1 * nc doubles of partials when this exceeds 1.
int lr_splits(int r0, int n, int r1, int nc);
void launch_lr(const LrArgs& g, int splits, double* partials, hipStream_t s);

// ---- general float64 MFMA GEMM (gemm.hip) ----------------------------------
// C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n), with arbitrary
// element strides.  B may instead be float storage Bf or bfloat16 storage
// Bh with a per-column power-of-two exponent bexp[n] (true B = Bf * 2^bexp[n]),
// and B may be stored as bslices slices bstride elements apart whose sum (in
// slice order, in the storage's arithmetic type) is B.
struct GemmArgs {
    int M, N, K;
    const double* A;
    int64_t sam, sak;
    const double* B;
    const float* Bf;             // FP32 storage (with bexp) instead of B
    const unsigned short* Bh;    // bfloat16 storage (with bexp) instead of B
    const int* bexp;
    int bslices;                 // <= 1: one slice
    int64_t bstride;
    int64_t sbk, sbn;
    double* C;
    int64_t scm, scn;
    int cdiv;                    // > 0: column c of C at (c / cdiv) * cs_hi + (c % cdiv) * scn
    int64_t cs_hi;
    double alpha, beta;
};
// `partials` must hold splits*M*N doubles when splits > 1.
void launch_gemm(const GemmArgs& g, int splits, double* partials, hipStream_t s);
// K slices launch_gemm uses for an M x N x K product; the caller provides
// splits * M * N doubles of partials when this exceeds 1.
int gemm_splits(int M, int N, int K);

// Sum of products over K segments in one launch (the sketch of a sum of TTs
// from its terms' W): C(m, n) = sum_s alpha_s sum_k A_s(m, k) B_s(k, n) for
// m < M, n < N, with A_s(m, k) at A[s][m * lda[s] + k] and B_s(k, n) the sum
// over slices q < slices[s] (in slice order) of B[s][q * ss[s] + n * ldb[s] +
// k]; C column-major, C(m, n) at C[m + n * ldc], overwritten.
constexpr int kSegGemmMax = 16;
struct SegGemm {
    int M, N, nseg;
    double* C;
    int64_t ldc;
    int K[kSegGemmMax];
    const double* A[kSegGemmMax];
    int64_t lda[kSegGemmMax];
    double alpha[kSegGemmMax];
    const double* B[kSegGemmMax];
    int64_t ldb[kSegGemmMax];
    int slices[kSegGemmMax];
    int64_t ss[kSegGemmMax];
};
void launch_seg_gemm(const SegGemm& g, hipStream_t s);

// ---- small utilities (util.hip) --------------------------------------------
// dst(i, j) = src(i, j) for a rows x cols matrix with arbitrary strides.
void launch_copy2d(const double* src, int64_t ssr, int64_t ssc, double* dst, int64_t dsr,
                   int64_t dsc, int rows, int cols, double scale, hipStream_t s);
// Deterministic sum of squares of a rows x cols strided matrix into *out
// (device).  `partial` holds >= 1024 doubles, `counter` one zeroed int.
void launch_sumsq(const double* a, int64_t sr, int64_t sc, int rows, int cols, double* out,
                  double* partial, int* counter, hipStream_t s);

// ---- thin QR, TSQR with Householder leaves (qr.hip) ------------------------
struct QrPlan {
    int m, b, lda;
    int hmax;      // max rows per leaf
    int P;         // leaves
    int levels;    // tree levels above the leaves
    int nodes;     // total nodes (leaves + internal)
    size_t lds_bytes;
};
QrPlan plan_qr(int m, int b, int lda);
size_t qr_workspace_doubles(const QrPlan& p);
// a (m x b, column-major, lda) is overwritten by Q with diag(R) >= 0.  If
// r_out is non-null, R (b x b, column-major, upper) is written there.
// `ws` holds qr_workspace_doubles(p) doubles, `counters` p.nodes zeroed ints
// (they are left zeroed on return).
void launch_qr(const QrPlan& p, double* a, double* r_out, double* ws, int* counters,
               hipStream_t s, const int* only_if = nullptr);
// CholeskyQR2 / shifted CholeskyQR3 fast path (qr_chol.hip), b <= 64,
// m >= b.  flags[0] is set to 1 when a pass breaks down (rank-deficient
// panel), in which case `a` is left untouched for the Householder path
// (launch_qr with only_if=flags); flags[1] records the shifted route.  A
// non-null `sticky` is also set to 1 on a breakdown and never cleared, so
// a caller can check many QRs at once.
size_t cq_workspace_doubles(int m, int b);
void launch_cq(double* a, int m, int b, int lda, double* r_out, double* ws, int* flags,
               hipStream_t s, int* sticky = nullptr);

// ---- small SVD by one-sided Jacobi (svd.hip) -------------------------------
// A (p x q, column-major, lda), p >= q, q <= 64.  On return: G (p x q,
// ld p) holds A*V with columns sorted by decreasing norm (= U*Sigma), Vs
// (q x q, ld q) the matching right singular vectors, sig[q] the singular
// values, and t_out[0] the kept rank: the smallest t >= 1 whose tail
// sqrt(sum_{j>=t} sig_j^2) <= tau if tau >= 0, else min(max(target,1), q)
// (t_out holds 4 ints: then sweeps and two counters of the split test).
// trans: A is given transposed, element (i, c) at A[i * lda + c] (a
// row-major p x q matrix, or the column-major R whose R^T is wanted).
// split_only (with tau < 0): the caller keeps only the first t = target
// columns of G and Vs and needs them to span the best rank-t subspaces,
// not to be singular vectors; sweeping stops once that split is certified
// (the kept columns of G are then orthogonal to the dropped ones, not
// necessarily to each other, and sig holds column norms).
void launch_svd_jacobi(const double* A, int lda, int p, int q, double* G, double* Vs,
                       double* sig, double tau, int target, int* t_out, hipStream_t s,
                       bool trans = false, bool split_only = false);

// Wide one-sided Jacobi (svd.hip), 1 <= q <= p, q <= svd_wide_max(): the
// same results as launch_svd_jacobi (G = A V sorted by decreasing column
// norm, Vs, sig, t_out[0] the kept rank, t_out[1] the sweeps) for any
// width.  The caller drives it: init (Aw = A scaled by a power of two,
// column-major ld p; Vw = I; sexp one device int), then sweeps of
// rounds 0 .. Q-2 (Q = q rounded up to even) with *rotated zeroed before
// each sweep and read after it (0: converged), then finish.  Aw, Vw must
// not alias A, G or Vs.
constexpr int kSvdWideMax = 512;
int svd_wide_max();
void launch_svd_wide_init(const double* A, int lda, int p, int q, bool trans, double* Aw, double* Vw, int* sexp,
                          hipStream_t s);
void launch_svd_wide_round(double* Aw, double* Vw, int p, int q, int round, unsigned* rotated, hipStream_t s);
void launch_svd_wide_finish(const double* Aw, const double* Vw, const int* sexp, int p, int q, double* G,
                            double* Vs, double* sig, double tau, int target, int sweeps, int* t_out,
                            hipStream_t s);

// dst = alpha src + beta dst for a rows x cols strided matrix; src == nullptr
// reads as zero and beta == 0 does not read dst (so this also fills zeros).
void launch_axpby2d(const double* src, int64_t ssr, int64_t ssc, double* dst, int64_t dsr, int64_t dsc, int rows,
                    int cols, double alpha, double beta, hipStream_t s);

int device_lds_limit();

}  // namespace ttr
