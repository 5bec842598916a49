/*
 * ttround.h -- C ABI of libttround.so: KRP-sketched randomized TT-rounding
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Al Daas, Ballard, Grigori, Martinez Aguilar, Saibaba, Verma,
 * "Adaptive Randomized Tensor Train Rounding using Khatri-Rao Products"
 * (arXiv 2511.03598).  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A TT tensor has d >= 2 cores X_k of shape (r_{k-1}, n_k, r_k) with
 *    r_0 = r_d = 1 (Sec. 2.2).  Cores are float64, row-major, so element
 *    (a, i, b) of core k sits at offset (a*n_k + i)*r_k + b; the vertical
 *    unfolding V(X_k) and horizontal unfolding H(X_k) are plain views.
 *  - Core and output pointers are DEVICE pointers on the current HIP
 *    device; the arrays that hold them, and dims/ranks, are HOST arrays.
 *  - Inputs are borrowed: they must stay valid and unmodified until the
 *    call returns (synchronous calls) or until tt_round_poll reports the
 *    request done (served calls).  The library never frees caller memory.
 *  - Work is enqueued on opts->stream (a hipStream_t; NULL = the null
 *    stream).  Synchronous entry points return after the result is complete
 *    on that stream (they synchronize it), so outputs are ready on return.
 *  - Errors are status codes; no exception crosses the ABI.  A thread-local
 *    message is available from tt_last_error().  On error the outputs are
 *    unspecified but no caller memory outside the outputs is written.
 *  - Determinism: the same inputs, seed and options give bitwise-identical
 *    outputs (fixed-order reductions, no floating-point atomics).
 *  - Threads: calls from different host threads are safe; calls that share
 *    a stream are serialized by it.
 *
 * Gaussian mode factors (Sec. 3.2, "Select random Gaussian matrices").  The
 * paper leaves the generator open; this library fixes Philox4x32-10
 * (Salmon et al., SC'11) with key (seed & 0xffffffff, seed >> 32) and
 * counter (p, c, j, 0x4B525031) for row pair p, global sketch column c and
 * 1-based mode j, and Box-Muller on two 53-bit uniforms
 * u = ((w_hi*2^32 + w_lo) >> 11) + 0.5) * 2^-53:
 *   Omega_j(2p, c)   = sqrt(-2 ln u1) cos(2 pi u2)
 *   Omega_j(2p+1, c) = sqrt(-2 ln u1) sin(2 pi u2).
 * Every entry is addressed by (seed, j, c, row), so a sketch column is the
 * same whichever pass or chunk generates it.
 */
#ifndef TTROUND_H
#define TTROUND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TT_OK = 0,
    TT_PENDING = 1,       /* served request not finished yet               */
    TT_EINVAL = -1,       /* bad argument (shape, rank, tol, pointer)      */
    TT_ENOMEM = -2,       /* output capacity too small or allocation failed */
    TT_ECAPACITY = -3,    /* admission refused (server budget)             */
    TT_EDEVICE = -4,      /* a HIP runtime error                           */
    TT_ENOTFOUND = -5,    /* unknown ticket                                */
    TT_EUNSUPPORTED = -6  /* valid request outside the implemented limits  */
} tt_status;

/* Precision of the right-to-left partial contractions (the KRP sketch,
 * Sec. 3.1) only; the sketch, QR, projection, estimator and recompression
 * steps always run in float64.  F32: float32 operands, storage and
 * accumulation.  BF16: cores rounded to bfloat16 in registers, W stored in
 * bfloat16, products accumulated in float32.  Reduced precisions keep a
 * power-of-two exponent per sketch column in int32 so that values stay in
 * range. */
typedef enum { TT_PREC_F64 = 0, TT_PREC_F32 = 1, TT_PREC_BF16 = 2 } tt_prec;

typedef struct {
    int32_t d;                  /* number of cores, >= 2                    */
    const int64_t* n;           /* host [d], n_k >= 1                       */
    const int64_t* ranks;       /* host [d+1], ranks[0] = ranks[d] = 1      */
    const double* const* cores; /* host [d] device pointers, see above      */
} tt_view;

typedef struct {
    int32_t d;                  /* must equal the input's d                 */
    int64_t* ranks;             /* host [d+1], written by the call          */
    double** cores;             /* host [d] caller-owned device buffers     */
    const int64_t* capacity;    /* host [d], elements per buffer            */
    int32_t orth;               /* written: 1 left-orth (all but last core),
                                   2 right-orth (all but first core)        */
} tt_out;

typedef struct {
    tt_prec prec;       /* partial-contraction precision, default F64        */
    double f_init;      /* initial sketch fraction, <= 0 means 0.1 (Sec. 3.3) */
    double nrmx;        /* ||X|| if known; <= 0: Remark 1 estimate             */
    int32_t recompress; /* adaptive: 1 = Remark 2 right-to-left truncation
                           pass with the same threshold tau; 0 = none        */
    void* stream;       /* hipStream_t; NULL = null stream                    */
} tt_opts;

typedef struct {        /* diagnostics of the calling thread's last rounding */
    double tau;         /* per-mode threshold tol*nrmx/sqrt(d-1)             */
    double nrmx;        /* norm used (given or Remark 1 estimate)            */
    double min_margin;  /* min |est - tau| / tau over adaptive decisions     */
    int32_t passes;     /* partial-contraction passes (1 + regenerations)    */
    int32_t iterations; /* adaptive loop iterations (estimates computed)     */
    int32_t qr_retries; /* 1 if the rounding was repeated because a CholeskyQR
                           broke down while the Householder fallback was
                           deferred (the result is that of the repeat)       */
    int64_t pc_launches; /* partial-contraction launches (one per core and
                            pass, Sec. 3.1)                                  */
    double pc_bytes;    /* their algorithmic bytes: one float64 read of every
                           contracted core plus the W_k writes               */
    double pc_flops;    /* their flops by the Sec. 3.1 cost model:
                           2 r_{k-1} n_k r_k l + 2 r_{k-1} r_k l per core      */
} tt_info;

/* Output capacity (elements) per core: cap[k-1] = c_{k-1} n_k c_k with
 * c_0 = c_d = 1 and c_k = min(r_k, n_1*...*n_k), which bounds the ranks of
 * every rounding of x (fixed or adaptive; target_ranks is accepted for
 * symmetry and may be NULL).  TT_EINVAL on a malformed view. */
tt_status tt_out_capacity(const tt_view* x, const int64_t* target_ranks, int64_t* cap);

/* Fixed-rank randomize-then-orthogonalize rounding with KRP sketches
 * (Sec. 3.2, Algorithm "Fixed Rank TT-Rounding: Randomize-then-Orthogonalize
 * using KRP").  Sketch size ell >= 1; the sketch rank at bond k is
 * l_k = min(ell, l_{k-1} n_k, r_k).  If target_ranks (host [d+1], may be
 * NULL) asks for fewer than l_k at some bond, a right-to-left SVD truncation
 * pass (Remark 2) cuts the result to min(target, l_k) there (oversampling).
 * y->orth is 1 without the pass, 2 with it.  Errors: TT_EINVAL (d < 2,
 * bad ranks, ell < 1, NULL pointers), TT_ENOMEM (capacity), TT_EDEVICE. */
tt_status tt_round_fixed(const tt_view* x, const int64_t* target_ranks, int64_t ell,
                         uint64_t seed, const tt_opts* opts, tt_out* y);

/* Allocation-free variant of tt_round_fixed, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result (bitwise the
 * same outputs and ranks) and errors as tt_round_fixed, but every device
 * buffer the rounding needs besides its inputs and outputs is carved from a
 * static device array of TT_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends; no hipMalloc, hipFree or
 * pinned host allocation happens in the call, and kernel timing
 * (tt_kernel_timing) does not record it.  TT_ENOMEM when the shape's
 * workspace estimate (tt_workspace_bytes with ell_max = ell) exceeds the
 * array, checked before any work is queued.  All calls on one GPU share the
 * array: the library serialises the calls of this process per device (each
 * returns after its stream is synchronized), and work queued on the array
 * by overlapping calls from elsewhere would race.  The Householder fallback
 * of the QRs is launched eagerly, so tt_last_info().qr_retries is 0. */
#define TT_NOALLOC_SCRATCH_BYTES (64u << 20)
tt_status tt_round_fixed_noalloc(const tt_view* x, const int64_t* target_ranks, int64_t ell,
                                 uint64_t seed, const tt_opts* opts, tt_out* y);

/* Adaptive-rank rounding to relative tolerance tol > 0 (Sec. 3.3, Algorithm
 * "Adaptive Rank TT-Rounding: Randomize-then-Orthogonalize using KRP", with
 * the residual sketching of Sec. 3.3 and Remark 1).  With tau =
 * tol*nrmx/sqrt(d-1), each mode starts from ceil(f_init*rbar_k) sketch
 * columns and grows by blocks of ell_block (<= 0: ceil(0.05*rbar_k)) while
 * ||S||_F/sqrt(b) > tau, drawing new Gaussian columns and re-running the
 * partial contractions on cores k+1..d when the sketch runs out.  Guarantee
 * (with high probability): ||X - Y|| <= tol ||X||.  Errors as above. */
tt_status tt_round_adaptive(const tt_view* x, double tol, int64_t ell_block, uint64_t seed,
                            const tt_opts* opts, tt_out* y);

/* ---- Rounding of a sum of TT tensors (the remark on sums, Sec. 3.3) ---- *
 * Y ~ sum_i w_i X^(i) for `count` >= 1 views of the same order d and mode
 * sizes (each with its own ranks), weights[count] on the host (NULL: all
 * 1).  The result is the rounding of the formal sum (first cores side by
 * side times the weights, block-diagonal middle cores, stacked last cores;
 * its ranks are the summed ranks) with the same seed, but the formal sum is
 * never assembled: every term is sketched on its own with the shared
 * Gaussian factors, so the partial contractions and the products with the
 * next cores cost sum_i r_i^2 instead of (sum_i r_i)^2.  Output capacities
 * and ranks are those of the formal sum (tt_sum_out_capacity).  Parameters,
 * options, guarantees and errors as for tt_round_fixed / tt_round_adaptive;
 * also TT_EINVAL when the views disagree in d or n. */
tt_status tt_sum_out_capacity(const tt_view* xs, int32_t count, const int64_t* target_ranks,
                              int64_t* cap);
tt_status tt_round_sum_fixed(const tt_view* xs, int32_t count, const double* weights,
                             const int64_t* target_ranks, int64_t ell, uint64_t seed,
                             const tt_opts* opts, tt_out* y);
tt_status tt_round_sum_adaptive(const tt_view* xs, int32_t count, const double* weights,
                                double tol, int64_t ell_block, uint64_t seed, const tt_opts* opts,
                                tt_out* y);

/* Deterministic TT-SVD rounding (Sec. 2.3, Algorithm "TT-Rounding"), the
 * same-GPU baseline of the randomized roundings: right-to-left
 * orthogonalisation of a working copy of x, then tau = tol ||X|| /
 * sqrt(d-1) and, left to right, a thin QR of V(Y_k), the SVD of its R
 * truncated by the tail rule (smallest t with sqrt(sum_{j>=t} s_j^2) <=
 * tau), Y_k = Q U_t and Y_{k+1} = S_t V_t^T H(Y_{k+1}).  With
 * target_ranks (host [d+1], interior entries >= 1) the bonds are truncated
 * to min(target, available) instead and tol is ignored.  Output: y
 * (capacities from tt_out_capacity), left-orthonormal (orth = 1); the
 * input is not modified.  Interior ranks up to 512 (TT_EUNSUPPORTED
 * otherwise).  Uses the library's workspace (about the size of x plus a
 * few cores), synchronises opts->stream, and records tau and ||X|| for
 * tt_last_info. */
tt_status tt_round_ttsvd(const tt_view* x, double tol, const int64_t* target_ranks, const tt_opts* opts,
                         tt_out* y);

/* Diagnostics of the calling thread's last tt_round_* call. */
tt_status tt_last_info(tt_info* info);

/* Thread-local message for the last non-OK status (never NULL). */
const char* tt_last_error(void);

/* ---- Hot-path components, exported for testing and benchmarking ----- */

/* Omega_mode(:, col0:col0+ncols) as a row-major n x ncols float64 device
 * array `out` (ld = ncols), mode 1-based (see the generator spec above). */
tt_status tt_gaussian_factor(uint64_t seed, int32_t mode, int64_t n, int64_t col0,
                             int64_t ncols, double* out, void* stream);

/* Raw Philox4x32-10 on `count` device counters/keys (uint32 ctr[4*count],
 * key[2*count]) into out[4*count]; for known-answer tests of the device
 * generator. */
tt_status tt_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                           int64_t count, void* stream);

/* Right-to-left KRP partial contractions (Sec. 3.1, Eq. 7-8):
 * W_d = H(X_d) Omega_d, W_k = H(X_k)[W_{k+1} (.) Omega_k], for k = d..t
 * over sketch columns [col0, col0+ncols), computed in `prec`.  w[k-t] is a
 * device float64 buffer for W_k of shape r_{k-1} x ncols, row-major
 * (ld = ncols), k = t..d; values are returned unscaled in float64. */
tt_status tt_partial_contractions(const tt_view* x, uint64_t seed, int64_t col0, int64_t ncols,
                                  int32_t t, tt_prec prec, double* const* w, void* stream);

/* Left-to-right KRP partial contractions (Sec. 3.1, the same recurrence
 * run from the first core): W^L_1 = V(X_1)^T Omega_1 and
 * W^L_k(b, c) = sum_{a,i} X_k(a, i, b) W^L_{k-1}(a, c) Omega_k(i, c), i.e.
 * W^L_k = V(X_k)^T [W^L_{k-1} (.) Omega_k], for k = 1..t (1 <= t <= d),
 * over sketch columns [col0, col0+ncols) of the factors drawn from `seed`
 * (the columns tt_gaussian_factor returns).  FP64 throughout.  w[k-1] is a
 * caller-owned device float64 buffer for W^L_k of shape r_k x ncols,
 * row-major (ld = ncols), k = 1..t; each W^L_k is read back as the operand
 * of the next core, so the buffers must not overlap.  Blocks until the
 * results are written.  TT_EINVAL for t outside [1, d], an empty or
 * negative column range or a null buffer. */
tt_status tt_partial_contractions_lr(const tt_view* x, uint64_t seed, int64_t col0, int64_t ncols,
                                     int32_t t, double* const* w, void* stream);

/* Thin QR with diag(R) >= 0 of an m x b column-major float64 device matrix
 * a (ld = m), m >= b >= 1, b <= 512: on return a holds Q (explicit).  The
 * same routine the rounding uses for its sketches: certified CholeskyQR2
 * with shifted-CholeskyQR3 and Householder fallbacks on panels of at most
 * 64 columns, and block Gram-Schmidt with reorthogonalisation across
 * panels when b > 64. */
tt_status tt_qr(double* a, int64_t m, int64_t b, void* stream);

/* SVD of a small p x q column-major float64 device matrix a (ld = p),
 * p >= q, 1 <= q <= 512, by one-sided Jacobi (the truncated SVD of the
 * right-to-left truncation pass, Remark 2): one workgroup when p, q <= 64,
 * else one launch per round of the column-pair tournament with a
 * readback of the rotation count per sweep.  Writes g = A V (p x q, ld p,
 * columns sorted by decreasing norm, i.e. U Sigma), v (q x q, ld q) and
 * sig[q]; *t_out (host) receives the kept rank: the smallest t >= 1 whose
 * tail sqrt(sum_{j>=t} sig_j^2) <= tau when tau >= 0, else
 * min(max(target, 1), q).  All arrays are device memory. */
tt_status tt_svd_small(const double* a, int64_t p, int64_t q, double* g, double* v, double* sig,
                       double tau, int64_t target, int64_t* t_out, void* stream);

/* Device workspace (bytes, an upper estimate) that one rounding of x uses
 * besides its inputs and outputs: ell_max > 0 for fixed rank with that
 * sketch size, <= 0 for adaptive (worst case: ranks up to the caps of
 * tt_out_capacity).  Host only.  TT_EINVAL on a malformed view. */
tt_status tt_workspace_bytes(const tt_view* x, int64_t ell_max, tt_prec prec, size_t* bytes);

/* Batched adaptive rounding (Sec. 3.3 applied to `count` independent
 * tensors): xs[i] is rounded to tol[i] with seed seeds[i] into ys[i] (caller
 * buffers sized by tt_out_capacity).  With a float64 sketch and no
 * recompression pass (opts NULL or prec F64, recompress 0) the batch runs
 * as one persistent launch (tt_batch_create / _launch / _finish below) on
 * a workspace the library keeps per device; every result is bitwise the
 * same alone or in any batch and agrees with tt_round_adaptive to rounding
 * error.  Otherwise the roundings run as tt_round_adaptive calls (bitwise
 * the same results) on a process-wide pool of worker threads, each with its
 * own HIP stream and workspace, so their kernels overlap on the device.
 * opts (may be NULL) applies to all; the call returns when every result is
 * complete.  Returns TT_OK, or the status of the first failed tensor (its
 * index is in tt_last_error()). */
tt_status tt_round_adaptive_batch(const tt_view* xs, int32_t count, const double* tol,
                                  int64_t ell_block, const uint64_t* seeds, const tt_opts* opts,
                                  tt_out* ys);

/* ---- Batched rounding in one persistent launch (graph-capturable) -------
 * The same roundings as tt_round_adaptive_batch (Sec. 3.3 on `count`
 * independent tensors, float64 sketch, no recompression pass), run by one
 * persistent kernel: workgroups take (tensor, member) tickets from a device
 * counter, largest tensors first, and each tensor is rounded by a team of
 * workgroups whose size depends on that tensor alone; every adaptive
 * decision is taken on the device.  A tensor's result is therefore bitwise
 * the same alone or in any batch; it agrees with tt_round_adaptive (the
 * same algorithm, seed and Gaussian factors, other kernels) to rounding
 * error.  Sketch blocks (ell_block and ceil(f_init rbar_k)) must not exceed
 * 64 columns (TT_EUNSUPPORTED).
 *
 * tt_batch_workspace_bytes: device workspace (bytes) of the batch.
 * tt_batch_create: validates the batch, lays it out in `workspace`
 *   (caller-owned device memory of at least that size) and uploads the
 *   descriptors (synchronising opts->stream).  The inputs, outputs (ys:
 *   caller buffers sized by tt_out_capacity) and workspace stay borrowed
 *   until tt_batch_destroy.  opts->prec must be F64 and opts->recompress 0
 *   (TT_EUNSUPPORTED otherwise).
 * tt_batch_launch: enqueues the counter reset and the persistent kernel on
 *   `stream` and returns; no allocation and no host synchronisation, so it
 *   may be recorded in a HIP graph and the graph replayed (every replay
 *   recomputes every result).
 * tt_batch_finish: synchronises `stream`, writes every ys[i].ranks and
 *   ys[i].orth (1), and returns TT_EDEVICE naming the first tensor whose
 *   team barrier timed out (the kernel still ends; such a result is
 *   invalid).
 * tt_batch_info: the run record of tensor i after tt_batch_finish (tau,
 *   nrmx, iterations, passes, min_margin, and the partial-contraction
 *   counters with pc_launches counting contracted cores over all passes).
 * tt_batch_team: the team size (workgroups) of tensor i.
 * tt_batch_record: tensor i's raw run record (below). */
typedef struct tt_batch tt_batch;
tt_status tt_batch_workspace_bytes(const tt_view* xs, int32_t count, int64_t ell_block,
                                   const tt_opts* opts, size_t* bytes);
tt_status tt_batch_create(const tt_view* xs, int32_t count, const double* tol, int64_t ell_block,
                          const uint64_t* seeds, const tt_opts* opts, tt_out* ys, void* workspace,
                          size_t workspace_bytes, tt_batch** batch);
tt_status tt_batch_launch(const tt_batch* batch, void* stream);
tt_status tt_batch_finish(tt_batch* batch, void* stream);
tt_status tt_batch_info(const tt_batch* batch, int32_t i, tt_info* info);
tt_status tt_batch_team(const tt_batch* batch, int32_t i, int32_t* team);
/* Raw run record of tensor i after tt_batch_finish, up to cap doubles into
 * out (count in *n): tau, nrmx, iterations, passes, generated columns,
 * Householder fallbacks, shifted CholeskyQR passes, min |est-tau|/tau, then
 * 24 (first core, columns) pairs of the partial-contraction passes, then
 * the device wall clock (100 MHz ticks) at the tensor's start and end. */
tt_status tt_batch_record(const tt_batch* batch, int32_t i, double* out, int32_t cap, int32_t* n);
void tt_batch_destroy(tt_batch* batch);

/* ---- Work-decomposition autotuner of the persistent batch --------------
 * A tensor of the batch is rounded by a team of T workgroups, T the largest
 * power of two (at most min(32, resident workgroups / 2)) with 2T times the
 * device's team threshold F0 below the tensor's work estimate (flops of the
 * rounding model of Sec. 3.1 and the sweep).  F0 sets how finely the
 * persistent kernel splits large tensors against how much it pays in team
 * barriers.  It belongs to the device, not to a batch, so a tensor's team,
 * and with it the bits of its result, is the same alone or in any batch
 * created while F0 is unchanged; a batch created before F0 changes keeps
 * its layout.
 *
 * tt_batch_autotune: rounds the given batch (arguments as tt_batch_create,
 *   results in ys) three times per candidate F0 (after one untimed launch),
 *   times each launch with HIP events on opts->stream, stores the median of
 *   the three in times_ms[j], sets the
 *   current device's F0 to the fastest candidate (*best) and, when the
 *   environment variable TTR_BATCH_TUNE_CACHE names a file, appends
 *   "<gcnArchName>/<compute units> <F0>" to it; the last such line for a
 *   device is its F0 in later processes.  A set-up call: it allocates and
 *   frees its own workspace and synchronises the stream.  ncand in [1, 64],
 *   candidates > 0 (TT_EINVAL otherwise).
 * tt_batch_team_flops: value > 0 sets the current device's F0, value < 0
 *   clears it (the cache file, then TTR_BATCH_TEAM_FLOPS, then 3e9 apply),
 *   0 leaves it; *current (may be NULL) receives the value in force. */
tt_status tt_batch_autotune(const tt_view* xs, int32_t count, const double* tol, int64_t ell_block,
                            const uint64_t* seeds, const tt_opts* opts, tt_out* ys, const double* candidates,
                            int32_t ncand, double* times_ms, double* best);
tt_status tt_batch_team_flops(double value, double* current);

/* ---- Served rounding ---------------------------------------------------
 * A server owns worker threads (one HIP stream each) on the device current
 * at creation.  Requests queue in arrival order and start as soon as a
 * worker is free and their device-memory footprint (tt_workspace_bytes plus
 * four times the output capacity: capacity-sized staging and the exact-size
 * result, each from power-of-two pool classes) fits the budget beside the
 * running requests and the results not yet released; a request that fits
 * may start before an earlier one that does not (at most four times per
 * waiting request).  The budget counts request footprints only: the
 * workspaces and pool buffers the library caches for reuse between requests
 * (at most one workspace per worker thread, grown to the largest request it
 * ran) are not counted, so leave headroom for them below the device's free
 * memory.
 * New requests are admitted while others run, and their kernels overlap on
 * the device.  Each result is bitwise the same as the synchronous call with
 * the same arguments. */
typedef struct {
    size_t mem_budget; /* bytes; 0 = 80% of the device's free memory        */
    int32_t workers;   /* requests in flight at once; <= 0 = 8 (max 64)      */
} tt_server_cfg;

typedef struct {
    int32_t kind;                /* 0 adaptive (tol, ell_block), 1 fixed   */
    tt_view x;                   /* borrowed until poll reports completion */
    double tol;                  /* adaptive                               */
    int64_t ell_block;           /* adaptive, as in tt_round_adaptive      */
    int64_t ell;                 /* fixed                                  */
    const int64_t* target_ranks; /* fixed, host [d+1] or NULL; copied     */
    uint64_t seed;
    tt_opts opts;                /* prec, f_init, nrmx, recompress; the
                                    stream field is ignored               */
} tt_request;

typedef struct {
    tt_status status;       /* TT_OK or the rounding's error status         */
    const char* error;      /* message when status != TT_OK, else ""        */
    int32_t d;
    const int64_t* ranks;   /* host [d+1]                                   */
    double* const* cores;   /* host [d] device pointers, library-owned,
                               exact size r_{k-1} n_k r_k, row-major        */
    int32_t orth;           /* 1 left-orth, 2 right-orth                    */
    tt_info info;
    double submit_s, start_s, done_s; /* host steady-clock times (seconds)  */
} tt_result;

typedef struct tt_server tt_server;

/* TT_EINVAL on NULL out; TT_EDEVICE if no device is usable. */
tt_status tt_server_create(const tt_server_cfg* cfg, tt_server** out);

/* Validates the request on the host and queues it; *ticket identifies it.
 * TT_ECAPACITY if its footprint exceeds the whole budget. */
tt_status tt_round_submit(tt_server* s, const tt_request* req, uint64_t* ticket);

/* TT_PENDING while queued or running; TT_OK with *out set once done (the
 * ticket is then consumed); TT_ENOTFOUND for an unknown ticket. */
tt_status tt_round_poll(tt_server* s, uint64_t ticket, tt_result** out);

/* Like tt_round_poll but blocks until the request is done. */
tt_status tt_round_wait(tt_server* s, uint64_t ticket, tt_result** out);

/* Copies the result's cores into caller device buffers dst[k] (each at
 * least ranks[k-1] n_k ranks[k] doubles) on `stream` and waits for the
 * copies.  TT_EINVAL for a NULL argument or a failed result. */
tt_status tt_result_copy(const tt_result* r, double* const* dst, void* stream);

/* Returns the result's device buffers to the server's pool.  Every result
 * must be released before its server is destroyed. */
void tt_result_release(tt_result* r);

/* Waits for running requests, drops queued ones, frees the pool. */
void tt_server_destroy(tt_server* s);

/* ---- Kernel timing (instrumentation) ----------------------------------
 * When enabled, the library records a pair of HIP events on the launch
 * stream around the launches of each kind below, in every thread: around
 * each GEMM, QR and SVD, and around the back-to-back partial-contraction
 * launches of a pass (counted as one launch per core); reading sums the
 * elapsed times of the recorded pairs.  Used to put per-launch durations
 * beside algorithmic byte and flop counts. */
typedef enum {
    TT_KERNEL_PARTIAL_CONTRACTION = 0, /* one launch per core and pass (Sec. 3.1)  */
    TT_KERNEL_GEMM = 1,                /* sketch, projection and core products     */
    TT_KERNEL_QR = 2,                  /* one thin QR (all of its kernels)         */
    TT_KERNEL_SVD = 3,                 /* one small SVD (Remark 2 truncation)      */
    TT_KERNEL_KINDS = 4
} tt_kernel_kind;

/* kinds != 0: clear the counters and start recording the kinds whose bit
 * (1 << tt_kernel_kind) is set, e.g. TT_KERNEL_TIMING_ALL; 0: stop
 * recording (recorded pairs stay readable).  Every recorded pair adds a
 * little time on the stream, so a measurement that only needs one kind
 * should record only that kind.  TT_EINVAL for bits beyond the kinds. */
#define TT_KERNEL_TIMING_ALL ((1 << TT_KERNEL_KINDS) - 1)
tt_status tt_kernel_timing(int32_t kinds);

/* Launches recorded for `kind` and their summed duration in milliseconds;
 * waits for the recorded events to complete.  TT_EINVAL on a bad kind or
 * NULL outputs. */
tt_status tt_kernel_timing_read(int32_t kind, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* TTROUND_H */
