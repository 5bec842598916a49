// Batched adaptive KRP rounding in one persistent launch (batch.hip): the
// per-tensor descriptor the host writes into device memory and the launch
// interface.
#pragma once

#include "common.hpp"

namespace ttr {

// Largest QR panel (sketch block) of the batched kernel.
constexpr int kBatchMaxBlock = 64;
// Doubles of each tensor's run record: tau, nrmx, iterations, passes,
// generated columns, Householder fallbacks, shifted CholeskyQR passes,
// smallest |est - tau| / tau, then (first core, columns) of every
// partial-contraction pass (at most kBatchMaxPasses), then the device
// wall clock (100 MHz ticks) when the first member started the tensor and
// when it finished.
constexpr int kBatchMaxPasses = 24;
constexpr int kBatchInfoClock = 8 + 2 * kBatchMaxPasses;
// Then the first member's time (ticks) in each phase: partial contractions
// (with Omega), sketch products, thin QRs, residual projections with the
// estimate, and the projection, output copy and next core.
constexpr int kBatchPhases = 5;
constexpr int kBatchInfo = kBatchInfoClock + 2 + kBatchPhases;

// One tensor of the batch.  Every pointer is device memory; the scratch
// pointers are this tensor's own regions of the caller's workspace.
struct BatchTT {
    int d;          // order
    int T;          // workgroups that round this tensor together (team size)
    int ell_block;  // columns per residual block; <= 0: ceil(0.05 rbar_k) per mode
    int lcap;       // sketch column capacity (row stride of Omega and W)
    int r0;         // ceil(f_init * max_k r_k): the Remark 1 sample
    int init_cols;  // columns of the first right-to-left pass (>= r0, <= lcap)
    int has_nrmx;   // 1: nrmx given, else the Remark 1 estimate
    int pad_;
    double tol, nrmx, f_init;
    uint64_t seed;
    const int64_t* n;         // [d]
    const int64_t* r;         // [d+1]
    const double* const* X;   // [d] input cores
    double* const* Y;         // [d] output cores (capacity checked by the host)
    int64_t* ranks;           // [d+1] output ranks
    const int64_t* ooff;      // [d+1] offset of Omega_j in om (j = 2..d)
    const int64_t* woff;      // [d+1] offset of W_j in w (j = 2..d)
    double* om;               // Omega_j(i, c) at om[ooff[j] + i*lcap + c]
    double* w;                // W_j(a, c) at w[woff[j] + a*lcap + c]
    double* q;                // sketch basis Q and residual block, column-major
    double* yb[2];            // ping-pong V(Y_k) of the sweep
    double* m;                // projection M_k (lcap x rmax)
    double* slots;            // 2 x T partial slots of pslot doubles
    double* priv;             // T member-private regions of privs doubles each
    int64_t privs;            // kBatchPrivRinv + lcap * kBatchMaxBlock
    double* hh;               // Householder reflectors (rows x kBatchMaxBlock)
    int64_t pslot;
    unsigned* bar;            // team barrier: arrivals, generation
    int* status;              // bit 0: a team barrier timed out
    double* info;             // kBatchInfo doubles
};

// Member-private doubles: R^{-1} (64 x 64), then the reduced Q^T S block
// (lcap x 64 at most).
constexpr int kBatchPrivRinv = kBatchMaxBlock * kBatchMaxBlock;

// Persistent launch: `grid` workgroups take (tensor, member) tickets from
// *ticket (zeroed by the launch) in the order order[0..count) with team
// slots prefix[0..count] (prefix[count] = total), and run the adaptive
// rounding of their tensor as one member of its team.  `zero` (zwords
// unsigned ints: ticket, barriers, statuses) is cleared first by a fill
// kernel on the same stream.
void launch_batch(const BatchTT* tts, const int* order, const int* prefix, int count, unsigned* ticket,
                  unsigned* zero, int64_t zwords, int grid, hipStream_t s);
// Workgroups of the persistent kernel that can be resident at once.
int batch_resident_workgroups();

}  // namespace ttr
