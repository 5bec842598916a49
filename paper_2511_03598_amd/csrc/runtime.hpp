// Host runtime of libttround: shape validation, workspace pool, and the
// launch sequences of the fixed-rank and adaptive KRP roundings.
#pragma once

#include <vector>

#include "kernels.hpp"

namespace ttr {

struct Shape {
    int d = 0;
    std::vector<int64_t> n;  // [d]
    std::vector<int64_t> r;  // [d+1]
};

struct Options {
    int prec = 0;          // 0 f64, 1 f32, 2 bf16 (partial contractions only)
    double f_init = 0.1;
    double nrmx = 0.0;     // <= 0: Remark 1 estimate
    int recompress = 0;
    hipStream_t stream = nullptr;
};

struct RoundInfo {
    double tau = 0, nrmx = 0, min_margin = 0;
    int passes = 0, iterations = 0;
    int qr_retries = 0;  // 1: repeated with the eager Householder fallback
    int64_t pc_launches = 0;              // partial-contraction launches
    double pc_bytes = 0.0, pc_flops = 0.0;  // their algorithmic bytes and flops
};

// Output cores: caller-owned device buffers with capacities (elements).
struct OutCores {
    double** cores;
    const int64_t* cap;
    int64_t* ranks;  // [d+1], written
    int orth = 0;    // written: 1 left, 2 right
};

// A TT given as a weighted sum of TTs with the same mode sizes (one term
// for a plain TT).  The formal shape has the summed interior ranks: the
// rounding of the sum is the rounding of the formal sum (first cores side
// by side with the weights, block-diagonal middle cores, stacked last
// cores), which is never assembled.
struct Summands {
    Shape fs;                                 // formal shape
    std::vector<Shape> sh;                    // per term
    std::vector<const double* const*> cores;  // per term: d device pointers
    std::vector<double> w;                    // per term weight (first core)
    std::vector<std::vector<int64_t>> off;    // per term: offsets in the formal ranks, [d+1]
    int m() const { return (int)sh.size(); }
};
Summands single_term(const Shape& s, const double* const* cores);
// weights: nullptr for all 1.
Summands make_sum(const std::vector<Shape>& sh, const std::vector<const double* const*>& cores,
                  const double* weights);

Shape make_shape(int d, const int64_t* n, const int64_t* ranks);
// c_k = min(r_k, n_1 ... n_k) (k = 0..d, c_0 = c_d = 1).
std::vector<int64_t> rank_caps(const Shape& s);

// Upper estimate of the device workspace one rounding of this shape uses:
// ell_max > 0 for fixed rank with that sketch size, <= 0 for adaptive.
size_t workspace_bytes(const Shape& s, int64_t ell_max, int prec);
size_t workspace_bytes(const Summands& x, int64_t ell_max, int prec);

void round_fixed(const Summands& x, const int64_t* target, int64_t ell, uint64_t seed,
                 const Options& o, OutCores& y, RoundInfo& info);
void round_adaptive(const Summands& x, double tol, int64_t ell_block, uint64_t seed,
                    const Options& o, OutCores& y, RoundInfo& info);
void round_fixed(const Shape& s, const double* const* cores, const int64_t* target, int64_t ell,
                 uint64_t seed, const Options& o, OutCores& y, RoundInfo& info);
void round_adaptive(const Shape& s, const double* const* cores, double tol, int64_t ell_block,
                    uint64_t seed, const Options& o, OutCores& y, RoundInfo& info);
// Deterministic TT-SVD rounding (Sec. 2.3): tolerance tol, or target ranks
// (host [d+1]) when target is given.
void round_ttsvd(const Shape& s, const double* const* cores, double tol, const int64_t* target,
                 const Options& o, OutCores& y, RoundInfo& info);

// round_fixed with all device memory carved from `region` (region_bytes):
// allocates nothing; the caller serialises calls that share a region.
void round_fixed_in(void* region, size_t region_bytes, const Shape& s, const double* const* cores,
                    const int64_t* target, int64_t ell, uint64_t seed, const Options& o, OutCores& y,
                    RoundInfo& info);

// round_fixed_in on this device's allocation-free scratch array (noalloc.hip).
void round_fixed_noalloc(const Shape& s, const double* const* cores, const int64_t* target,
                         int64_t ell, uint64_t seed, const Options& o, OutCores& y, RoundInfo& info);

void gaussian_factor(uint64_t seed, int mode, int64_t n, int64_t col0, int64_t ncols, double* out,
                     hipStream_t st);
void partial_contractions(const Shape& s, const double* const* cores, uint64_t seed, int64_t col0,
                          int64_t ncols, int t, int prec, double* const* w, hipStream_t st);
void partial_contractions_lr(const Shape& s, const double* const* cores, uint64_t seed, int64_t col0,
                             int64_t ncols, int t, double* const* w, hipStream_t st);
void qr_inplace(double* a, int64_t m, int64_t b, hipStream_t st);
int64_t svd_small(const double* a, int64_t p, int64_t q, double* g, double* v, double* sig,
                  double tau, int64_t target, hipStream_t st);

// Kernel timing: HIP event pairs around launches of each kind (see
// tt_kernel_timing in the C header).
enum { KT_PC = 0, KT_GEMM = 1, KT_QR = 2, KT_SVD = 3, KT_KINDS = 4 };
void timing_enable(unsigned kinds);  // bit k records kind k; 0 stops
void timing_read(int kind, int64_t* launches, double* total_ms);

// RAII: no TimedScope on this thread records anything while it lives.
class TimingPause {
   public:
    TimingPause();
    ~TimingPause();
    TimingPause(const TimingPause&) = delete;
    TimingPause& operator=(const TimingPause&) = delete;

   private:
    bool prev_;
};

// RAII scope: records a start event on construction and a stop event on
// destruction when timing is enabled; no-op otherwise.  `launches` is the
// number of back-to-back launches of the kind that the scope brackets.
class TimedScope {
   public:
    TimedScope(int kind, hipStream_t s, int launches = 1);
    ~TimedScope();
    TimedScope(const TimedScope&) = delete;
    TimedScope& operator=(const TimedScope&) = delete;

   private:
    int kind_;
    hipStream_t s_;
    int launches_;
    hipEvent_t e0_ = nullptr;
};

}  // namespace ttr
