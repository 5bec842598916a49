// Host planning of the persistent batched adaptive rounding (batch.hip).
#pragma once

#include <string>
#include <vector>

#include "batch.hpp"
#include "runtime.hpp"

namespace ttr {

// Workspace bytes of a batch (descriptors, barriers and every tensor's
// sketch, basis, cores, partial slots), with the same checks as
// BatchPlan::create.
// team_flops <= 0: batch_team_flops().
size_t batch_workspace_bytes(const std::vector<Shape>& sh, int64_t ell_block, double f_init,
                             double team_flops = 0.0);
// Work (flops of the rounding model) per team member: a tensor gets the
// largest power-of-two team T with 2T times this below its work estimate,
// capped by batch_team_cap().  The value is the current device's tuned one
// (set_batch_team_flops, tt_batch_autotune), else the entry for this
// device in the file named by TTR_BATCH_TUNE_CACHE, else
// TTR_BATCH_TEAM_FLOPS, else 3e9.  It depends on the device only, never on
// the batch, so a tensor's team (and its result bits) is the same alone or
// in any batch once the value is fixed.
double batch_team_flops();
// Set the current device's value (> 0), or clear it (<= 0: the cache file
// is consulted again on the next use).
void set_batch_team_flops(double v);
// Append "key value" for the current device to the TTR_BATCH_TUNE_CACHE
// file (no-op when the variable is unset).
void save_batch_team_flops(double v);
// "gcnArchName/compute units" of the current device: the cache file's key.
std::string batch_device_key();
int batch_team_cap();

// A batch laid out in a caller's workspace: create() validates, carves the
// workspace and uploads the descriptors (synchronising opts.stream);
// launch() enqueues the counter reset and the persistent kernel only (no
// allocation, no host synchronisation: it may be captured in a graph and
// replayed); results() synchronises the stream and reads ranks, run
// records and statuses.
struct BatchPlan {
    int count = 0, grid = 1;
    std::vector<int> order, prefix, team;
    BatchTT* d_tts = nullptr;
    int* d_order = nullptr;
    int* d_prefix = nullptr;
    unsigned* d_zero = nullptr;
    int64_t zwords = 0;
    size_t bytes_used = 0;
    std::vector<int64_t*> ranks_dev;
    std::vector<double*> info_dev;
    std::vector<int> d_of;

    void create(const std::vector<Shape>& sh, const std::vector<const double* const*>& cores,
                const std::vector<double>& tol, int64_t ell_block, const std::vector<uint64_t>& seeds,
                const Options& o, const std::vector<OutCores>& outs, void* ws, size_t ws_bytes,
                double team_flops = 0.0);
    void launch(hipStream_t st) const;
    void results(hipStream_t st, std::vector<std::vector<int64_t>>& ranks, std::vector<std::vector<double>>& info,
                 std::vector<int>& status) const;
    // Partial contractions of tensor i by its run record's pass log (Sec. 3.1
    // cost model): one float64 read of each contracted core and one write of
    // its W columns per pass, 2 r_{k-1} n_k r_k l + 2 r_{k-1} r_k l flops per
    // core; `cores` counts the contracted cores over all passes.
    void pc_work(int i, const std::vector<double>& info, int64_t& cores, double& bytes, double& flops) const;
    std::vector<Shape> shapes;
};

}  // namespace ttr
