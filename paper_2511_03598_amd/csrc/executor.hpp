// Many roundings at once: worker threads, each with its own HIP stream (and,
// through the runtime's pool, its own workspace), take jobs from a FIFO
// queue.  A job is admitted when a worker is free and its device-memory
// footprint fits the budget next to the jobs already running and the
// results not yet released; a queued job that fits may pass one that does
// not, at most a few times (then the head waits).  Admission happens
// whenever a job finishes or a result is released, so new requests start
// while others are still on the device and their kernels overlap there.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "runtime.hpp"

namespace ttr {

// Caching pool of device buffers (power-of-two size classes); buffers
// return to the pool on free and are released to HIP when the pool dies.
class DevicePool {
   public:
    explicit DevicePool(int device) : device_(device) {}
    ~DevicePool();
    void* alloc(size_t bytes, size_t* rounded);
    void free(void* p, size_t rounded);
    static size_t round_up(size_t bytes);

   private:
    int device_;
    std::mutex mu_;
    std::map<size_t, std::vector<void*>> free_;
    std::vector<void*> all_;
};

struct Job {
    enum Kind { ADAPTIVE = 0, FIXED = 1 };
    int kind = ADAPTIVE;
    Shape shape;
    std::vector<const double*> cores;  // borrowed device pointers
    double tol = 0;
    int64_t ell_block = 0, ell = 0;
    std::vector<int64_t> target;  // fixed rank, may be empty
    uint64_t seed = 0;
    Options opts;
    // Output: caller buffers (batch) or, when owned, pool buffers sized to
    // the result and handed over in the result.
    bool owned_output = false;
    std::vector<double*> out_cores;
    std::vector<int64_t> out_cap;
    std::vector<int64_t> out_ranks;
    std::vector<size_t> out_rounded;  // pool size classes of owned outputs
    int orth = 0;
    size_t footprint = 0;     // bytes reserved while running (workspace,
                              // capacity staging and result, upper bounds)
    size_t held = 0;          // bytes an owned result keeps until release
    int bypassed = 0;
    // completion
    int status = 0;
    std::string error;
    RoundInfo info;
    double t_submit = 0, t_start = 0, t_done = 0;
    std::atomic<int> state{0};  // 0 queued, 1 running, 2 done
};

class Executor {
   public:
    Executor(int device, int workers, size_t budget);
    ~Executor();
    // Enqueue; throws Error(-3) if the job can never fit the budget.
    void submit(const std::shared_ptr<Job>& j);
    // Block until every job in the list is done.
    void wait_all(const std::vector<std::shared_ptr<Job>>& jobs);
    // Give back the bytes an owned result holds (its buffers return to the pool).
    void release_result(Job& j);
    size_t budget() const { return budget_; }
    int device() const { return device_; }
    static double now();

   private:
    void worker_main(int idx);
    bool admissible_locked(std::shared_ptr<Job>* out);
    void run(Job& j, hipStream_t st);

    int device_;
    size_t budget_;
    size_t in_use_ = 0;
    bool stop_ = false;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<std::shared_ptr<Job>> queue_;
    std::vector<std::thread> threads_;
    DevicePool pool_;
};

// Process-wide executor for the batch entry point (created on first use on
// the current device).
Executor& default_executor();

}  // namespace ttr
