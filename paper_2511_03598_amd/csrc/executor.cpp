// Worker-thread executor for batched and served roundings (see executor.hpp).
#include "executor.hpp"

#include <algorithm>
#include <chrono>

namespace ttr {

// ---------------------------------------------------------------------------
// DevicePool
// ---------------------------------------------------------------------------
size_t DevicePool::round_up(size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
}

void* DevicePool::alloc(size_t bytes, size_t* rounded) {
    const size_t c = round_up(std::max<size_t>(bytes, 1));
    *rounded = c;
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = free_.find(c);
        if (it != free_.end() && !it->second.empty()) {
            void* p = it->second.back();
            it->second.pop_back();
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(-2, "device allocation of " + std::to_string(c) + " bytes failed");
    }
    std::lock_guard<std::mutex> lk(mu_);
    all_.push_back(p);
    return p;
}

void DevicePool::free(void* p, size_t rounded) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_[rounded].push_back(p);
}

DevicePool::~DevicePool() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device_);
    for (void* p : all_) (void)hipFree(p);
    (void)hipSetDevice(cur);
}

// ---------------------------------------------------------------------------
// Executor
// ---------------------------------------------------------------------------
double Executor::now() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

Executor::Executor(int device, int workers, size_t budget)
    : device_(device), budget_(budget), pool_(device) {
    workers = std::max(1, std::min(workers, 64));
    for (int i = 0; i < workers; ++i) threads_.emplace_back(&Executor::worker_main, this, i);
}

Executor::~Executor() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
        // queued jobs never start
        for (auto& j : queue_) {
            j->status = -4;
            j->error = "executor shut down before the job started";
            j->t_done = now();
            j->state.store(2);
        }
        queue_.clear();
    }
    cv_work_.notify_all();
    for (auto& t : threads_) t.join();
    cv_done_.notify_all();
}

void Executor::submit(const std::shared_ptr<Job>& j) {
    if (j->footprint > budget_)
        throw Error(-3, "request needs " + std::to_string(j->footprint) +
                            " bytes of device memory, budget is " + std::to_string(budget_));
    j->t_submit = now();
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) throw Error(-4, "executor is shutting down");
        queue_.push_back(j);
    }
    cv_work_.notify_all();
}

// First queued job that fits, unless the head has already been passed over
// four times (then only the head may start).  Caller holds mu_.
bool Executor::admissible_locked(std::shared_ptr<Job>* out) {
    if (queue_.empty()) return false;
    const size_t avail = budget_ > in_use_ ? budget_ - in_use_ : 0;
    auto& head = queue_.front();
    if (head->footprint <= avail) {
        *out = head;
        queue_.pop_front();
        return true;
    }
    if (head->bypassed >= 4) return false;
    for (size_t i = 1; i < queue_.size(); ++i) {
        if (queue_[i]->footprint <= avail) {
            *out = queue_[i];
            queue_.erase(queue_.begin() + (long)i);
            head->bypassed += 1;
            return true;
        }
    }
    return false;
}

void Executor::worker_main(int idx) {
    (void)idx;
    if (hipSetDevice(device_) != hipSuccess) return;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    for (;;) {
        std::shared_ptr<Job> j;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_work_.wait(lk, [&] { return stop_ || admissible_locked(&j); });
            if (!j) break;  // stop_ with nothing admitted
            in_use_ += j->footprint;
        }
        j->t_start = now();
        j->state.store(1);
        run(*j, st);
        j->t_done = now();
        {
            std::lock_guard<std::mutex> lk(mu_);
            // the running footprint is returned; an owned result keeps its
            // exact-size buffers (`held`) until release
            in_use_ -= j->footprint;
            if (j->status == 0 && j->owned_output) in_use_ += j->held;
            j->state.store(2);
        }
        cv_work_.notify_all();
        cv_done_.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
}

void Executor::release_result(Job& j) {
    if (!j.owned_output) return;
    for (size_t k = 0; k < j.out_cores.size(); ++k) {
        if (j.out_cores[k]) pool_.free(j.out_cores[k], j.out_rounded[k]);
        j.out_cores[k] = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (j.status == 0) in_use_ -= j.held;
        j.held = 0;
    }
    cv_work_.notify_all();
}

void Executor::run(Job& j, hipStream_t st) {
    const int d = j.shape.d;
    std::vector<double*> cap_bufs;
    std::vector<size_t> cap_rounded;
    try {
        Options o = j.opts;
        o.stream = st;
        OutCores oc;
        if (j.owned_output) {
            // capacity-sized staging from the pool, then exact-size results
            cap_bufs.assign(d, nullptr);
            cap_rounded.assign(d, 0);
            for (int k = 0; k < d; ++k)
                cap_bufs[k] = static_cast<double*>(pool_.alloc((size_t)j.out_cap[k] * 8, &cap_rounded[k]));
            oc.cores = cap_bufs.data();
        } else {
            oc.cores = j.out_cores.data();
        }
        oc.cap = j.out_cap.data();
        j.out_ranks.assign(d + 1, 1);
        oc.ranks = j.out_ranks.data();
        if (j.kind == Job::ADAPTIVE)
            round_adaptive(j.shape, j.cores.data(), j.tol, j.ell_block, j.seed, o, oc, j.info);
        else
            round_fixed(j.shape, j.cores.data(), j.target.empty() ? nullptr : j.target.data(), j.ell,
                        j.seed, o, oc, j.info);
        j.orth = oc.orth;
        if (j.owned_output) {
            j.out_cores.assign(d, nullptr);
            j.out_rounded.assign(d, 0);
            j.held = 0;
            for (int k = 0; k < d; ++k) {
                const size_t bytes = (size_t)j.out_ranks[k] * j.shape.n[k] * j.out_ranks[k + 1] * 8;
                j.out_cores[k] = static_cast<double*>(pool_.alloc(bytes, &j.out_rounded[k]));
                j.held += j.out_rounded[k];
                TTR_HIP(hipMemcpyAsync(j.out_cores[k], cap_bufs[k], bytes, hipMemcpyDeviceToDevice, st));
            }
            TTR_HIP(hipStreamSynchronize(st));
        }
        j.status = 0;
    } catch (const Error& e) {
        j.status = e.code;
        j.error = e.what();
    } catch (const std::exception& e) {
        j.status = -4;
        j.error = e.what();
    }
    // On an error kernels may still be queued that write the staging or
    // result buffers: drain the stream before they return to the pool, where
    // a rounding on another worker's stream could take them.
    if (j.status != 0) {
        (void)hipStreamSynchronize(st);
        (void)hipGetLastError();
    }
    for (size_t k = 0; k < cap_bufs.size(); ++k) pool_.free(cap_bufs[k], cap_rounded[k]);
    if (j.status != 0 && j.owned_output) {
        for (size_t k = 0; k < j.out_cores.size(); ++k)
            if (j.out_cores[k]) pool_.free(j.out_cores[k], j.out_rounded[k]);
        j.out_cores.clear();
        j.held = 0;
    }
}

void Executor::wait_all(const std::vector<std::shared_ptr<Job>>& jobs) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] {
        for (auto& j : jobs)
            if (j->state.load() != 2) return false;
        return true;
    });
}

Executor& default_executor() {
    static std::mutex mu;
    static Executor* ex = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!ex) {
        int dev = 0;
        TTR_HIP(hipGetDevice(&dev));
        size_t free_b = 0, total_b = 0;
        TTR_HIP(hipMemGetInfo(&free_b, &total_b));
        ex = new Executor(dev, 8, free_b / 10 * 8);  // kept until process exit
    }
    return *ex;
}

}  // namespace ttr
