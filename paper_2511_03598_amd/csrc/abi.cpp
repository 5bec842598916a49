// extern "C" boundary of libttround (declared in include/ttround.h): argument
// validation, status codes and the thread-local error message.  No C++
// exception crosses this layer.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "../../include/ttround.h"
#include "batch_host.hpp"
#include "executor.hpp"
#include "runtime.hpp"

namespace {

thread_local std::string g_err;
thread_local tt_info g_info{};

tt_status fail(int code, const std::string& msg) {
    g_err = msg;
    return (tt_status)code;
}

template <typename F>
tt_status guarded(F&& f) {
    try {
        f();
        g_err.clear();
        return TT_OK;
    } catch (const ttr::Error& e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(TT_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(TT_EDEVICE, e.what());
    } catch (...) {
        return fail(TT_EDEVICE, "unknown error");
    }
}

ttr::Shape view_shape(const tt_view* x) {
    if (!x) throw ttr::Error(TT_EINVAL, "null tt_view");
    if (!x->cores) throw ttr::Error(TT_EINVAL, "null core array");
    ttr::Shape s = ttr::make_shape(x->d, x->n, x->ranks);
    for (int k = 0; k < x->d; ++k)
        if (!x->cores[k]) throw ttr::Error(TT_EINVAL, "null core pointer");
    return s;
}

ttr::Options make_opts(const tt_opts* o) {
    ttr::Options r;
    if (o) {
        if (o->prec != TT_PREC_F64 && o->prec != TT_PREC_F32 && o->prec != TT_PREC_BF16)
            throw ttr::Error(TT_EINVAL, "unknown precision");
        r.prec = (int)o->prec;
        r.f_init = o->f_init;
        if (o->f_init > 0.0 && !(o->f_init < 1.0))
            throw ttr::Error(TT_EINVAL, "f_init must be in (0, 1)");
        r.nrmx = o->nrmx;
        r.recompress = o->recompress;
        r.stream = (hipStream_t)o->stream;
    }
    return r;
}

ttr::OutCores out_of(const tt_out* y, int d) {
    if (!y || !y->cores || !y->ranks || !y->capacity)
        throw ttr::Error(TT_EINVAL, "null tt_out field");
    if (y->d != d) throw ttr::Error(TT_EINVAL, "tt_out.d differs from the input's d");
    for (int k = 0; k < d; ++k)
        if (!y->cores[k]) throw ttr::Error(TT_EINVAL, "null output core pointer");
    ttr::OutCores o;
    o.cores = y->cores;
    o.cap = y->capacity;
    o.ranks = y->ranks;
    return o;
}

void store_info(const ttr::RoundInfo& i) {
    g_info.tau = i.tau;
    g_info.nrmx = i.nrmx;
    g_info.min_margin = i.min_margin;
    g_info.passes = i.passes;
    g_info.iterations = i.iterations;
    g_info.qr_retries = i.qr_retries;
    g_info.pc_launches = i.pc_launches;
    g_info.pc_bytes = i.pc_bytes;
    g_info.pc_flops = i.pc_flops;
}


void fill_info(tt_info& o, const ttr::RoundInfo& i) {
    o.tau = i.tau;
    o.nrmx = i.nrmx;
    o.min_margin = i.min_margin;
    o.passes = i.passes;
    o.iterations = i.iterations;
    o.qr_retries = i.qr_retries;
    o.pc_launches = i.pc_launches;
    o.pc_bytes = i.pc_bytes;
    o.pc_flops = i.pc_flops;
}

int64_t out_capacity_total(const ttr::Shape& s, std::vector<int64_t>* per_core) {
    std::vector<int64_t> c = ttr::rank_caps(s);
    int64_t tot = 0;
    per_core->assign(s.d, 0);
    for (int k = 1; k <= s.d; ++k) {
        (*per_core)[k - 1] = c[k - 1] * s.n[k - 1] * c[k];
        tot += (*per_core)[k - 1];
    }
    return tot;
}

}  // namespace

struct tt_server {
    std::unique_ptr<ttr::Executor> ex;
    std::mutex mu;
    std::map<uint64_t, std::shared_ptr<ttr::Job>> jobs;
    uint64_t next = 1;
};

namespace {

struct ResultImpl {
    tt_result pub;  // first member: tt_result* <-> ResultImpl*
    std::shared_ptr<ttr::Job> job;
    tt_server* server;
    std::string err;
};

tt_result* make_result(tt_server* s, const std::shared_ptr<ttr::Job>& j) {
    ResultImpl* r = new ResultImpl();
    r->job = j;
    r->server = s;
    r->err = j->error;
    tt_result& p = r->pub;
    p.status = (tt_status)j->status;
    p.error = r->err.c_str();
    p.d = j->shape.d;
    p.ranks = j->out_ranks.data();
    p.cores = j->out_cores.data();
    p.orth = j->orth;
    fill_info(p.info, j->info);
    p.submit_s = j->t_submit;
    p.start_s = j->t_start;
    p.done_s = j->t_done;
    return &r->pub;
}

std::shared_ptr<ttr::Job> job_from_view(const tt_view* x, int prec) {
    auto j = std::make_shared<ttr::Job>();
    j->shape = view_shape(x);
    j->cores.assign(x->cores, x->cores + x->d);
    (void)prec;
    return j;
}
}  // namespace

extern "C" {

tt_status tt_out_capacity(const tt_view* x, const int64_t* target_ranks, int64_t* cap) {
    (void)target_ranks;
    return guarded([&] {
        if (!cap) throw ttr::Error(TT_EINVAL, "null cap");
        if (!x) throw ttr::Error(TT_EINVAL, "null tt_view");
        ttr::Shape s = ttr::make_shape(x->d, x->n, x->ranks);
        std::vector<int64_t> c = ttr::rank_caps(s);
        for (int k = 1; k <= s.d; ++k) cap[k - 1] = c[k - 1] * s.n[k - 1] * c[k];
    });
}

tt_status tt_round_fixed(const tt_view* x, const int64_t* target_ranks, int64_t ell, uint64_t seed,
                         const tt_opts* opts, tt_out* y) {
    return guarded([&] {
        ttr::Shape s = view_shape(x);
        ttr::Options o = make_opts(opts);
        if (ell < 1) throw ttr::Error(TT_EINVAL, "ell must be >= 1");
        if (target_ranks) {
            if (target_ranks[0] != 1 || target_ranks[s.d] != 1)
                throw ttr::Error(TT_EINVAL, "target_ranks[0] and [d] must be 1");
            for (int k = 1; k < s.d; ++k)
                if (target_ranks[k] < 1) throw ttr::Error(TT_EINVAL, "target ranks must be >= 1");
        }
        ttr::OutCores oc = out_of(y, s.d);
        ttr::RoundInfo info;
        ttr::round_fixed(s, x->cores, target_ranks, ell, seed, o, oc, info);
        y->orth = oc.orth;
        store_info(info);
    });
}

tt_status tt_round_fixed_noalloc(const tt_view* x, const int64_t* target_ranks, int64_t ell,
                                 uint64_t seed, const tt_opts* opts, tt_out* y) {
    return guarded([&] {
        ttr::Shape s = view_shape(x);
        ttr::Options o = make_opts(opts);
        if (ell < 1) throw ttr::Error(TT_EINVAL, "ell must be >= 1");
        if (target_ranks) {
            if (target_ranks[0] != 1 || target_ranks[s.d] != 1)
                throw ttr::Error(TT_EINVAL, "target_ranks[0] and [d] must be 1");
            for (int k = 1; k < s.d; ++k)
                if (target_ranks[k] < 1) throw ttr::Error(TT_EINVAL, "target ranks must be >= 1");
        }
        ttr::OutCores oc = out_of(y, s.d);
        ttr::RoundInfo info;
        ttr::round_fixed_noalloc(s, x->cores, target_ranks, ell, seed, o, oc, info);
        y->orth = oc.orth;
        store_info(info);
    });
}

namespace {
ttr::Summands sum_of(const tt_view* xs, int32_t count, const double* weights) {
    if (!xs) throw ttr::Error(TT_EINVAL, "null tt_view array");
    if (count < 1) throw ttr::Error(TT_EINVAL, "count must be >= 1");
    std::vector<ttr::Shape> sh;
    std::vector<const double* const*> cores;
    for (int32_t i = 0; i < count; ++i) {
        sh.push_back(view_shape(&xs[i]));
        cores.push_back(xs[i].cores);
    }
    if (weights)
        for (int32_t i = 0; i < count; ++i)
            if (!std::isfinite(weights[i])) throw ttr::Error(TT_EINVAL, "weights must be finite");
    return ttr::make_sum(sh, cores, weights);
}
}  // namespace

tt_status tt_sum_out_capacity(const tt_view* xs, int32_t count, const int64_t* target_ranks,
                              int64_t* cap) {
    (void)target_ranks;
    return guarded([&] {
        if (!cap) throw ttr::Error(TT_EINVAL, "null cap");
        if (!xs) throw ttr::Error(TT_EINVAL, "null tt_view array");
        if (count < 1) throw ttr::Error(TT_EINVAL, "count must be >= 1");
        std::vector<ttr::Shape> sh;
        std::vector<const double* const*> cores;
        for (int32_t i = 0; i < count; ++i) {
            sh.push_back(ttr::make_shape(xs[i].d, xs[i].n, xs[i].ranks));
            cores.push_back(nullptr);
        }
        const ttr::Summands x = ttr::make_sum(sh, cores, nullptr);
        std::vector<int64_t> c = ttr::rank_caps(x.fs);
        for (int k = 1; k <= x.fs.d; ++k) cap[k - 1] = c[k - 1] * x.fs.n[k - 1] * c[k];
    });
}

tt_status tt_round_sum_fixed(const tt_view* xs, int32_t count, const double* weights,
                             const int64_t* target_ranks, int64_t ell, uint64_t seed,
                             const tt_opts* opts, tt_out* y) {
    return guarded([&] {
        const ttr::Summands x = sum_of(xs, count, weights);
        ttr::Options o = make_opts(opts);
        if (ell < 1) throw ttr::Error(TT_EINVAL, "ell must be >= 1");
        const int d = x.fs.d;
        if (target_ranks) {
            if (target_ranks[0] != 1 || target_ranks[d] != 1)
                throw ttr::Error(TT_EINVAL, "target_ranks[0] and [d] must be 1");
            for (int k = 1; k < d; ++k)
                if (target_ranks[k] < 1) throw ttr::Error(TT_EINVAL, "target ranks must be >= 1");
        }
        ttr::OutCores oc = out_of(y, d);
        ttr::RoundInfo info;
        ttr::round_fixed(x, target_ranks, ell, seed, o, oc, info);
        y->orth = oc.orth;
        store_info(info);
    });
}

tt_status tt_round_sum_adaptive(const tt_view* xs, int32_t count, const double* weights,
                                double tol, int64_t ell_block, uint64_t seed, const tt_opts* opts,
                                tt_out* y) {
    return guarded([&] {
        const ttr::Summands x = sum_of(xs, count, weights);
        ttr::Options o = make_opts(opts);
        if (!(tol > 0.0)) throw ttr::Error(TT_EINVAL, "tol must be > 0");
        ttr::OutCores oc = out_of(y, x.fs.d);
        ttr::RoundInfo info;
        ttr::round_adaptive(x, tol, ell_block, seed, o, oc, info);
        y->orth = oc.orth;
        store_info(info);
    });
}

tt_status tt_round_adaptive(const tt_view* x, double tol, int64_t ell_block, uint64_t seed,
                            const tt_opts* opts, tt_out* y) {
    return guarded([&] {
        ttr::Shape s = view_shape(x);
        ttr::Options o = make_opts(opts);
        if (!(tol > 0.0)) throw ttr::Error(TT_EINVAL, "tol must be > 0");
        ttr::OutCores oc = out_of(y, s.d);
        ttr::RoundInfo info;
        ttr::round_adaptive(s, x->cores, tol, ell_block, seed, o, oc, info);
        y->orth = oc.orth;
        store_info(info);
    });
}

tt_status tt_round_ttsvd(const tt_view* x, double tol, const int64_t* target_ranks, const tt_opts* opts,
                         tt_out* y) {
    return guarded([&] {
        ttr::Shape s = view_shape(x);
        ttr::Options o = make_opts(opts);
        if (!target_ranks && !(tol > 0.0)) throw ttr::Error(TT_EINVAL, "tol must be > 0");
        if (target_ranks)
            for (int k = 1; k < s.d; ++k)
                if (target_ranks[k] < 1) throw ttr::Error(TT_EINVAL, "target ranks must be >= 1");
        ttr::OutCores oc = out_of(y, s.d);
        ttr::RoundInfo info;
        ttr::round_ttsvd(s, x->cores, tol, target_ranks, o, oc, info);
        y->orth = oc.orth;
        store_info(info);
    });
}

tt_status tt_last_info(tt_info* info) {
    if (!info) return fail(TT_EINVAL, "null info");
    *info = g_info;
    return TT_OK;
}

const char* tt_last_error(void) { return g_err.c_str(); }

tt_status tt_gaussian_factor(uint64_t seed, int32_t mode, int64_t n, int64_t col0, int64_t ncols,
                             double* out, void* stream) {
    return guarded([&] {
        ttr::gaussian_factor(seed, mode, n, col0, ncols, out, (hipStream_t)stream);
    });
}

tt_status tt_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                           void* stream) {
    return guarded([&] {
        if (!ctr || !key || !out || count < 0) throw ttr::Error(TT_EINVAL, "bad Philox arguments");
        ttr::launch_philox(ctr, key, out, count, (hipStream_t)stream);
        TTR_HIP(hipStreamSynchronize((hipStream_t)stream));
    });
}

tt_status tt_partial_contractions(const tt_view* x, uint64_t seed, int64_t col0, int64_t ncols,
                                  int32_t t, tt_prec prec, double* const* w, void* stream) {
    return guarded([&] {
        ttr::Shape s = view_shape(x);
        if (!w) throw ttr::Error(TT_EINVAL, "null W array");
        for (int k = t; k <= s.d; ++k)
            if (t >= 2 && !w[k - t]) throw ttr::Error(TT_EINVAL, "null W pointer");
        ttr::partial_contractions(s, x->cores, seed, col0, ncols, t, (int)prec, w,
                                  (hipStream_t)stream);
    });
}

tt_status tt_partial_contractions_lr(const tt_view* x, uint64_t seed, int64_t col0, int64_t ncols,
                                     int32_t t, double* const* w, void* stream) {
    return guarded([&] {
        ttr::Shape s = view_shape(x);
        if (!w) throw ttr::Error(TT_EINVAL, "null W array");
        if (t < 1 || t > s.d) throw ttr::Error(TT_EINVAL, "t must be in [1, d]");
        for (int k = 1; k <= t; ++k)
            if (!w[k - 1]) throw ttr::Error(TT_EINVAL, "null W pointer");
        ttr::partial_contractions_lr(s, x->cores, seed, col0, ncols, t, w, (hipStream_t)stream);
    });
}

tt_status tt_qr(double* a, int64_t m, int64_t b, void* stream) {
    return guarded([&] { ttr::qr_inplace(a, m, b, (hipStream_t)stream); });
}

tt_status tt_svd_small(const double* a, int64_t p, int64_t q, double* g, double* v, double* sig,
                       double tau, int64_t target, int64_t* t_out, void* stream) {
    return guarded([&] {
        if (!t_out) throw ttr::Error(TT_EINVAL, "null t_out");
        *t_out = ttr::svd_small(a, p, q, g, v, sig, tau, target, (hipStream_t)stream);
    });
}

tt_status tt_kernel_timing(int32_t kinds) {
    return guarded([&] {
        if (kinds < 0 || kinds > TT_KERNEL_TIMING_ALL) throw ttr::Error(TT_EINVAL, "unknown kernel kinds");
        ttr::timing_enable((unsigned)kinds);
    });
}

tt_status tt_kernel_timing_read(int32_t kind, int64_t* launches, double* total_ms) {
    return guarded([&] {
        if (!launches || !total_ms) throw ttr::Error(TT_EINVAL, "null output");
        if (kind < 0 || kind >= TT_KERNEL_KINDS) throw ttr::Error(TT_EINVAL, "unknown kernel kind");
        ttr::timing_read(kind, launches, total_ms);
    });
}


tt_status tt_workspace_bytes(const tt_view* x, int64_t ell_max, tt_prec prec, size_t* bytes) {
    return guarded([&] {
        if (!bytes) throw ttr::Error(TT_EINVAL, "null bytes");
        if (!x) throw ttr::Error(TT_EINVAL, "null tt_view");
        if (prec != TT_PREC_F64 && prec != TT_PREC_F32 && prec != TT_PREC_BF16)
            throw ttr::Error(TT_EINVAL, "unknown precision");
        ttr::Shape s = ttr::make_shape(x->d, x->n, x->ranks);
        *bytes = ttr::workspace_bytes(s, ell_max, (int)prec);
    });
}

}  // extern "C"

struct tt_batch {
    ttr::BatchPlan plan;
    std::vector<tt_out> ys;  // the caller's output descriptors (ranks written by finish)
    std::vector<std::vector<double>> info;
    int device = 0;
};

namespace {

struct BatchArgs {
    std::vector<ttr::Shape> sh;
    std::vector<const double* const*> cores;
    std::vector<double> tol;
    std::vector<uint64_t> seeds;
    std::vector<ttr::OutCores> outs;
};

BatchArgs batch_args(const tt_view* xs, int32_t count, const double* tol, const uint64_t* seeds, tt_out* ys) {
    if (count < 1) throw ttr::Error(TT_EINVAL, "count must be >= 1");
    if (!xs || !tol || !seeds || !ys) throw ttr::Error(TT_EINVAL, "null batch array");
    BatchArgs a;
    for (int32_t i = 0; i < count; ++i) {
        if (!(tol[i] > 0.0)) throw ttr::Error(TT_EINVAL, "tol[" + std::to_string(i) + "] must be > 0");
        a.sh.push_back(view_shape(&xs[i]));
        a.cores.push_back(xs[i].cores);
        a.tol.push_back(tol[i]);
        a.seeds.push_back(seeds[i]);
        a.outs.push_back(out_of(&ys[i], xs[i].d));
    }
    return a;
}

// Read back ranks, run records and statuses of a launched batch into the
// caller's tt_out descriptors.
void batch_finish_impl(tt_batch* b, hipStream_t st) {
    std::vector<std::vector<int64_t>> ranks;
    std::vector<int> status;
    b->plan.results(st, ranks, b->info, status);
    int bad = -1;
    for (int i = 0; i < b->plan.count; ++i) {
        if (status[i] != 0 && bad < 0) bad = i;
        for (size_t k = 0; k < ranks[i].size(); ++k) b->ys[i].ranks[k] = ranks[i][k];
        b->ys[i].orth = 1;
    }
    if (bad >= 0)
        throw ttr::Error(TT_EDEVICE, "tensor " + std::to_string(bad) + ": a team barrier of the batched rounding timed out");
}

void fill_batch_info(tt_info& o, const ttr::BatchPlan& plan, int i, const std::vector<double>& v) {
    o = tt_info{};
    o.tau = v[0];
    o.nrmx = v[1];
    o.iterations = (int32_t)v[2];
    o.passes = (int32_t)v[3];
    o.min_margin = v[7];
    o.qr_retries = 0;
    plan.pc_work(i, v, o.pc_launches, o.pc_bytes, o.pc_flops);
}

// Library-owned workspace of the synchronous batch call, per device, kept
// and grown as needed.
struct BatchCache {
    std::mutex mu;
    void* p = nullptr;
    size_t cap = 0;
};
BatchCache g_batch_cache[64];

}  // namespace

extern "C" {

tt_status tt_batch_workspace_bytes(const tt_view* xs, int32_t count, int64_t ell_block, const tt_opts* opts,
                                   size_t* bytes) {
    return guarded([&] {
        if (!bytes) throw ttr::Error(TT_EINVAL, "null bytes");
        if (!xs || count < 1) throw ttr::Error(TT_EINVAL, "bad batch");
        ttr::Options o = make_opts(opts);
        std::vector<ttr::Shape> sh;
        for (int32_t i = 0; i < count; ++i) sh.push_back(ttr::make_shape(xs[i].d, xs[i].n, xs[i].ranks));
        *bytes = ttr::batch_workspace_bytes(sh, ell_block, o.f_init > 0.0 ? o.f_init : 0.1);
    });
}

tt_status tt_batch_create(const tt_view* xs, int32_t count, const double* tol, int64_t ell_block,
                          const uint64_t* seeds, const tt_opts* opts, tt_out* ys, void* workspace,
                          size_t workspace_bytes, tt_batch** out) {
    return guarded([&] {
        if (!out) throw ttr::Error(TT_EINVAL, "null out");
        *out = nullptr;
        ttr::Options o = make_opts(opts);
        BatchArgs a = batch_args(xs, count, tol, seeds, ys);
        std::unique_ptr<tt_batch> b(new tt_batch());
        TTR_HIP(hipGetDevice(&b->device));
        b->plan.create(a.sh, a.cores, a.tol, ell_block, a.seeds, o, a.outs, workspace, workspace_bytes);
        b->ys.assign(ys, ys + count);
        *out = b.release();
    });
}

tt_status tt_batch_launch(const tt_batch* b, void* stream) {
    return guarded([&] {
        if (!b) throw ttr::Error(TT_EINVAL, "null batch");
        b->plan.launch((hipStream_t)stream);
    });
}

tt_status tt_batch_finish(tt_batch* b, void* stream) {
    return guarded([&] {
        if (!b) throw ttr::Error(TT_EINVAL, "null batch");
        batch_finish_impl(b, (hipStream_t)stream);
    });
}

tt_status tt_batch_info(const tt_batch* b, int32_t i, tt_info* info) {
    return guarded([&] {
        if (!b || !info) throw ttr::Error(TT_EINVAL, "null argument");
        if (i < 0 || i >= b->plan.count) throw ttr::Error(TT_EINVAL, "tensor index out of range");
        if (b->info.empty()) throw ttr::Error(TT_EINVAL, "tt_batch_finish has not run");
        fill_batch_info(*info, b->plan, i, b->info[i]);
    });
}

tt_status tt_batch_team(const tt_batch* b, int32_t i, int32_t* team) {
    return guarded([&] {
        if (!b || !team) throw ttr::Error(TT_EINVAL, "null argument");
        if (i < 0 || i >= b->plan.count) throw ttr::Error(TT_EINVAL, "tensor index out of range");
        *team = b->plan.team[i];
    });
}

tt_status tt_batch_record(const tt_batch* b, int32_t i, double* out, int32_t cap, int32_t* n) {
    return guarded([&] {
        if (!b || !out || !n) throw ttr::Error(TT_EINVAL, "null argument");
        if (i < 0 || i >= b->plan.count) throw ttr::Error(TT_EINVAL, "tensor index out of range");
        if (b->info.empty()) throw ttr::Error(TT_EINVAL, "tt_batch_finish has not run");
        const int k = std::min<int>(cap, (int)b->info[i].size());
        for (int j = 0; j < k; ++j) out[j] = b->info[i][j];
        *n = k;
    });
}

void tt_batch_destroy(tt_batch* b) { delete b; }

tt_status tt_batch_autotune(const tt_view* xs, int32_t count, const double* tol, int64_t ell_block,
                            const uint64_t* seeds, const tt_opts* opts, tt_out* ys, const double* candidates,
                            int32_t ncand, double* times_ms, double* best) {
    return guarded([&] {
        if (!candidates || !times_ms || !best) throw ttr::Error(TT_EINVAL, "null autotune array");
        if (ncand < 1 || ncand > 64) throw ttr::Error(TT_EINVAL, "ncand must be in [1, 64]");
        for (int j = 0; j < ncand; ++j)
            if (!(candidates[j] > 0.0)) throw ttr::Error(TT_EINVAL, "candidates must be > 0");
        BatchArgs a = batch_args(xs, count, tol, seeds, ys);
        ttr::Options o = make_opts(opts);
        const double f_init = o.f_init > 0.0 ? o.f_init : 0.1;
        hipStream_t st = o.stream;
        size_t need = 0;
        for (int j = 0; j < ncand; ++j)
            need = std::max(need, ttr::batch_workspace_bytes(a.sh, ell_block, f_init, candidates[j]));
        // tuning is a set-up step: its scratch is allocated here and freed
        // before returning
        struct Scratch {
            void* p = nullptr;
            hipEvent_t e[2] = {nullptr, nullptr};
            hipStream_t st = nullptr;
            ~Scratch() {
                if (st) (void)hipStreamSynchronize(st);
                if (p) (void)hipFree(p);
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } sc;
        sc.st = st;
        if (hipMalloc(&sc.p, need) != hipSuccess) {
            (void)hipGetLastError();
            sc.p = nullptr;
            throw ttr::Error(TT_ENOMEM, "autotune workspace allocation of " + std::to_string(need) + " bytes failed");
        }
        TTR_HIP(hipEventCreate(&sc.e[0]));
        TTR_HIP(hipEventCreate(&sc.e[1]));
        double best_ms = 0.0;
        int bj = -1;
        for (int j = 0; j < ncand; ++j) {
            tt_batch b;
            TTR_HIP(hipGetDevice(&b.device));
            b.plan.create(a.sh, a.cores, a.tol, ell_block, a.seeds, o, a.outs, sc.p, need, candidates[j]);
            b.ys.assign(ys, ys + count);
            if (j == 0) {  // untimed first launch
                b.plan.launch(st);
                batch_finish_impl(&b, st);
            }
            // the median of three launches: one launch can land on either
            // side of a close pair of candidates
            float rep[3];
            for (float& ms : rep) {
                TTR_HIP(hipEventRecord(sc.e[0], st));
                b.plan.launch(st);
                TTR_HIP(hipEventRecord(sc.e[1], st));
                batch_finish_impl(&b, st);
                TTR_HIP(hipEventElapsedTime(&ms, sc.e[0], sc.e[1]));
            }
            std::sort(rep, rep + 3);
            const double ms = rep[1];
            times_ms[j] = ms;
            if (bj < 0 || ms < best_ms) {
                best_ms = ms;
                bj = j;
            }
        }
        *best = candidates[bj];
        ttr::set_batch_team_flops(*best);
        ttr::save_batch_team_flops(*best);
    });
}

tt_status tt_batch_team_flops(double value, double* current) {
    return guarded([&] {
        if (value != 0.0) ttr::set_batch_team_flops(value);
        if (current) *current = ttr::batch_team_flops();
    });
}

tt_status tt_round_adaptive_batch(const tt_view* xs, int32_t count, const double* tol,
                                  int64_t ell_block, const uint64_t* seeds, const tt_opts* opts,
                                  tt_out* ys) {
    return guarded([&] {
        if (count < 0) throw ttr::Error(TT_EINVAL, "count must be >= 0");
        if (count == 0) return;
        if (!xs || !tol || !seeds || !ys) throw ttr::Error(TT_EINVAL, "null batch array");
        ttr::Options o = make_opts(opts);
        if (o.prec == 0 && !o.recompress) {
            // one persistent launch over a library-owned workspace
            BatchArgs a = batch_args(xs, count, tol, seeds, ys);
            const size_t need = ttr::batch_workspace_bytes(a.sh, ell_block, o.f_init > 0.0 ? o.f_init : 0.1);
            int dev = 0;
            TTR_HIP(hipGetDevice(&dev));
            if (dev < 0 || dev >= 64) throw ttr::Error(TT_EUNSUPPORTED, "device index out of range");
            BatchCache& c = g_batch_cache[dev];
            std::lock_guard<std::mutex> lk(c.mu);
            if (c.cap < need) {
                if (c.p) {
                    TTR_HIP(hipDeviceSynchronize());
                    TTR_HIP(hipFree(c.p));
                    c.p = nullptr;
                    c.cap = 0;
                }
                if (hipMalloc(&c.p, need) != hipSuccess) {
                    (void)hipGetLastError();
                    c.p = nullptr;
                    throw ttr::Error(TT_ENOMEM, "batch workspace allocation of " + std::to_string(need) + " bytes failed");
                }
                c.cap = need;
            }
            tt_batch b;
            b.device = dev;
            b.plan.create(a.sh, a.cores, a.tol, ell_block, a.seeds, o, a.outs, c.p, c.cap);
            b.ys.assign(ys, ys + count);
            b.plan.launch(o.stream);
            batch_finish_impl(&b, o.stream);
            tt_info last{};
            fill_batch_info(last, b.plan, count - 1, b.info[count - 1]);
            g_info = last;
            return;
        }
        std::vector<std::shared_ptr<ttr::Job>> jobs;
        jobs.reserve(count);
        for (int i = 0; i < count; ++i) {
            if (!(tol[i] > 0.0)) throw ttr::Error(TT_EINVAL, "tol[" + std::to_string(i) + "] must be > 0");
            auto j = job_from_view(&xs[i], o.prec);
            ttr::OutCores oc = out_of(&ys[i], j->shape.d);
            j->kind = ttr::Job::ADAPTIVE;
            j->tol = tol[i];
            j->ell_block = ell_block;
            j->seed = seeds[i];
            j->opts = o;
            j->out_cores.assign(oc.cores, oc.cores + j->shape.d);
            j->out_cap.assign(oc.cap, oc.cap + j->shape.d);
            j->footprint = ttr::workspace_bytes(j->shape, 0, o.prec);
            jobs.push_back(j);
        }
        TTR_HIP(hipStreamSynchronize(o.stream));
        ttr::Executor& ex = ttr::default_executor();
        int submitted = 0;
        std::string first_err;
        int first_code = 0;
        try {
            for (auto& j : jobs) {
                ex.submit(j);
                ++submitted;
            }
        } catch (const ttr::Error& e) {
            first_code = e.code;
            first_err = e.what();
        }
        jobs.resize(submitted);
        ex.wait_all(jobs);
        for (int i = 0; i < submitted; ++i) {
            const auto& j = jobs[i];
            if (j->status == 0) {
                for (int k = 0; k <= j->shape.d; ++k) ys[i].ranks[k] = j->out_ranks[k];
                ys[i].orth = j->orth;
            } else if (first_code == 0) {
                first_code = j->status;
                first_err = "tensor " + std::to_string(i) + ": " + j->error;
            }
        }
        if (!jobs.empty()) store_info(jobs.back()->info);
        if (first_code != 0) throw ttr::Error(first_code, first_err);
    });
}

tt_status tt_server_create(const tt_server_cfg* cfg, tt_server** out) {
    return guarded([&] {
        if (!out) throw ttr::Error(TT_EINVAL, "null out");
        *out = nullptr;
        int dev = 0;
        TTR_HIP(hipGetDevice(&dev));
        size_t budget = cfg ? cfg->mem_budget : 0;
        if (budget == 0) {
            size_t free_b = 0, total_b = 0;
            TTR_HIP(hipMemGetInfo(&free_b, &total_b));
            budget = free_b / 10 * 8;
        }
        const int workers = (cfg && cfg->workers > 0) ? cfg->workers : 8;
        std::unique_ptr<tt_server> s(new tt_server());
        s->ex.reset(new ttr::Executor(dev, workers, budget));
        *out = s.release();
    });
}

tt_status tt_round_submit(tt_server* s, const tt_request* req, uint64_t* ticket) {
    return guarded([&] {
        if (!s || !req || !ticket) throw ttr::Error(TT_EINVAL, "null argument");
        ttr::Options o = make_opts(&req->opts);
        o.stream = nullptr;
        auto j = job_from_view(&req->x, o.prec);
        const int d = j->shape.d;
        if (req->kind == 0) {
            if (!(req->tol > 0.0)) throw ttr::Error(TT_EINVAL, "tol must be > 0");
            j->kind = ttr::Job::ADAPTIVE;
            j->tol = req->tol;
            j->ell_block = req->ell_block;
        } else if (req->kind == 1) {
            if (req->ell < 1) throw ttr::Error(TT_EINVAL, "ell must be >= 1");
            if (req->ell > 64) throw ttr::Error(TT_EUNSUPPORTED, "fixed-rank sketch size ell > 64 is not supported");
            j->kind = ttr::Job::FIXED;
            j->ell = req->ell;
            if (req->target_ranks) {
                if (req->target_ranks[0] != 1 || req->target_ranks[d] != 1)
                    throw ttr::Error(TT_EINVAL, "target_ranks[0] and [d] must be 1");
                for (int k = 1; k < d; ++k)
                    if (req->target_ranks[k] < 1) throw ttr::Error(TT_EINVAL, "target ranks must be >= 1");
                j->target.assign(req->target_ranks, req->target_ranks + d + 1);
            }
        } else {
            throw ttr::Error(TT_EINVAL, "request kind must be 0 (adaptive) or 1 (fixed)");
        }
        j->seed = req->seed;
        j->opts = o;
        j->owned_output = true;
        const int64_t cap_total = out_capacity_total(j->shape, &j->out_cap);
        // workspace + capacity staging + exact result, each pool buffer at
        // most twice its size (power-of-two classes)
        j->footprint = ttr::workspace_bytes(j->shape, j->kind == ttr::Job::FIXED ? j->ell : 0, o.prec) +
                       4 * (size_t)cap_total * 8;
        std::lock_guard<std::mutex> lk(s->mu);
        s->ex->submit(j);
        const uint64_t t = s->next++;
        s->jobs[t] = j;
        *ticket = t;
    });
}

static tt_status poll_impl(tt_server* s, uint64_t ticket, tt_result** out, bool block) {
    return guarded([&] {
        if (!s || !out) throw ttr::Error(TT_EINVAL, "null argument");
        *out = nullptr;
        std::shared_ptr<ttr::Job> j;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            auto it = s->jobs.find(ticket);
            if (it == s->jobs.end()) throw ttr::Error(TT_ENOTFOUND, "unknown ticket");
            j = it->second;
        }
        if (j->state.load() != 2) {
            if (!block) throw ttr::Error(TT_PENDING, "request not finished");
            s->ex->wait_all({j});
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->jobs.erase(ticket);
        }
        *out = make_result(s, j);
    });
}

tt_status tt_round_poll(tt_server* s, uint64_t ticket, tt_result** out) {
    return poll_impl(s, ticket, out, false);
}

tt_status tt_round_wait(tt_server* s, uint64_t ticket, tt_result** out) {
    return poll_impl(s, ticket, out, true);
}

tt_status tt_result_copy(const tt_result* r, double* const* dst, void* stream) {
    return guarded([&] {
        if (!r || !dst) throw ttr::Error(TT_EINVAL, "null argument");
        if (r->status != TT_OK) throw ttr::Error(TT_EINVAL, "result holds an error");
        const ResultImpl* ri = reinterpret_cast<const ResultImpl*>(r);
        const auto& j = *ri->job;
        hipStream_t st = (hipStream_t)stream;
        for (int k = 0; k < r->d; ++k) {
            const size_t bytes = (size_t)j.out_ranks[k] * j.shape.n[k] * j.out_ranks[k + 1] * 8;
            if (bytes == 0) continue;
            if (!dst[k]) throw ttr::Error(TT_EINVAL, "null destination core");
            TTR_HIP(hipMemcpyAsync(dst[k], j.out_cores[k], bytes, hipMemcpyDeviceToDevice, st));
        }
        TTR_HIP(hipStreamSynchronize(st));
    });
}

void tt_result_release(tt_result* r) {
    if (!r) return;
    ResultImpl* ri = reinterpret_cast<ResultImpl*>(r);
    try {
        ri->server->ex->release_result(*ri->job);
    } catch (...) {
    }
    delete ri;
}

void tt_server_destroy(tt_server* s) {
    if (!s) return;
    try {
        s->ex.reset();
    } catch (...) {
    }
    delete s;
}

}  // extern "C"
