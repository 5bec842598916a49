// extern "C" boundary of libttround (declared in include/ttround.h): argument
// validation, status codes and the thread-local error message.  No C++
// exception crosses this layer.
#include <cstring>
#include <string>

#include "../../include/ttround.h"
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

tt_status tt_kernel_timing(int32_t enable) {
    return guarded([&] { ttr::timing_enable(enable != 0); });
}

tt_status tt_kernel_timing_read(int32_t kind, int64_t* launches, double* total_ms) {
    return guarded([&] {
        if (!launches || !total_ms) throw ttr::Error(TT_EINVAL, "null output");
        if (kind < 0 || kind >= TT_KERNEL_KINDS) throw ttr::Error(TT_EINVAL, "unknown kernel kind");
        ttr::timing_read(kind, launches, total_ms);
    });
}

}  // extern "C"
