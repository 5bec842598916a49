// Host runtime of libttround: the launch sequences of the KRP roundings.
//
//  fixed rank (Sec. 3.2):   Omega -> partial contractions W_d..W_2 ->
//     for k = 1..d-1: S = V(Y_k) W_{k+1}; Q = qr(S); M = Q^T V(Y_k);
//     V(Y_k) <- Q; H(Y_{k+1}) = M H(X_{k+1})  -> optional Remark 2 pass.
//  adaptive (Sec. 3.3):     same sweep, growing Q by residual sketches
//     S = V(Y_k) W_{k+1}(:, new); S -= Q Q^T S; est = ||S||_F / sqrt(b);
//     while est > tau: Q_new = qr(S); Q_new = qr(Q_new - Q Q^T Q_new); ...
//     The projection M and the next core are formed once at loop exit
//     (the same product as the paper's row-by-row appends).
//
// Every step runs in the library's HIP kernels; the host only sequences
// launches and, in the adaptive loop, reads back the scalar estimate.
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <memory>
#include <mutex>

namespace ttr {

// ---------------------------------------------------------------------------
// Device buffers and the workspace pool
// ---------------------------------------------------------------------------
namespace {

// A fixed region of device memory handed out front to back: the scratch of
// the allocation-free entry point.  A carve that does not fit throws
// ENOMEM; nothing is ever returned before the region is reset.
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
    void* carve(size_t bytes) {
        const size_t b = (bytes + 255) / 256 * 256;
        if (b > size - used)
            throw Error(-2, "allocation-free scratch exhausted: " + std::to_string(used + b) +
                                " bytes needed, " + std::to_string(size) + " available");
        void* p = base + used;
        used += b;
        return p;
    }
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Arena* arena = nullptr;  // set: carve from the arena instead of hipMalloc
    void* get(size_t bytes) {
        if (bytes == 0) bytes = 256;
        if (bytes > cap && arena) {
            // a larger request takes a new slice (contents are never kept
            // across a growth, as with hipMalloc below)
            p = arena->carve(bytes);
            cap = (bytes + 255) / 256 * 256;
            return p;
        }
        if (bytes > cap) {
            if (p) TTR_HIP(hipFree(p));
            p = nullptr;
            cap = 0;
            const size_t want = bytes + bytes / 4;
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                throw Error(-2, "device allocation of " + std::to_string(want) + " bytes failed");
            }
            cap = want;
        }
        return p;
    }
    template <typename T>
    T* as(size_t count) {
        return static_cast<T*>(get(count * sizeof(T)));
    }
    ~DevBuf() {
        if (p && !arena) (void)hipFree(p);
    }
};

struct Workspace {
    int device = -1;
    DevBuf omega, w, colexp, maxexp, dn, doff, y0, y1, q, sbuf, tbuf, m, qrws, cqws, qrcnt, part, scal,
        sumpart, sumcnt, small1, small2, small3, small4, tint, tmp, qrsticky, wq1, wq2, ptab;
    // Deferred Householder fallback: while a rounding runs with lazy_qr set,
    // qr() launches only the CholeskyQR kernels and a breakdown sets the
    // device int qr_sticky; scalar readbacks fetch it too (host_int[1]) and
    // the rounding is redone with the eager fallback if it was set.
    bool lazy_qr = false;
    int* qr_sticky = nullptr;
    double* host = nullptr;  // pinned scalars
    int* host_int = nullptr;
    int zeroed_qrcnt = 0, zeroed_sumcnt = 0;
    double host_plain[64];  // host scalars of an arena workspace (not pinned)
    bool pinned = false;
    Workspace() {
        TTR_HIP(hipGetDevice(&device));
        TTR_HIP(hipHostMalloc((void**)&host, 64 * sizeof(double), hipHostMallocDefault));
        pinned = true;
        host_int = reinterpret_cast<int*>(host + 32);
    }
    // Every device buffer carved from `a`, host scalars in plain memory:
    // constructing and using this workspace allocates nothing.
    explicit Workspace(Arena* a) {
        TTR_HIP(hipGetDevice(&device));
        host = host_plain;
        host_int = reinterpret_cast<int*>(host + 32);
        for (DevBuf* b : {&omega, &w, &colexp, &maxexp, &dn, &doff, &y0, &y1, &q, &sbuf, &tbuf, &m, &qrws,
                          &cqws, &qrcnt, &part, &scal, &sumpart, &sumcnt, &small1, &small2, &small3,
                          &small4, &tint, &tmp, &qrsticky, &wq1, &wq2, &ptab})
            b->arena = a;
    }
    ~Workspace() {
        if (host && pinned) (void)hipHostFree(host);
    }
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    int* qr_counters(int n, hipStream_t s) {
        const size_t before = qrcnt.cap;
        int* p = qrcnt.as<int>(std::max(n, 1024));
        if (qrcnt.cap != before || !zeroed_qrcnt) {
            launch_fill_int(p, 0, (int64_t)(qrcnt.cap / sizeof(int)), s);
            zeroed_qrcnt = 1;
        }
        return p;
    }
    void begin_lazy_qr(hipStream_t s) {
        qr_sticky = qrsticky.as<int>(16);
        launch_fill_int(qr_sticky, 0, 16, s);
        host_int[1] = 0;
        lazy_qr = true;
    }
    void end_lazy_qr() { lazy_qr = false; }
    int* sum_counter(hipStream_t s) {
        const size_t before = sumcnt.cap;
        int* p = sumcnt.as<int>(16);
        if (sumcnt.cap != before || !zeroed_sumcnt) {
            launch_fill_int(p, 0, (int64_t)(sumcnt.cap / sizeof(int)), s);
            zeroed_sumcnt = 1;
        }
        return p;
    }
};

std::mutex g_pool_mu;
std::vector<std::unique_ptr<Workspace>> g_pool;

// A workspace taken from the pool for one call.  `stream` is the stream the
// call enqueues on: if an error unwinds past the lease after kernels were
// queued, the stream is drained before the workspace goes back to the pool,
// so no other call (on another stream) can take buffers that queued kernels
// still read or write.
struct WsLease {
    std::unique_ptr<Workspace> ws;
    hipStream_t stream;
    int unwinding_at_entry;
    explicit WsLease(hipStream_t s) : stream(s), unwinding_at_entry(std::uncaught_exceptions()) {
        int dev = 0;
        TTR_HIP(hipGetDevice(&dev));
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            for (size_t i = 0; i < g_pool.size(); ++i) {
                if (g_pool[i]->device == dev) {
                    ws = std::move(g_pool[i]);
                    g_pool.erase(g_pool.begin() + i);
                    break;
                }
            }
        }
        if (!ws) ws.reset(new Workspace());
    }
    ~WsLease() {
        if (ws) {
            if (std::uncaught_exceptions() > unwinding_at_entry) {
                // an error on the way out: wait for what was queued (and clear
                // a sticky error so the next call does not report it)
                (void)hipStreamSynchronize(stream);
                (void)hipGetLastError();
            }
            std::lock_guard<std::mutex> lk(g_pool_mu);
            g_pool.push_back(std::move(ws));
        }
    }
    Workspace* operator->() { return ws.get(); }
};

// ---------------------------------------------------------------------------
// Thin wrappers
// ---------------------------------------------------------------------------
void gemm(Workspace& ws, hipStream_t s, int M, int N, int K, const double* A, int64_t sam,
          int64_t sak, const double* B, int64_t sbk, int64_t sbn, double* C, int64_t scm,
          int64_t scn, double alpha = 1.0, double beta = 0.0, const float* Bf = nullptr,
          const int* bexp = nullptr, const unsigned short* Bh = nullptr, int bslices = 1,
          int64_t bstride = 0) {
    if (M <= 0 || N <= 0) return;
    GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.Bf = Bf;
    g.Bh = Bh;
    g.bexp = bexp;
    g.bslices = bslices;
    g.bstride = bstride;
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.scm = scm;
    g.scn = scn;
    g.alpha = alpha;
    g.beta = beta;
    const int splits = gemm_splits(M, N, K);
    double* partials = nullptr;
    if (splits > 1) partials = ws.part.as<double>((size_t)splits * M * N);
    TimedScope ts(KT_GEMM, s);
    launch_gemm(g, splits, partials, s);
}

// The same launch policy for a fully specified GemmArgs.
void gemm_args(Workspace& ws, hipStream_t s, const GemmArgs& g) {
    if (g.M <= 0 || g.N <= 0) return;
    const int splits = gemm_splits(g.M, g.N, g.K);
    double* partials = nullptr;
    if (splits > 1) partials = ws.part.as<double>((size_t)splits * g.M * g.N);
    TimedScope ts(KT_GEMM, s);
    launch_gemm(g, splits, partials, s);
}

double read_scalar(Workspace& ws, hipStream_t s, const double* dev) {
    TTR_HIP(hipMemcpyAsync(ws.host, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    if (ws.lazy_qr)
        TTR_HIP(hipMemcpyAsync(ws.host_int + 1, ws.qr_sticky, sizeof(int), hipMemcpyDeviceToHost, s));
    TTR_HIP(hipStreamSynchronize(s));
    return ws.host[0];
}

// Lazy-QR mode: has a CholeskyQR broken down since begin_lazy_qr (as of the
// last scalar readback or final_sync)?
bool qr_broke(const Workspace& ws) { return ws.lazy_qr && ws.host_int[1] != 0; }

// End-of-rounding synchronisation that also fetches the breakdown flag.
void final_sync(Workspace& ws, hipStream_t s) {
    if (ws.lazy_qr)
        TTR_HIP(hipMemcpyAsync(ws.host_int + 1, ws.qr_sticky, sizeof(int), hipMemcpyDeviceToHost, s));
    TTR_HIP(hipStreamSynchronize(s));
}

int read_int(Workspace& ws, hipStream_t s, const int* dev) {
    TTR_HIP(hipMemcpyAsync(ws.host_int, dev, sizeof(int), hipMemcpyDeviceToHost, s));
    TTR_HIP(hipStreamSynchronize(s));
    return ws.host_int[0];
}

// Thin QR: CholeskyQR2 when the panel is certified well conditioned, else
// (decided on the device) Householder TSQR on the untouched panel.  In
// lazy-QR mode the Householder kernels are not launched: a breakdown only
// raises the workspace's sticky flag (the caller redoes its rounding).
void qr(Workspace& ws, hipStream_t s, double* a, int m, int b, int lda, double* r_out = nullptr) {
    const QrPlan p = plan_qr(m, b, lda);
    TimedScope ts(KT_QR, s);
    // Route flags first (reset by every QR's first kernel), then the
    // Householder tree counters (zero between QRs): kept apart so that flags
    // a QR leaves behind never land among the counters of a QR of another
    // shape.
    int* base = ws.qr_counters(p.nodes + 16, s);
    int* flags = base;
    int* cnt = base + 8;
    double* cw = ws.cqws.as<double>(cq_workspace_doubles(m, b));
    launch_cq(a, m, b, lda, r_out, cw, flags, s, ws.lazy_qr ? ws.qr_sticky : nullptr);
    if (!ws.lazy_qr) {
        double* w = ws.qrws.as<double>(qr_workspace_doubles(p));
        launch_qr(p, a, r_out, w, cnt, s, flags);
    }
    static const bool trace = std::getenv("TTR_TRACE_QR") != nullptr;
    if (trace) {
        const int f = read_int(ws, s, flags);
        const int sh = read_int(ws, s, flags + 1);
        const int ni = read_int(ws, s, flags + 2);
        std::fprintf(stderr, "ttr qr m=%d b=%d route=%s near_identity_passes=%d\n", m, b,
                     f ? "householder" : (sh ? "shifted-cholqr3" : "cholqr2"), ni);
    }
}

// Thin QR of any width: block Gram-Schmidt with reorthogonalisation
// (BCGS2) over panels of at most 64 columns, each panel factored by qr()
// with its certificate and fallbacks.  R (b x b, column-major, ld b, zero
// below the diagonal) is written when r_out is given.
void qr_any(Workspace& ws, hipStream_t s, double* a, int m, int b, int lda, double* r_out = nullptr) {
    if (b <= 64) {
        qr(ws, s, a, m, b, lda, r_out);
        return;
    }
    if (m < b) throw Error(-1, "QR needs m >= b");
    double* C = ws.wq1.as<double>((size_t)b * 64 + 64);  // projection coefficients (p0 x bp, ld p0)
    double* Rp = ws.wq2.as<double>(64 * 64 + 64);        // R of one panel
    if (r_out) launch_axpby2d(nullptr, 0, 0, r_out, 1, b, b, b, 0.0, 0.0, s);
    for (int p0 = 0; p0 < b; p0 += 64) {
        const int bp = std::min(64, b - p0);
        double* P = a + (size_t)p0 * lda;
        for (int pass = 0; pass < (p0 > 0 ? 2 : 0); ++pass) {
            // C = Q_{<p0}^T P, then P -= Q_{<p0} C, and R[:p0, panel] += C
            gemm(ws, s, p0, bp, m, a, lda, 1, P, 1, lda, C, 1, p0);
            gemm(ws, s, m, bp, p0, a, 1, lda, C, 1, p0, P, 1, lda, -1.0, 1.0);
            if (r_out)
                launch_axpby2d(C, 1, p0, r_out + (size_t)p0 * b, 1, b, p0, bp, 1.0, pass == 0 ? 0.0 : 1.0, s);
        }
        qr(ws, s, P, m, bp, lda, r_out ? Rp : nullptr);
        if (r_out) launch_copy2d(Rp, 1, bp, r_out + (size_t)p0 * b + p0, 1, b, bp, bp, 1.0, s);
    }
}

// Small SVD of any width up to svd_wide_max(): the one-workgroup kernel
// for p, q <= 64, else the wide Jacobi driven from here (a readback of the
// rotation count per sweep).  Arguments as launch_svd_jacobi; t_dev holds
// 16 ints.
void svd_any(Workspace& ws, hipStream_t st, const double* A, int lda, int p, int q, double* G, double* Vs,
             double* sig, double tau, int target, int* t_dev, bool trans, bool split_only) {
    TimedScope ts(KT_SVD, st);
    if (p <= 64 && q <= 64) {
        launch_svd_jacobi(A, lda, p, q, G, Vs, sig, tau, target, t_dev, st, trans, split_only);
        return;
    }
    if (q > svd_wide_max() || p < q) throw Error(-6, "SVD wider than 512 columns is not supported");
    double* Aw = ws.small1.as<double>((size_t)p * q + 64);
    double* Vw = ws.tmp.as<double>((size_t)q * q + 64);
    int* sexp = t_dev + 8;
    unsigned* rot = reinterpret_cast<unsigned*>(t_dev + 9);
    launch_svd_wide_init(A, lda, p, q, trans, Aw, Vw, sexp, st);
    const int Q = q + (q & 1);
    int sweeps = 0;
    for (int sw = 0; sw < 60 && q >= 2; ++sw) {
        launch_fill_int(t_dev + 9, 0, 1, st);
        for (int r = 0; r < Q - 1; ++r) launch_svd_wide_round(Aw, Vw, p, q, r, rot, st);
        sweeps = sw + 1;
        if (read_int(ws, st, t_dev + 9) == 0) break;
    }
    launch_svd_wide_finish(Aw, Vw, sexp, p, q, G, Vs, sig, tau, target, sweeps, t_dev, st);
}

double sumsq(Workspace& ws, hipStream_t s, const double* a, int64_t sr, int64_t sc, int rows,
             int cols) {
    double* out = ws.scal.as<double>(8);
    double* part = ws.sumpart.as<double>(1024);
    launch_sumsq(a, sr, sc, rows, cols, out, part, ws.sum_counter(s), s);
    return read_scalar(ws, s, out);
}

int64_t prod_capped(const std::vector<int64_t>& n, int upto, int64_t cap) {
    int64_t p = 1;
    for (int i = 0; i < upto; ++i) {
        if (p > cap / std::max<int64_t>(n[i], 1)) return cap;
        p *= n[i];
    }
    return std::min(p, cap);
}

// ---------------------------------------------------------------------------
// Partial contractions state (Omega and W for modes 2..d).  For a sum of
// TTs every term has its own W_j (the formal sum's W_j is the terms' W_j
// stacked by rows) and all terms share Omega.
// ---------------------------------------------------------------------------
struct Sketch {
    const Summands& x;
    uint64_t seed;
    int prec;
    int64_t lcap;  // column capacity (storage stride)
    hipStream_t st;
    Workspace& ws;
    std::vector<int64_t> om_off;  // by 1-based mode
    struct TermW {
        std::vector<int64_t> off, ld, ss, mx;  // by 1-based mode j: storage offset, row
                                               // stride (transposed), slice stride, exponent slots
        std::vector<int> sl;                   // slices of W_j
        int64_t cexp_off = 0;
    };
    std::vector<TermW> tw;
    double* om = nullptr;
    void* w = nullptr;
    // FP64 sums whose terms share one shape: core k of every term is
    // contracted in one launch (Xt, Wnt, Woutt per mode in ptab), and the
    // slices are sized for the terms' rows together
    bool grouped = false;
    const void** ptab = nullptr;
    std::vector<const void*> hptab;
    int* colexp = nullptr;
    int* maxexp = nullptr;
    int64_t* dn = nullptr;
    int64_t* doff = nullptr;
    int64_t ncols = 0;  // generated columns (storage col == global col - gcol0)
    int64_t gcol0 = 0;
    int passes = 0;
    // Algorithmic work of the partial contractions so far (Sec. 3.1 cost
    // model): one float64 read of each contracted core and one write of
    // each W_k column block per pass, 2 r_{k-1} n_k r_k l + 2 r_{k-1} r_k l
    // flops per core (2 r_{d-1} n_d l for the last), one launch per core.
    int64_t pc_launches = 0;
    double pc_bytes = 0.0, pc_flops = 0.0;

    Sketch(const Summands& xs, uint64_t sd, int pr, int64_t cap, hipStream_t stream, Workspace& w_,
           int64_t global_col0 = 0)
        : x(xs), seed(sd), prec(pr), lcap(cap), st(stream), ws(w_), gcol0(global_col0) {
        const Shape& s = x.fs;
        const int d = s.d;
        om_off.assign(d + 2, 0);
        int64_t o = 0;
        for (int j = 2; j <= d; ++j) {
            om_off[j] = o;
            o += s.n[j - 1] * lcap;
        }
        const int64_t gy = (lcap + 63) / 64;
        int64_t wo = 0, mo = 0, co = 0;
        grouped = prec == 0 && x.m() > 1 && x.m() <= kSegGemmMax;
        for (int i = 1; grouped && i < x.m(); ++i)
            grouped = x.sh[i].r == x.sh[0].r;
        const int64_t gm = grouped ? x.m() : 1;
        tw.resize(x.m());
        for (int i = 0; i < x.m(); ++i) {
            const Shape& si = x.sh[i];
            TermW& t = tw[i];
            t.off.assign(d + 2, 0);
            t.ld.assign(d + 2, 4);
            t.ss.assign(d + 2, 0);
            t.mx.assign(d + 2, 0);
            t.sl.assign(d + 2, 1);
            for (int j = 2; j <= d; ++j) {
                t.off[j] = wo;
                t.sl[j] = pc_slices(gm * si.r[j - 1], si.r[j], prec);
                t.ld[j] = (si.r[j - 1] + 3) / 4 * 4;
                t.ss[j] = t.ld[j] * lcap;
                wo += t.sl[j] * t.ss[j];
                t.mx[j] = mo;
                mo += si.r[j - 1] * gy * t.sl[j];
            }
            t.cexp_off = co;
            co += (int64_t)(d + 2) * lcap;
        }
        om = ws.omega.as<double>(o);
        const size_t esz = (prec == 0) ? sizeof(double) : (prec == 1 ? sizeof(float) : 2);
        w = ws.w.get(wo * esz);
        if (grouped) {
            // per mode k = 1..d: X_k of every term, then W_{k+1}, then W_k
            const int m = x.m();
            hptab.assign((size_t)3 * m * (d + 1), nullptr);
            for (int k = 1; k <= d; ++k)
                for (int i = 0; i < m; ++i) {
                    hptab[(size_t)(3 * k + 0) * m + i] = x.cores[i][k - 1];
                    hptab[(size_t)(3 * k + 1) * m + i] = k < d ? wk(i, k + 1) : nullptr;
                    hptab[(size_t)(3 * k + 2) * m + i] = k >= 2 ? wk(i, k) : nullptr;
                }
            ptab = static_cast<const void**>(ws.ptab.get(hptab.size() * sizeof(void*)));
            TTR_HIP(hipMemcpyAsync(ptab, hptab.data(), hptab.size() * sizeof(void*), hipMemcpyHostToDevice, st));
        }
        if (prec != 0) {
            colexp = ws.colexp.as<int>(co);
            maxexp = ws.maxexp.as<int>(mo + 64);
        }
        // Per-mode sizes/offsets for modes 2..d (uploaded once per call).
        std::vector<int64_t> hn(d + 1, 0), ho(d + 1, 0);
        for (int j = 2; j <= d; ++j) {
            hn[j - 2] = s.n[j - 1];
            ho[j - 2] = om_off[j];
        }
        dn = ws.dn.as<int64_t>(d + 1);
        doff = ws.doff.as<int64_t>(d + 1);
        TTR_HIP(hipMemcpyAsync(dn, hn.data(), (d + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
        TTR_HIP(hipMemcpyAsync(doff, ho.data(), (d + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }

    double* omega(int j) { return om + om_off[j]; }
    void* wk(int i, int k) {
        const size_t esz = (prec == 0) ? sizeof(double) : (prec == 1 ? sizeof(float) : 2);
        return static_cast<char*>(w) + (size_t)tw[i].off[k] * esz;
    }
    const int* cexp(int i, int k) const {
        return colexp ? colexp + tw[i].cexp_off + (size_t)k * lcap : nullptr;
    }

    // Generate columns [ncols, ncols+nc) of Omega_t..Omega_d and contract
    // cores t..d of every term (one right-to-left pass).
    void pass(int t, int64_t nc) {
        const Shape& s = x.fs;
        const int d = s.d;
        if (nc <= 0) return;
        if (ncols + nc > lcap) throw Error(-6, "sketch column capacity exceeded");
        OmegaArgs oa{};
        oa.seed = seed;
        oa.first_mode = t;
        oa.n = dn + (t - 2);
        oa.off = doff + (t - 2);
        oa.base = om;
        oa.ld = lcap;
        oa.col0 = gcol0 + ncols;
        oa.store_col0 = ncols;
        oa.ncols = nc;
        int64_t maxn = 1;
        for (int j = t; j <= d; ++j) maxn = std::max(maxn, s.n[j - 1]);
        launch_omega(oa, d - t + 1, maxn, st);
        // one event pair around the back-to-back partial-contraction launches
        TimedScope ts(KT_PC, st, (d - t + 1) * (grouped ? 1 : x.m()));
        if (grouped) {
            const Shape& s0 = x.sh[0];
            const TermW& t0 = tw[0];
            const int m = x.m();
            for (int k = d; k >= t; --k) {
                PcArgs a{};
                a.terms = m;
                a.X = x.cores[0][k - 1];
                a.Xt = reinterpret_cast<const double* const*>(ptab + (size_t)(3 * k + 0) * m);
                a.r0 = (int)s0.r[k - 1];
                a.n = (int)s0.n[k - 1];
                a.r1 = (int)s0.r[k];
                a.Om = omega(k);
                a.ldo = lcap;
                a.Wnt = ptab + (size_t)(3 * k + 1) * m;  // null entries at k = d
                if (k < d) {
                    a.Wn = wk(0, k + 1);
                    a.in_ld = t0.ld[k + 1];
                    a.in_ss = t0.ss[k + 1];
                    a.in_slices = t0.sl[k + 1];
                }
                a.Wout = wk(0, k);
                a.Woutt = const_cast<void* const*>(ptab + (size_t)(3 * k + 2) * m);
                a.out_ld = t0.ld[k];
                a.out_ss = t0.ss[k];
                a.c0 = (int)ncols;
                a.nc = (int)nc;
                launch_pc_f64(a, st);
            }
        }
        for (int i = 0; i < (grouped ? 0 : x.m()); ++i) {
            const Shape& si = x.sh[i];
            const TermW& tm = tw[i];
            for (int k = d; k >= t; --k) {
                PcArgs a{};
                a.X = x.cores[i][k - 1];
                a.r0 = (int)si.r[k - 1];
                a.n = (int)si.n[k - 1];
                a.r1 = (int)si.r[k];
                a.Om = omega(k);
                a.ldo = lcap;
                if (k < d) {
                    a.Wn = wk(i, k + 1);
                    a.in_ld = tm.ld[k + 1];
                    a.in_ss = tm.ss[k + 1];
                    a.in_slices = tm.sl[k + 1];
                }
                a.Wout = wk(i, k);
                a.out_ld = tm.ld[k];
                a.out_ss = tm.ss[k];
                a.c0 = (int)ncols;
                a.nc = (int)nc;
                if (prec == 0) {
                    launch_pc_f64(a, st);
                } else {
                    a.in_maxexp = (k == d) ? nullptr : maxexp + tm.mx[k + 1];
                    a.out_maxexp = maxexp + tm.mx[k];
                    a.in_colexp = (k == d) ? nullptr : cexp(i, k + 1);
                    a.out_colexp = const_cast<int*>(cexp(i, k));
                    if (prec == 2)
                        launch_pc_bf16(a, st);
                    else
                        launch_pc_f32(a, st);
                }
            }
        }
        const double esz = prec == 0 ? 8.0 : (prec == 1 ? 4.0 : 2.0);
        for (int i = 0; i < x.m(); ++i) {
            const Shape& si = x.sh[i];
            for (int k = d; k >= t; --k) {
                const double r0 = (double)si.r[k - 1], nk = (double)si.n[k - 1], r1 = (double)si.r[k];
                pc_bytes += 8.0 * r0 * nk * r1 + esz * r0 * (double)nc;
                pc_flops += 2.0 * r0 * nk * r1 * (double)nc + (k < d ? 2.0 * r0 * r1 * (double)nc : 0.0);
                if (!grouped || i == 0) ++pc_launches;
            }
        }
        ncols += nc;
        ++passes;
    }

    // Z = V(Y_k) of the formal sum by column blocks: term i's block starts
    // at z[i] with row stride ldz[i] and is scaled by zs[i].
    struct ZBlocks {
        std::vector<const double*> z;
        std::vector<int64_t> ldz;
        std::vector<double> zs;
    };

    // S(rows x nb) = sum_i Z_i W^(i)_{k+1}(:, c0:c0+nb), S column-major (ld);
    // W is stored transposed (entry (b, c) at c * ld + b).
    void sketch_gemm(int k, const ZBlocks& zb, int rows, int64_t c0, int nb, double* S, int64_t ld) {
        if (grouped) {
            // every term in one launch: the products summed over the terms'
            // K segments (with W sliced for the terms' rows together, most
            // often one slice)
            SegGemm g{};
            g.M = rows;
            g.N = nb;
            g.nseg = x.m();
            g.C = S;
            g.ldc = ld;
            for (int i = 0; i < x.m(); ++i) {
                const TermW& tm = tw[i];
                g.K[i] = (int)x.sh[i].r[k];
                g.A[i] = zb.z[i];
                g.lda[i] = zb.ldz[i];
                g.alpha[i] = zb.zs[i];
                g.B[i] = static_cast<const double*>(wk(i, k + 1)) + c0 * tm.ld[k + 1];
                g.ldb[i] = tm.ld[k + 1];
                g.slices[i] = tm.sl[k + 1];
                g.ss[i] = tm.ss[k + 1];
            }
            TimedScope ts(KT_GEMM, st);
            launch_seg_gemm(g, st);
            return;
        }
        for (int i = 0; i < x.m(); ++i) {
            const TermW& tm = tw[i];
            const int K = (int)x.sh[i].r[k];
            const int sl = tm.sl[k + 1];
            const int64_t ss = tm.ss[k + 1], wl = tm.ld[k + 1], off = c0 * wl;
            const double beta = i > 0 ? 1.0 : 0.0;
            const double* Z = zb.z[i];
            const int64_t lz = zb.ldz[i];
            const double al = zb.zs[i];
            if (prec == 0)
                gemm(ws, st, rows, nb, K, Z, lz, 1, static_cast<const double*>(wk(i, k + 1)) + off, 1, wl, S,
                     1, ld, al, beta, nullptr, nullptr, nullptr, sl, ss);
            else if (prec == 1)
                gemm(ws, st, rows, nb, K, Z, lz, 1, nullptr, 1, wl, S, 1, ld, al, beta,
                     static_cast<const float*>(wk(i, k + 1)) + off, cexp(i, k + 1) + c0, nullptr, sl, ss);
            else
                gemm(ws, st, rows, nb, K, Z, lz, 1, nullptr, 1, wl, S, 1, ld, al, beta, nullptr,
                     cexp(i, k + 1) + c0, static_cast<const unsigned short*>(wk(i, k + 1)) + off, sl, ss);
        }
    }
};

// Z blocks of mode k: the terms' first cores (with their weights) at k = 1,
// else column blocks of the formal V(Y_k) held in ycur (row stride R_k).
Sketch::ZBlocks z_blocks(const Summands& x, int k, const double* ycur) {
    Sketch::ZBlocks zb;
    for (int i = 0; i < x.m(); ++i) {
        if (k == 1) {
            zb.z.push_back(x.cores[i][0]);
            zb.ldz.push_back(x.sh[i].r[1]);
            zb.zs.push_back(x.w[i]);
        } else {
            zb.z.push_back(ycur + x.off[i][k]);
            zb.ldz.push_back(x.fs.r[k]);
            zb.zs.push_back(1.0);
        }
    }
    return zb;
}

// M(lk x R_k, row stride R_k) = Q^T Z, block by block.
void project(Workspace& ws, hipStream_t st, const Summands& x, const Sketch::ZBlocks& zb, int k,
             const double* Q, int rows, int lk, double* M) {
    const int64_t R = x.fs.r[k];
    for (int i = 0; i < x.m(); ++i)
        gemm(ws, st, lk, (int)x.sh[i].r[k], rows, Q, rows, 1, zb.z[i], zb.ldz[i], 1, M + x.off[i][k], R, 1,
             zb.zs[i], 0.0);
}

// Formal Y_{k+1} = M H(X_{k+1}): term i's block of M times its core k+1,
// written into the term's column block of Y_{k+1} (or, for the last core,
// summed).  dst is lk x n_{k+1} x R_{k+1} row-major.
void next_core(Workspace& ws, hipStream_t st, const Summands& x, int k, const double* M, int lk,
               double* dst) {
    const Shape& fs = x.fs;
    const int d = fs.d;
    const int64_t R = fs.r[k], R1 = fs.r[k + 1], n1 = fs.n[k];
    for (int i = 0; i < x.m(); ++i) {
        const int64_t ri = x.sh[i].r[k], ri1 = x.sh[i].r[k + 1];
        const int nn = (int)(n1 * ri1);
        GemmArgs g{};
        g.M = lk;
        g.N = nn;
        g.K = (int)ri;
        g.A = M + x.off[i][k];
        g.sam = R;
        g.sak = 1;
        g.B = x.cores[i][k];
        g.sbk = nn;
        g.sbn = 1;
        g.alpha = 1.0;
        if (k + 1 == d || x.m() == 1) {
            g.C = dst;
            g.scm = n1 * R1;
            g.scn = 1;
            g.beta = (k + 1 == d && i > 0) ? 1.0 : 0.0;
        } else {
            g.C = dst + x.off[i][k + 1];
            g.scm = n1 * R1;
            g.scn = 1;
            g.cdiv = (int)ri1;
            g.cs_hi = R1;
            g.beta = 0.0;
        }
        gemm_args(ws, st, g);
    }
}

// Right-to-left truncation pass (Remark 2) on caller cores in place.  tau >=
// 0 selects the tail rule, else target ranks (host [d+1]).
// The core being truncated lives in one of two scratch buffers (the sweep
// ping-pong, free by now): step k factors its core there, writes the
// truncated core k straight into cores[k-1] and the updated core k-1 into
// the other buffer, so only the first and the last core are copied.
void recompress(Workspace& ws, hipStream_t st, const Shape& s, double** cores, int64_t* ranks,
                double tau, const int64_t* target) {
    const int d = s.d;
    // every step factors a core whose left rank is an untruncated bond rank:
    // reject before anything of the pass is queued
    for (int k = 1; k < d; ++k)
        if (ranks[k] > svd_wide_max()) throw Error(-6, "recompression supports ranks <= 512");
    int64_t maxcore = 0;
    for (int k = 1; k <= d; ++k) maxcore = std::max(maxcore, ranks[k - 1] * s.n[k - 1] * ranks[k]);
    double* buf[2] = {ws.y0.as<double>(maxcore + 64), ws.y1.as<double>(maxcore + 64)};
    int cb = 0;
    TTR_HIP(hipMemcpyAsync(buf[0], cores[d - 1], (size_t)(ranks[d - 1] * s.n[d - 1] * ranks[d]) * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
    for (int k = d; k >= 2; --k) {
        const int b = (int)ranks[k - 1];
        const int m = (int)(s.n[k - 1] * ranks[k]);
        double* H = buf[cb];  // b x m row-major
        double* G = ws.small2.as<double>((size_t)b * b + 64);
        double* Vs = ws.small3.as<double>((size_t)b * b + 64);
        double* sig = ws.small4.as<double>(b + 64);
        int* tdev = ws.tint.as<int>(16);
        const int tgt = target ? (int)target[k - 1] : 0;
        int q;
        if (m >= b) {
            // H^T (m x b, column-major) is the row-major H buffer itself; the
            // SVD reads R^T straight from the column-major R.
            double* R = ws.tbuf.as<double>((size_t)b * b + 64);
            qr_any(ws, st, H, m, b, m, R);
            q = b;
            svd_any(ws, st, R, b, b, q, G, Vs, sig, tau, tgt, tdev, true, tau < 0.0);
        } else {
            q = m;
            svd_any(ws, st, H, m, b, q, G, Vs, sig, tau, tgt, tdev, true, tau < 0.0);
        }
        // a target rank is known on the host; the tail rule needs the device
        const int t = (tau >= 0.0) ? read_int(ws, st, tdev) : std::min(std::max(tgt, 1), q);
        static const bool trace = std::getenv("TTR_TRACE_QR") != nullptr;
        if (trace)
            std::fprintf(stderr, "ttr svd p=%d q=%d kept=%d sweeps=%d chol=%d failpiv=%d\n", b, q, t,
                         read_int(ws, st, tdev + 1), read_int(ws, st, tdev + 2), read_int(ws, st, tdev + 3));
        // Truncated core k: H(Y_k) = V_t^T Q^T (t x m), or V_t^T when m < b.
        if (m >= b) {
            gemm(ws, st, t, m, b, Vs, q, 1, H, m, 1, cores[k - 1], m, 1);
        } else {
            launch_copy2d(Vs, q, 1, cores[k - 1], m, 1, t, m, 1.0, st);
        }
        // Updated core k-1: V(Y_{k-1}) G_t, into the other buffer.
        const int rows = (int)(ranks[k - 2] * s.n[k - 2]);
        gemm(ws, st, rows, t, b, cores[k - 2], b, 1, G, 1, b, buf[1 - cb], t, 1);
        cb = 1 - cb;
        ranks[k - 1] = t;
    }
    TTR_HIP(hipMemcpyAsync(cores[0], buf[cb], (size_t)(ranks[0] * s.n[0] * ranks[1]) * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
}

void check_capacity(const Shape& s, const std::vector<int64_t>& l, const OutCores& y) {
    for (int k = 1; k <= s.d; ++k) {
        const int64_t need = l[k - 1] * s.n[k - 1] * l[k];
        if (need > y.cap[k - 1])
            throw Error(-2, "output core " + std::to_string(k) + " needs " + std::to_string(need) +
                                " elements, capacity " + std::to_string(y.cap[k - 1]));
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Shapes
// ---------------------------------------------------------------------------
Shape make_shape(int d, const int64_t* n, const int64_t* ranks) {
    if (d < 2) throw Error(-1, "d must be >= 2");
    if (!n || !ranks) throw Error(-1, "null dims or ranks");
    Shape s;
    s.d = d;
    s.n.assign(n, n + d);
    s.r.assign(ranks, ranks + d + 1);
    if (s.r[0] != 1 || s.r[d] != 1) throw Error(-1, "ranks[0] and ranks[d] must be 1");
    for (int k = 0; k < d; ++k) {
        if (s.n[k] < 1 || s.n[k] > (1 << 20)) throw Error(-1, "mode size out of range");
        if (s.r[k + 1] < 1 || s.r[k + 1] > (1 << 16)) throw Error(-1, "rank out of range");
    }
    for (int k = 0; k < d; ++k)
        if (s.r[k] * s.n[k] * s.r[k + 1] > ((int64_t)1 << 31))
            throw Error(-6, "core too large (more than 2^31 elements)");
    return s;
}

Summands single_term(const Shape& s, const double* const* cores) {
    Summands x;
    x.fs = s;
    x.sh.push_back(s);
    x.cores.push_back(cores);
    x.w.push_back(1.0);
    x.off.push_back(std::vector<int64_t>(s.d + 1, 0));
    return x;
}

Summands make_sum(const std::vector<Shape>& sh, const std::vector<const double* const*>& cores,
                  const double* weights) {
    if (sh.empty() || sh.size() != cores.size()) throw Error(-1, "a sum needs at least one term");
    const int d = sh[0].d;
    Summands x;
    x.fs.d = d;
    x.fs.n = sh[0].n;
    x.fs.r.assign(d + 1, 0);
    x.fs.r[0] = x.fs.r[d] = 1;
    for (size_t i = 0; i < sh.size(); ++i) {
        if (sh[i].d != d || sh[i].n != sh[0].n)
            throw Error(-1, "all terms of a sum need the same order and mode sizes");
        std::vector<int64_t> off(d + 1, 0);
        for (int k = 1; k < d; ++k) {
            off[k] = x.fs.r[k];
            x.fs.r[k] += sh[i].r[k];
            if (x.fs.r[k] > (1 << 16)) throw Error(-1, "summed rank out of range");
        }
        x.sh.push_back(sh[i]);
        x.cores.push_back(cores[i]);
        x.w.push_back(weights ? weights[i] : 1.0);
        x.off.push_back(off);
    }
    for (int k = 0; k < d; ++k)
        if (x.fs.r[k] * x.fs.n[k] * x.fs.r[k + 1] > ((int64_t)1 << 31))
            throw Error(-6, "formal core too large (more than 2^31 elements)");
    return x;
}

std::vector<int64_t> rank_caps(const Shape& s) {
    std::vector<int64_t> c(s.d + 1, 1);
    for (int k = 1; k < s.d; ++k) c[k] = std::min(s.r[k], prod_capped(s.n, k, INT64_MAX / 4));
    return c;
}

// ---------------------------------------------------------------------------
// Workspace estimate
// ---------------------------------------------------------------------------
size_t workspace_bytes(const Summands& x, int64_t ell_max, int prec) {
    const Shape& s = x.fs;
    const int d = s.d;
    const std::vector<int64_t> cap = rank_caps(s);
    std::vector<int64_t> l(d + 1, 1);
    int64_t lcap = 1, rmax = 1;
    if (ell_max > 0) {
        for (int k = 1; k < d; ++k) l[k] = std::min<int64_t>({ell_max, l[k - 1] * s.n[k - 1], s.r[k]});
        lcap = ell_max;
    } else {
        l = cap;
        for (int k = 1; k < d; ++k) lcap = std::max(lcap, cap[k]);
        lcap = std::max<int64_t>(lcap, (int64_t)std::ceil(0.1 * (double)lcap));
    }
    for (int k = 0; k <= d; ++k) rmax = std::max(rmax, s.r[k]);
    const size_t esz = prec == 0 ? 8 : (prec == 1 ? 4 : 2);
    size_t b = 0;
    int64_t maxy = 1, maxrows = 1;
    for (int k = 1; k <= d; ++k) {
        maxy = std::max(maxy, l[k - 1] * s.n[k - 1] * s.r[k]);
        maxrows = std::max(maxrows, l[k - 1] * s.n[k - 1]);
        if (k >= 2) {
            b += (size_t)s.n[k - 1] * lcap * 8;       // Omega
            for (const Shape& si : x.sh) {
                const int64_t sl = pc_slices(si.r[k - 1], si.r[k], prec);
                b += (size_t)sl * ((si.r[k - 1] + 3) / 4 * 4) * lcap * esz;  // W slices
                b += (size_t)sl * si.r[k - 1] * ((lcap + 63) / 64) * 4;      // exponent slots
            }
        }
    }
    b += (size_t)x.m() * (d + 2) * lcap * 4;          // column exponents
    b += 2 * (size_t)maxy * 8;                        // sweep ping-pong
    b += (size_t)maxrows * lcap * 8;                  // Q
    b += (size_t)lcap * rmax * 8 + (size_t)lcap * 64 * 8;  // M, residual block
    b += 3 * (size_t)maxrows * 64 * 8;                // QR scratch (CholeskyQR + TSQR)
    b += (size_t)64 * 64 * 64 * 8;                    // split-K GEMM partials
    if (lcap > 64)  // wide QR panels' coefficients, wide SVD (A, V, R, G, Vs)
        b += ((size_t)lcap * 64 + 5 * (size_t)lcap * lcap + 64 * 64) * 8;
    return b + b / 8 + ((size_t)16 << 20);
}

size_t workspace_bytes(const Shape& s, int64_t ell_max, int prec) {
    return workspace_bytes(single_term(s, nullptr), ell_max, prec);
}

// ---------------------------------------------------------------------------
// Fixed rank (Sec. 3.2)
// ---------------------------------------------------------------------------
// TTR_FORCE_QR_RETRY (read per call): repeat every rounding as if a QR had
// broken down, so tests can run the repeat path on well-posed inputs.
static bool force_qr_retry() { return std::getenv("TTR_FORCE_QR_RETRY") != nullptr; }

// Lazy-QR mode for the duration of one rounding attempt (always left off).
struct LazyQr {
    Workspace& ws;
    LazyQr(Workspace& w, hipStream_t s, bool on) : ws(w) {
        if (on) ws.begin_lazy_qr(s);
    }
    ~LazyQr() { ws.end_lazy_qr(); }
    LazyQr(const LazyQr&) = delete;
    LazyQr& operator=(const LazyQr&) = delete;
};

// One attempt of the fixed-rank rounding; false if a CholeskyQR broke down
// in lazy-QR mode (the outputs are then incomplete).
static bool round_fixed_once(Workspace& ws, const Summands& x, const int64_t* target, int64_t ell,
                             uint64_t seed, const Options& o, OutCores& y, RoundInfo& info) {
    const Shape& s = x.fs;
    const int d = s.d;
    hipStream_t st = o.stream;

    std::vector<int64_t> l(d + 1, 1);
    for (int k = 1; k < d; ++k) l[k] = std::min<int64_t>({ell, l[k - 1] * s.n[k - 1], s.r[k]});
    check_capacity(s, l, y);

    Sketch sk(x, seed, o.prec, ell, st, ws);
    sk.pass(2, ell);

    int64_t maxy = 0, maxrows = 0;
    for (int k = 1; k <= d; ++k) {
        maxy = std::max(maxy, l[k - 1] * s.n[k - 1] * s.r[k]);
        maxrows = std::max(maxrows, l[k - 1] * s.n[k - 1]);
    }
    double* ybuf[2] = {ws.y0.as<double>(maxy), ws.y1.as<double>(maxy)};
    double* Q = ws.q.as<double>(maxrows * ell);
    double* M = ws.m.as<double>((size_t)ell * *std::max_element(s.r.begin(), s.r.end()));

    const double* ycur = nullptr;
    for (int k = 1; k < d; ++k) {
        const int rows = (int)(l[k - 1] * s.n[k - 1]);
        const int lk = (int)l[k];
        const Sketch::ZBlocks zb = z_blocks(x, k, ycur);
        sk.sketch_gemm(k, zb, rows, 0, lk, Q, rows);
        qr_any(ws, st, Q, rows, lk, rows);
        project(ws, st, x, zb, k, Q, rows, lk, M);
        launch_copy2d(Q, 1, rows, y.cores[k - 1], lk, 1, rows, lk, 1.0, st);
        double* dst = (k == d - 1) ? y.cores[d - 1] : ybuf[k & 1];
        next_core(ws, st, x, k, M, lk, dst);
        ycur = dst;
    }
    for (int k = 0; k <= d; ++k) y.ranks[k] = l[k];
    y.orth = 1;
    bool cut = false;
    if (target)
        for (int k = 1; k < d; ++k) cut = cut || (target[k] < l[k]);
    if (cut) {
        std::vector<int64_t> tg(d + 1, 1);
        for (int k = 1; k < d; ++k) tg[k] = std::max<int64_t>(1, std::min(target[k], l[k]));
        recompress(ws, st, s, y.cores, y.ranks, -1.0, tg.data());
        y.orth = 2;
    }
    final_sync(ws, st);
    info = RoundInfo{};
    info.passes = sk.passes;
    info.pc_launches = sk.pc_launches;
    info.pc_bytes = sk.pc_bytes;
    info.pc_flops = sk.pc_flops;
    return !qr_broke(ws);
}

// The first attempt defers the Householder fallback of every QR (one flag
// checked when the rounding ends); a breakdown, which none of the measured
// workloads hits, repeats the rounding with the fallback launched per QR.
void round_fixed(const Summands& x, const int64_t* target, int64_t ell, uint64_t seed,
                 const Options& o, OutCores& y, RoundInfo& info) {
    if (ell < 1) throw Error(-1, "ell must be >= 1");
    if (ell > svd_wide_max()) throw Error(-6, "fixed-rank sketch size ell > 512 is not supported");
    WsLease lease(o.stream);
    const bool force = force_qr_retry();
    for (int attempt = 0; attempt < 2; ++attempt) {
        LazyQr lq(*lease.ws, o.stream, attempt == 0);
        if (round_fixed_once(*lease.ws, x, target, ell, seed, o, y, info) && !(force && attempt == 0)) {
            info.qr_retries = attempt;
            return;
        }
    }
}

void round_fixed(const Shape& s, const double* const* cores, const int64_t* target, int64_t ell,
                 uint64_t seed, const Options& o, OutCores& y, RoundInfo& info) {
    round_fixed(single_term(s, cores), target, ell, seed, o, y, info);
}

// The fixed-rank rounding with every device buffer carved from the
// caller's region (the allocation-free entry point).  The Householder
// fallback is launched eagerly (a breakdown costs no repeat and no host
// readback); the result is the same as round_fixed's.  On an error the
// stream is drained before returning, so the region is idle again.
void round_fixed_in(void* region, size_t region_bytes, const Shape& s, const double* const* cores,
                    const int64_t* target, int64_t ell, uint64_t seed, const Options& o, OutCores& y,
                    RoundInfo& info) {
    if (ell < 1) throw Error(-1, "ell must be >= 1");
    if (ell > svd_wide_max()) throw Error(-6, "fixed-rank sketch size ell > 512 is not supported");
    Arena arena;
    arena.base = static_cast<char*>(region);
    arena.size = region_bytes;
    Workspace ws(&arena);
    TimingPause no_timing;
    try {
        round_fixed_once(ws, single_term(s, cores), target, ell, seed, o, y, info);
    } catch (...) {
        (void)hipStreamSynchronize(o.stream);
        (void)hipGetLastError();
        throw;
    }
    info.qr_retries = 0;
}

// ---------------------------------------------------------------------------
// Adaptive rank (Sec. 3.3)
// ---------------------------------------------------------------------------
// One attempt of the adaptive rounding; false if a CholeskyQR broke down in
// lazy-QR mode (seen at a scalar readback or at the end).
static bool round_adaptive_once(Workspace& ws, const Summands& x, double tol, int64_t ell_block,
                                uint64_t seed, const Options& o, OutCores& y, RoundInfo& info) {
    const Shape& s = x.fs;
    const int d = s.d;
    hipStream_t st = o.stream;
    const double f_init = (o.f_init > 0.0) ? o.f_init : 0.1;

    const std::vector<int64_t> cap = rank_caps(s);
    int64_t rmax = 1, lcap = 1, maxrows = 1, maxy = 1;
    for (int k = 1; k < d; ++k) {
        rmax = std::max(rmax, s.r[k]);
        lcap = std::max(lcap, cap[k]);
    }
    for (int k = 1; k <= d; ++k) {
        maxrows = std::max(maxrows, cap[k - 1] * s.n[k - 1]);
        maxy = std::max(maxy, cap[k - 1] * s.n[k - 1] * s.r[k]);
    }
    const int64_t r0 = (int64_t)std::ceil(f_init * (double)rmax);
    lcap = std::max(lcap, r0);
    // Output capacity check against the worst-case ranks.
    check_capacity(s, cap, y);

    Sketch sk(x, seed, o.prec, lcap, st, ws);
    sk.pass(2, r0);

    int64_t bmax = 1;
    for (int k = 1; k < d; ++k) {
        const int64_t rb = cap[k];
        const int64_t bi = (int64_t)std::ceil(f_init * (double)rb);
        const int64_t bl = ell_block > 0 ? ell_block : (int64_t)std::ceil(0.05 * (double)rb);
        bmax = std::max({bmax, bi, bl});
    }
    bmax = std::min(bmax, lcap);
    if (bmax > 64) throw Error(-6, "adaptive sketch blocks wider than 64 are not supported");

    double* ybuf[2] = {ws.y0.as<double>(maxy), ws.y1.as<double>(maxy)};
    double* Q = ws.q.as<double>(maxrows * lcap);
    double* T = ws.tbuf.as<double>(lcap * bmax + 64);
    double* M = ws.m.as<double>(lcap * rmax);

    double nrmx = o.nrmx;
    if (!(nrmx > 0.0)) {
        // Remark 1: ||X|| ~ ||V(X_1) W_2||_F / sqrt(r0).
        const int rows = (int)s.n[0];
        double* tmp = ws.sbuf.as<double>((size_t)rows * r0 + 64);
        sk.sketch_gemm(1, z_blocks(x, 1, nullptr), rows, 0, (int)r0, tmp, rows);
        nrmx = std::sqrt(sumsq(ws, st, tmp, 1, rows, rows, (int)r0) / (double)r0);
    }
    const double tau = tol * nrmx / std::sqrt((double)(d - 1));
    info = RoundInfo{};
    info.tau = tau;
    info.nrmx = nrmx;
    info.min_margin = INFINITY;

    const double* ycur = nullptr;
    int64_t lprev = 1;
    for (int k = 1; k < d; ++k) {
        const int rows = (int)(lprev * s.n[k - 1]);
        const int cols = (int)s.r[k];
        const int rbar = std::min(rows, cols);
        const int binit = std::max(1, std::min(rbar, (int)std::ceil(f_init * (double)rbar)));
        const Sketch::ZBlocks zb = z_blocks(x, k, ycur);
        sk.sketch_gemm(k, zb, rows, 0, binit, Q, rows);
        qr(ws, st, Q, rows, binit, rows);
        int ncq = binit;
        const int blk = ell_block > 0 ? (int)ell_block : (int)std::ceil(0.05 * (double)rbar);
        while (ncq < rbar) {
            const int bb = std::min(blk, rbar - ncq);
            const int64_t need = ncq + bb;
            if (sk.ncols < need) {
                const int64_t grow = std::min(lcap - sk.ncols, std::max(need - sk.ncols, sk.ncols));
                sk.pass(k + 1, grow);
            }
            double* S = Q + (size_t)ncq * rows;  // candidate columns follow Q
            sk.sketch_gemm(k, zb, rows, ncq, bb, S, rows);
            // S -= Q (Q^T S)
            gemm(ws, st, ncq, bb, rows, Q, rows, 1, S, 1, rows, T, bb, 1);
            gemm(ws, st, rows, bb, ncq, Q, 1, rows, T, bb, 1, S, 1, rows, -1.0, 1.0);
            const double est = std::sqrt(sumsq(ws, st, S, 1, rows, rows, bb) / (double)bb);
            if (qr_broke(ws)) return false;
            info.iterations++;
            if (tau > 0) info.min_margin = std::min(info.min_margin, std::fabs(est - tau) / tau);
            if (!(est > tau)) break;
            {
                // The residual block is where a sketch wider than the numerical
                // rank shows up: its QR keeps the eager fallback, so such a
                // breakdown costs no repeat of the rounding.
                const bool lazy = ws.lazy_qr;
                ws.lazy_qr = false;
                qr(ws, st, S, rows, bb, rows);
                ws.lazy_qr = lazy;
            }
            gemm(ws, st, ncq, bb, rows, Q, rows, 1, S, 1, rows, T, bb, 1);
            gemm(ws, st, rows, bb, ncq, Q, 1, rows, T, bb, 1, S, 1, rows, -1.0, 1.0);
            qr(ws, st, S, rows, bb, rows);
            ncq += bb;
        }
        const int lk = ncq;
        project(ws, st, x, zb, k, Q, rows, lk, M);
        launch_copy2d(Q, 1, rows, y.cores[k - 1], lk, 1, rows, lk, 1.0, st);
        double* dst = (k == d - 1) ? y.cores[d - 1] : ybuf[k & 1];
        next_core(ws, st, x, k, M, lk, dst);
        ycur = dst;
        y.ranks[k] = lk;
        lprev = lk;
    }
    y.ranks[0] = y.ranks[d] = 1;
    y.orth = 1;
    if (o.recompress) {
        recompress(ws, st, s, y.cores, y.ranks, tau, nullptr);
        y.orth = 2;
    }
    final_sync(ws, st);
    info.passes = sk.passes;
    info.pc_launches = sk.pc_launches;
    info.pc_bytes = sk.pc_bytes;
    info.pc_flops = sk.pc_flops;
    if (info.iterations == 0) info.min_margin = INFINITY;
    return !qr_broke(ws);
}

// Deferred Householder fallback as in round_fixed; the breakdown flag is
// also read with every estimator readback, so a failed attempt stops early.
void round_adaptive(const Summands& x, double tol, int64_t ell_block, uint64_t seed,
                    const Options& o, OutCores& y, RoundInfo& info) {
    if (!(tol > 0.0)) throw Error(-1, "tol must be > 0");
    WsLease lease(o.stream);
    const bool force = force_qr_retry();
    for (int attempt = 0; attempt < 2; ++attempt) {
        LazyQr lq(*lease.ws, o.stream, attempt == 0);
        if (round_adaptive_once(*lease.ws, x, tol, ell_block, seed, o, y, info) && !(force && attempt == 0)) {
            info.qr_retries = attempt;
            return;
        }
    }
}

void round_adaptive(const Shape& s, const double* const* cores, double tol, int64_t ell_block,
                    uint64_t seed, const Options& o, OutCores& y, RoundInfo& info) {
    round_adaptive(single_term(s, cores), tol, ell_block, seed, o, y, info);
}

// ---------------------------------------------------------------------------
// Deterministic TT-SVD rounding (Sec. 2.3, Algorithm "TT-Rounding"): the
// same-GPU baseline of the randomized roundings.
// ---------------------------------------------------------------------------
// Right-to-left orthogonalisation of a working copy of X, then tau =
// tol ||Y_1|| / sqrt(d-1), then left to right: V(Y_k) = Q R, the SVD of R
// truncated by the tail rule (or to the target rank), Y_k = Q U_t,
// Y_{k+1} = S_t V_t^T H(Y_{k+1}).  The Jacobi runs on R^T (R^T W = G with
// orthogonal W), so U_t = W_t and S_t V_t^T = G_t^T come out without a
// division by a singular value.  A factor with fewer rows than columns is
// taken by the SVD alone (its QR would not be thin).
void round_ttsvd(const Shape& s, const double* const* cores, double tol, const int64_t* target,
                 const Options& o, OutCores& y, RoundInfo& info) {
    const int d = s.d;
    hipStream_t st = o.stream;
    if (!target && !(tol > 0.0)) throw Error(-1, "tol must be > 0");
    for (int k = 1; k < d; ++k)
        if (s.r[k] > svd_wide_max()) throw Error(-6, "TT-SVD supports ranks <= 512");
    WsLease lease(st);
    Workspace& ws = *lease.ws;
    std::vector<int64_t> off(d + 1, 0), r(s.r);
    int64_t maxcore = 1;
    for (int k = 1; k <= d; ++k) {
        const int64_t sz = s.r[k - 1] * s.n[k - 1] * s.r[k];
        off[k] = off[k - 1] + sz;
        maxcore = std::max(maxcore, sz);
    }
    double* Z = ws.w.as<double>(off[d] + 64);  // working copy of the cores
    for (int k = 1; k <= d; ++k)
        TTR_HIP(hipMemcpyAsync(Z + off[k - 1], cores[k - 1], (size_t)(off[k] - off[k - 1]) * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
    double* tmp = ws.y0.as<double>(maxcore + 64);
    int rmax = 1;
    for (int k = 0; k <= d; ++k) rmax = std::max<int>(rmax, (int)s.r[k]);
    double* R = ws.tbuf.as<double>((size_t)rmax * rmax + 64);
    double* G = ws.small2.as<double>((size_t)rmax * rmax + 64);
    double* Vs = ws.small3.as<double>((size_t)rmax * rmax + 64);
    double* sig = ws.small4.as<double>(rmax + 64);
    int* tdev = ws.tint.as<int>(16);

    // 1. right-to-left orthogonalisation (ranks only shrink)
    for (int k = d; k >= 2; --k) {
        const int b = (int)r[k - 1];
        const int m = (int)(s.n[k - 1] * r[k]);
        double* H = Z + off[k - 1];  // H(Y_k): b x m row-major = H^T column-major (ld m)
        double* Yp = Z + off[k - 2];
        const int rows = (int)(r[k - 2] * s.n[k - 2]);
        if (m >= b) {
            qr_any(ws, st, H, m, b, m, R);  // H^T = Q R: the new H(Y_k) is Q^T in place
            gemm(ws, st, rows, b, b, Yp, b, 1, R, b, 1, tmp, b, 1);  // V(Y_{k-1}) R^T
            TTR_HIP(hipMemcpyAsync(Yp, tmp, (size_t)rows * b * sizeof(double), hipMemcpyDeviceToDevice, st));
        } else {
            // H (b x m, b > m) = G W^T: the new H(Y_k) is W^T (m x m), V(Y_{k-1}) G
            svd_any(ws, st, H, m, b, m, G, Vs, sig, -1.0, m, tdev, true, false);
            TTR_HIP(hipMemcpyAsync(H, Vs, (size_t)m * m * sizeof(double), hipMemcpyDeviceToDevice, st));
            gemm(ws, st, rows, m, b, Yp, b, 1, G, 1, b, tmp, m, 1);
            TTR_HIP(hipMemcpyAsync(Yp, tmp, (size_t)rows * m * sizeof(double), hipMemcpyDeviceToDevice, st));
            r[k - 1] = m;
        }
    }
    // 2. the bond threshold from ||Y_1||
    const double nrm = std::sqrt(sumsq(ws, st, Z, (int64_t)1, 0, (int)(r[0] * s.n[0] * r[1]), 1));
    const double tau = target ? -1.0 : tol * nrm / std::sqrt((double)(d - 1));
    info = RoundInfo{};
    info.tau = tau;
    info.nrmx = nrm;
    // 3. left-to-right truncation
    double* cur = Z;  // V(Y_k), row-major rows x b
    double* carry[2] = {ws.y1.as<double>(maxcore + 64), tmp};
    double* T = ws.q.as<double>(maxcore + 64);
    for (int k = 1; k < d; ++k) {
        const int b = (int)r[k];
        const int rows = (int)(r[k - 1] * s.n[k - 1]);
        const int tgt = target ? (int)target[k] : 0;
        int q;
        if (rows >= b) {
            launch_copy2d(cur, b, 1, T, 1, rows, rows, b, 1.0, st);  // to column-major
            qr_any(ws, st, T, rows, b, rows, R);
            q = b;
            svd_any(ws, st, R, b, b, q, G, Vs, sig, tau, tgt, tdev, true, false);
        } else {
            q = rows;  // V(Y_k)^T (b x rows) is the row-major buffer read column-major
            svd_any(ws, st, cur, b, b, q, G, Vs, sig, tau, tgt, tdev, false, false);
        }
        const int t = (tau >= 0.0) ? read_int(ws, st, tdev) : std::min(std::max(tgt, 1), q);
        if ((int64_t)rows * t > y.cap[k - 1])
            throw Error(-2, "output core " + std::to_string(k) + " needs " + std::to_string((int64_t)rows * t) +
                                " elements, capacity " + std::to_string(y.cap[k - 1]));
        if (rows >= b)
            gemm(ws, st, rows, t, b, T, 1, rows, Vs, 1, q, y.cores[k - 1], t, 1);  // Q W_t
        else
            launch_copy2d(Vs, 1, q, y.cores[k - 1], t, 1, rows, t, 1.0, st);  // W_t
        // H(Y_{k+1}) <- G_t^T H(Y_{k+1})
        const int64_t nr = s.n[k] * r[k + 1];
        double* nxt = carry[k & 1];
        gemm(ws, st, t, (int)nr, b, G, b, 1, Z + off[k], nr, 1, nxt, nr, 1);
        r[k] = t;
        y.ranks[k] = t;
        cur = nxt;
    }
    const int64_t last = r[d - 1] * s.n[d - 1];
    if (last > y.cap[d - 1]) throw Error(-2, "output core " + std::to_string(d) + " exceeds its capacity");
    TTR_HIP(hipMemcpyAsync(y.cores[d - 1], cur, (size_t)last * sizeof(double), hipMemcpyDeviceToDevice, st));
    y.ranks[0] = 1;
    y.ranks[d] = 1;
    y.orth = 1;
    TTR_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// Components
// ---------------------------------------------------------------------------
void gaussian_factor(uint64_t seed, int mode, int64_t n, int64_t col0, int64_t ncols, double* out,
                     hipStream_t st) {
    if (mode < 1 || n < 1 || ncols < 0 || col0 < 0 || !out) throw Error(-1, "bad Omega request");
    WsLease lease(st);
    int64_t* dn = lease->dn.as<int64_t>(2);
    int64_t* doff = lease->doff.as<int64_t>(2);
    const int64_t hn[2] = {n, 0}, ho[2] = {0, 0};
    TTR_HIP(hipMemcpyAsync(dn, hn, sizeof(hn), hipMemcpyHostToDevice, st));
    TTR_HIP(hipMemcpyAsync(doff, ho, sizeof(ho), hipMemcpyHostToDevice, st));
    OmegaArgs a{};
    a.seed = seed;
    a.first_mode = mode;
    a.n = dn;
    a.off = doff;
    a.base = out;
    a.ld = ncols;
    a.col0 = col0;
    a.store_col0 = 0;
    a.ncols = ncols;
    launch_omega(a, 1, n, st);
    TTR_HIP(hipStreamSynchronize(st));
}

void partial_contractions(const Shape& s, const double* const* cores, uint64_t seed, int64_t col0,
                          int64_t ncols, int t, int prec, double* const* w, hipStream_t st) {
    if (t < 2 || t > s.d) throw Error(-1, "t must be in [2, d]");
    if (ncols < 1 || col0 < 0) throw Error(-1, "bad column range");
    if (prec < 0 || prec > 2) throw Error(-6, "precision not supported for partial contractions");
    WsLease lease(st);
    Workspace& ws = *lease.ws;
    const Summands x = single_term(s, cores);
    Sketch sk(x, seed, prec, ncols, st, ws, col0);
    sk.pass(t, ncols);
    for (int k = t; k <= s.d; ++k)
        launch_w_export(prec, sk.wk(0, k), sk.cexp(0, k), sk.tw[0].ld[k], (int)s.r[k - 1], 0, (int)ncols,
                        sk.tw[0].sl[k], sk.tw[0].ss[k], w[k - t], ncols, st);
    TTR_HIP(hipStreamSynchronize(st));
}

// W^L_1..W^L_t of the left-to-right recurrence: Omega_1..Omega_t in one
// launch, then one fused contraction per core (lr.hip), each reading the
// previous core's output.
void partial_contractions_lr(const Shape& s, const double* const* cores, uint64_t seed, int64_t col0,
                             int64_t ncols, int t, double* const* w, hipStream_t st) {
    if (t < 1 || t > s.d) throw Error(-1, "t must be in [1, d]");
    if (ncols < 1 || col0 < 0) throw Error(-1, "bad column range");
    if (ncols > (int64_t)1 << 20) throw Error(-1, "column range too large");
    WsLease lease(st);
    Workspace& ws = *lease.ws;
    std::vector<int64_t> hn(t), ho(t);
    int64_t total = 0, maxn = 1;
    size_t part = 0;
    for (int k = 1; k <= t; ++k) {
        hn[k - 1] = s.n[k - 1];
        ho[k - 1] = total;
        total += s.n[k - 1] * ncols;
        maxn = std::max(maxn, s.n[k - 1]);
        const int sp = lr_splits((int)s.r[k - 1], (int)s.n[k - 1], (int)s.r[k], (int)ncols);
        if (sp > 1) part = std::max(part, (size_t)sp * s.r[k] * ncols);
    }
    int64_t* dn = ws.dn.as<int64_t>(t);
    int64_t* doff = ws.doff.as<int64_t>(t);
    TTR_HIP(hipMemcpyAsync(dn, hn.data(), t * sizeof(int64_t), hipMemcpyHostToDevice, st));
    TTR_HIP(hipMemcpyAsync(doff, ho.data(), t * sizeof(int64_t), hipMemcpyHostToDevice, st));
    double* om = ws.omega.as<double>(total);
    OmegaArgs oa{};
    oa.seed = seed;
    oa.first_mode = 1;
    oa.n = dn;
    oa.off = doff;
    oa.base = om;
    oa.ld = ncols;
    oa.col0 = col0;
    oa.store_col0 = 0;
    oa.ncols = ncols;
    launch_omega(oa, t, maxn, st);
    double* partials = part ? ws.part.as<double>(part) : nullptr;
    for (int k = 1; k <= t; ++k) {
        LrArgs g{};
        g.X = cores[k - 1];
        g.r0 = (int)s.r[k - 1];
        g.n = (int)s.n[k - 1];
        g.r1 = (int)s.r[k];
        g.Wp = k > 1 ? w[k - 2] : nullptr;
        g.ldw = ncols;
        g.Om = om + ho[k - 1];
        g.ldo = ncols;
        g.W = w[k - 1];
        g.ldwo = ncols;
        g.nc = (int)ncols;
        TimedScope ts(KT_PC, st);
        launch_lr(g, lr_splits(g.r0, g.n, g.r1, g.nc), partials, st);
    }
    TTR_HIP(hipStreamSynchronize(st));
}

void qr_inplace(double* a, int64_t m, int64_t b, hipStream_t st) {
    if (!a || m < 1 || b < 1) throw Error(-1, "bad QR request");
    if (m < b) throw Error(-1, "QR needs m >= b");
    if (b > svd_wide_max()) throw Error(-6, "QR wider than 512 columns is not supported");
    WsLease lease(st);
    qr_any(*lease.ws, st, a, (int)m, (int)b, (int)m);
    TTR_HIP(hipStreamSynchronize(st));
}

int64_t svd_small(const double* a, int64_t p, int64_t q, double* g, double* v, double* sig,
                  double tau, int64_t target, hipStream_t st) {
    if (!a || !g || !v || !sig || q < 1 || q > svd_wide_max() || p < q || p > (1 << 20))
        throw Error(-1, "bad SVD request");
    WsLease lease(st);
    int* tdev = lease->tint.as<int>(16);
    svd_any(*lease.ws, st, a, (int)p, (int)p, (int)q, g, v, sig, tau, (int)target, tdev, false, false);
    return read_int(*lease.ws, st, tdev);
}

// ---------------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------------
namespace {
struct TimingState {
    std::mutex mu;
    unsigned kinds = 0;  // bit k: record kind k
    struct Rec {
        hipEvent_t e0, e1;
        int launches;
    };
    std::vector<Rec> pending[KT_KINDS];
    std::vector<hipEvent_t> free_events;
    int64_t launches[KT_KINDS] = {0, 0, 0, 0};
    double ms[KT_KINDS] = {0, 0, 0, 0};
};
TimingState& timing() {
    static TimingState* t = new TimingState();  // kept until process exit
    return *t;
}
// Resolve the recorded pairs of one kind into the totals (caller holds mu).
void drain(TimingState& t, int kind) {
    for (auto& pr : t.pending[kind]) {
        TTR_HIP(hipEventSynchronize(pr.e1));
        float ms = 0.f;
        TTR_HIP(hipEventElapsedTime(&ms, pr.e0, pr.e1));
        t.ms[kind] += ms;
        t.launches[kind] += pr.launches;
        t.free_events.push_back(pr.e0);
        t.free_events.push_back(pr.e1);
    }
    t.pending[kind].clear();
}
// An event from the pool or a new one; nullptr if creation fails.
hipEvent_t take_event(TimingState& t) {
    if (!t.free_events.empty()) {
        hipEvent_t e = t.free_events.back();
        t.free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}
}  // namespace

void timing_enable(unsigned kinds) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (kinds) {
        for (int k = 0; k < KT_KINDS; ++k) {
            drain(t, k);
            t.launches[k] = 0;
            t.ms[k] = 0.0;
        }
    }
    t.kinds = kinds;
}

void timing_read(int kind, int64_t* launches, double* total_ms) {
    if (kind < 0 || kind >= KT_KINDS) throw Error(-1, "unknown kernel kind");
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    drain(t, kind);
    *launches = t.launches[kind];
    *total_ms = t.ms[kind];
}

namespace {
// Set while an allocation-free rounding runs on this thread: its launches
// are not timed (recording them would create events).
thread_local bool t_timing_off = false;
}  // namespace

TimingPause::TimingPause() : prev_(t_timing_off) { t_timing_off = true; }
TimingPause::~TimingPause() { t_timing_off = prev_; }

TimedScope::TimedScope(int kind, hipStream_t s, int launches)
    : kind_(kind), s_(s), launches_(launches) {
    if (t_timing_off) return;
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!((t.kinds >> kind) & 1u)) return;
    e0_ = take_event(t);
    if (e0_ && hipEventRecord(e0_, s_) != hipSuccess) {
        (void)hipGetLastError();
        t.free_events.push_back(e0_);
        e0_ = nullptr;
    }
}

TimedScope::~TimedScope() {
    if (!e0_) return;
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    hipEvent_t e1 = take_event(t);
    if (!e1 || hipEventRecord(e1, s_) != hipSuccess) {
        (void)hipGetLastError();
        t.free_events.push_back(e0_);
        if (e1) t.free_events.push_back(e1);
        return;
    }
    t.pending[kind_].push_back(TimingState::Rec{e0_, e1, launches_});
}

}  // namespace ttr
