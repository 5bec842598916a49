// Host side of the persistent batched rounding (batch.hip): validation,
// team sizes, the workspace layout of every tensor, the descriptor upload
// and the result readback.
#include "batch_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>

namespace ttr {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Flops of one rounding of this shape by the model of Sec. 3.1 and the
// sweep (partial contractions and next cores with the full sketch, the
// residual projections and QRs): used only to size teams.
double tensor_flops(const Shape& s, const std::vector<int64_t>& cap, int64_t lcap) {
    double f = 0.0;
    const int d = s.d;
    for (int k = 1; k <= d; ++k) {
        const double core = (double)s.r[k - 1] * s.n[k - 1] * s.r[k];
        f += 2.0 * core * (double)lcap;  // partial contraction
        if (k >= 2) f += 2.0 * (double)cap[k - 1] * (double)s.r[k - 1] * (double)s.n[k - 1] * (double)s.r[k];  // next core
        const double rows = (double)cap[k - 1] * s.n[k - 1];
        f += 2.0 * rows * (double)s.r[k] * (double)cap[k];     // sketches and projection
        f += 6.0 * rows * (double)cap[k] * (double)cap[k];     // residual projections and QRs
    }
    return f;
}

}  // namespace

namespace {
std::mutex g_tune_mu;
constexpr int kTuneDevices = 64;
double g_tuned[kTuneDevices] = {};
bool g_cache_read[kTuneDevices] = {};

double env_team_flops() {
    const char* e = std::getenv("TTR_BATCH_TEAM_FLOPS");
    const double x = e ? std::atof(e) : 0.0;
    return x > 0.0 ? x : 3.0e9;
}

int tune_device() {
    int dev = 0;
    TTR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kTuneDevices) throw Error(-6, "device index out of range");
    return dev;
}

// The last entry for `key` in the cache file, or 0.
double cache_lookup(const std::string& key) {
    const char* path = std::getenv("TTR_BATCH_TUNE_CACHE");
    if (!path || !*path) return 0.0;
    std::ifstream f(path);
    double v = 0.0;
    std::string k;
    double x = 0.0;
    while (f >> k >> x)
        if (k == key && x > 0.0) v = x;
    return v;
}
}  // namespace

std::string batch_device_key() {
    int dev = tune_device();
    hipDeviceProp_t p;
    TTR_HIP(hipGetDeviceProperties(&p, dev));
    std::string arch(p.gcnArchName);
    for (char& c : arch)
        if (c == ' ') c = '_';
    return arch + "/" + std::to_string(p.multiProcessorCount);
}

double batch_team_flops() {
    const int dev = tune_device();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tuned[dev] > 0.0) return g_tuned[dev];
        if (g_cache_read[dev]) return env_team_flops();
    }
    const double v = cache_lookup(batch_device_key());
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_cache_read[dev] = true;
    if (v > 0.0 && !(g_tuned[dev] > 0.0)) g_tuned[dev] = v;
    return g_tuned[dev] > 0.0 ? g_tuned[dev] : env_team_flops();
}

void set_batch_team_flops(double v) {
    const int dev = tune_device();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[dev] = v > 0.0 ? v : 0.0;
    if (!(v > 0.0)) g_cache_read[dev] = false;
}

void save_batch_team_flops(double v) {
    const char* path = std::getenv("TTR_BATCH_TUNE_CACHE");
    if (!path || !*path || !(v > 0.0)) return;
    const std::string key = batch_device_key();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ofstream f(path, std::ios::app);
    f.precision(17);
    f << key << " " << v << "\n";
    if (!f) throw Error(-1, std::string("cannot write the tuning cache ") + path);
}

// Per-tensor sizes (doubles unless stated) of the workspace regions.
struct TensorLayout {
    Shape s;
    std::vector<int64_t> cap;
    int64_t lcap = 1, r0 = 1, rmax = 1, maxrows = 1, maxy = 1, pslot = 1, privs = 1;
    int T = 1;
    double flops = 0.0;
    size_t bytes = 0;  // total, aligned regions
    std::vector<int64_t> ooff, woff;
    int64_t om = 0, w = 0;
};

static TensorLayout layout_of(const Shape& s, int64_t ell_block, double f_init, int tmax, double f0) {
    TensorLayout L;
    L.s = s;
    const int d = s.d;
    L.cap = rank_caps(s);
    for (int k = 1; k < d; ++k) {
        L.rmax = std::max(L.rmax, s.r[k]);
        L.lcap = std::max(L.lcap, L.cap[k]);
    }
    L.r0 = (int64_t)std::ceil(f_init * (double)L.rmax);
    L.lcap = std::max(L.lcap, L.r0);
    int64_t bmax = 1;
    for (int k = 1; k < d; ++k) {
        const int64_t rb = L.cap[k];
        const int64_t bi = (int64_t)std::ceil(f_init * (double)rb);
        const int64_t bl = ell_block > 0 ? ell_block : (int64_t)std::ceil(0.05 * (double)rb);
        bmax = std::max({bmax, bi, bl});
    }
    if (std::min(bmax, L.lcap) > kBatchMaxBlock)
        throw Error(-6, "batched rounding: sketch blocks wider than 64 are not supported");
    for (int k = 1; k <= d; ++k) {
        L.maxrows = std::max(L.maxrows, L.cap[k - 1] * s.n[k - 1]);
        if (k >= 2) L.maxy = std::max(L.maxy, L.cap[k - 1] * s.n[k - 1] * s.r[k]);
    }
    if (L.maxrows * L.lcap > ((int64_t)1 << 31) || L.maxy > ((int64_t)1 << 31))
        throw Error(-6, "batched rounding: a sketch panel exceeds 2^31 elements");
    L.ooff.assign(d + 1, 0);
    L.woff.assign(d + 1, 0);
    for (int j = 2; j <= d; ++j) {
        L.ooff[j] = L.om;
        L.om += s.n[j - 1] * L.lcap;
        L.woff[j] = L.w;
        L.w += s.r[j - 1] * L.lcap;
    }
    L.flops = tensor_flops(s, L.cap, L.lcap);
    int T = 1;
    while (T < tmax && (double)(2 * T) * f0 <= L.flops) T *= 2;
    L.T = T;
    L.pslot = std::max<int64_t>(L.lcap * std::max<int64_t>(L.rmax, kBatchMaxBlock), 16);
    L.privs = kBatchPrivRinv + L.lcap * kBatchMaxBlock;
    size_t b = 0;
    b += align_up(L.om * 8);                               // Omega
    b += align_up(L.w * 8);                                // W
    b += align_up(L.maxrows * L.lcap * 8);                 // Q
    b += 2 * align_up(L.maxy * 8);                         // ping-pong cores
    b += align_up(L.lcap * L.rmax * 8);                    // M
    b += align_up(2 * (size_t)T * L.pslot * 8);            // partial slots
    b += align_up((size_t)T * L.privs * 8);                // member-private
    b += align_up(L.maxrows * kBatchMaxBlock * 8);         // Householder reflectors
    b += align_up((size_t)(5 * (d + 1)) * 8);              // n, r, ooff, woff, ranks
    b += align_up((size_t)(2 * d) * sizeof(void*));        // X, Y pointers
    b += align_up(kBatchInfo * 8);                         // run record
    L.bytes = b;
    return L;
}

int batch_team_cap() {
    static const int v = [] { return std::max(1, std::min(32, batch_resident_workgroups() / 2)); }();
    return v;
}

static size_t header_bytes(int count) {
    size_t b = 0;
    b += align_up((size_t)count * sizeof(BatchTT));
    b += align_up((size_t)count * sizeof(int));         // order
    b += align_up((size_t)(count + 1) * sizeof(int));   // prefix
    b += align_up((size_t)(1 + 3 * count) * sizeof(unsigned));  // ticket, barriers, statuses
    return b;
}

size_t batch_workspace_bytes(const std::vector<Shape>& sh, int64_t ell_block, double f_init, double team_flops) {
    const int tmax = batch_team_cap();
    const double f0 = team_flops > 0.0 ? team_flops : batch_team_flops();
    size_t b = header_bytes((int)sh.size());
    for (const Shape& s : sh) b += layout_of(s, ell_block, f_init, tmax, f0).bytes;
    return b;
}

void BatchPlan::create(const std::vector<Shape>& sh, const std::vector<const double* const*>& cores,
                       const std::vector<double>& tol, int64_t ell_block, const std::vector<uint64_t>& seeds,
                       const Options& o, const std::vector<OutCores>& outs, void* ws, size_t ws_bytes,
                       double team_flops) {
    count = (int)sh.size();
    if (count < 1) throw Error(-1, "a batch needs at least one tensor");
    if (o.prec != 0) throw Error(-6, "batched rounding runs with a float64 sketch only");
    if (o.recompress) throw Error(-6, "batched rounding has no recompression pass");
    const double f_init = (o.f_init > 0.0) ? o.f_init : 0.1;
    const int tmax = batch_team_cap();
    const double f0 = team_flops > 0.0 ? team_flops : batch_team_flops();
    std::vector<TensorLayout> L;
    L.reserve(count);
    for (int i = 0; i < count; ++i) L.push_back(layout_of(sh[i], ell_block, f_init, tmax, f0));
    size_t need = header_bytes(count);
    for (const auto& l : L) need += l.bytes;
    if (!ws || ws_bytes < need)
        throw Error(-2, "batch workspace too small: " + std::to_string(need) + " bytes needed");
    for (int i = 0; i < count; ++i) {
        const Shape& s = sh[i];
        for (int k = 1; k <= s.d; ++k) {
            const int64_t c = L[i].cap[k - 1] * s.n[k - 1] * L[i].cap[k];
            if (outs[i].cap[k - 1] < c)
                throw Error(-2, "tensor " + std::to_string(i) + ": output core " + std::to_string(k) +
                                    " needs " + std::to_string(c) + " elements");
        }
    }
    // processing order: largest first (ties by index)
    order.resize(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L[a].flops > L[b].flops; });
    prefix.assign(count + 1, 0);
    for (int t = 0; t < count; ++t) prefix[t + 1] = prefix[t] + L[order[t]].T;
    team.resize(count);
    for (int i = 0; i < count; ++i) team[i] = L[i].T;
    shapes = sh;

    // carve the workspace
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off += align_up(bytes);
        return p;
    };
    d_tts = reinterpret_cast<BatchTT*>(take((size_t)count * sizeof(BatchTT)));
    d_order = reinterpret_cast<int*>(take((size_t)count * sizeof(int)));
    d_prefix = reinterpret_cast<int*>(take((size_t)(count + 1) * sizeof(int)));
    d_zero = reinterpret_cast<unsigned*>(take((size_t)(1 + 3 * count) * sizeof(unsigned)));
    zwords = 1 + 3 * (int64_t)count;
    std::vector<BatchTT> tts(count);
    struct Upload {
        void* dst;
        std::vector<char> bytes;
    };
    std::vector<Upload> ups;
    ranks_dev.assign(count, nullptr);
    info_dev.assign(count, nullptr);
    d_of.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        const TensorLayout& l = L[i];
        const Shape& s = l.s;
        const int d = s.d;
        BatchTT& t = tts[i];
        std::memset(&t, 0, sizeof(t));
        t.d = d;
        t.T = l.T;
        t.ell_block = (int)ell_block;
        t.lcap = (int)l.lcap;
        t.r0 = (int)l.r0;
        // Every sketch column the rounding may use is drawn in the first
        // right-to-left pass: a column's values do not depend on the pass
        // that makes it, so the result is the same as with regeneration on
        // demand, and the cores are read once instead of once per pass.
        t.init_cols = (int)l.lcap;
        t.has_nrmx = o.nrmx > 0.0 ? 1 : 0;
        t.tol = tol[i];
        t.nrmx = o.nrmx;
        t.f_init = f_init;
        t.seed = seeds[i];
        t.om = reinterpret_cast<double*>(take(l.om * 8));
        t.w = reinterpret_cast<double*>(take(l.w * 8));
        t.q = reinterpret_cast<double*>(take(l.maxrows * l.lcap * 8));
        t.yb[0] = reinterpret_cast<double*>(take(l.maxy * 8));
        t.yb[1] = reinterpret_cast<double*>(take(l.maxy * 8));
        t.m = reinterpret_cast<double*>(take(l.lcap * l.rmax * 8));
        t.slots = reinterpret_cast<double*>(take(2 * (size_t)l.T * l.pslot * 8));
        t.pslot = l.pslot;
        t.priv = reinterpret_cast<double*>(take((size_t)l.T * l.privs * 8));
        t.privs = l.privs;
        t.hh = reinterpret_cast<double*>(take(l.maxrows * kBatchMaxBlock * 8));
        int64_t* tab = reinterpret_cast<int64_t*>(take((size_t)(5 * (d + 1)) * 8));
        void** ptrs = reinterpret_cast<void**>(take((size_t)(2 * d) * sizeof(void*)));
        double* info = reinterpret_cast<double*>(take(kBatchInfo * 8));
        t.n = tab;
        t.r = tab + (d + 1);
        t.ooff = tab + 2 * (d + 1);
        t.woff = tab + 3 * (d + 1);
        t.ranks = tab + 4 * (d + 1);
        t.X = reinterpret_cast<const double* const*>(ptrs);
        t.Y = reinterpret_cast<double* const*>(ptrs + d);
        t.bar = d_zero + 1 + 2 * i;
        t.status = reinterpret_cast<int*>(d_zero + 1 + 2 * count + i);
        t.info = info;
        ranks_dev[i] = t.ranks;
        info_dev[i] = info;
        d_of[i] = d;
        // table contents
        Upload u1;
        u1.dst = tab;
        u1.bytes.resize((size_t)(5 * (d + 1)) * 8, 0);
        int64_t* h = reinterpret_cast<int64_t*>(u1.bytes.data());
        for (int k = 0; k < d; ++k) h[k] = s.n[k];
        for (int k = 0; k <= d; ++k) {
            h[(d + 1) + k] = s.r[k];
            h[2 * (d + 1) + k] = l.ooff[k];
            h[3 * (d + 1) + k] = l.woff[k];
        }
        ups.push_back(std::move(u1));
        Upload u2;
        u2.dst = ptrs;
        u2.bytes.resize((size_t)(2 * d) * sizeof(void*));
        const void** hp = reinterpret_cast<const void**>(u2.bytes.data());
        for (int k = 0; k < d; ++k) {
            hp[k] = cores[i][k];
            hp[d + k] = outs[i].cores[k];
        }
        ups.push_back(std::move(u2));
    }
    if (off > ws_bytes) throw Error(-2, "batch workspace layout overflow");
    bytes_used = off;
    hipStream_t st = o.stream;
    TTR_HIP(hipMemcpyAsync(d_tts, tts.data(), (size_t)count * sizeof(BatchTT), hipMemcpyHostToDevice, st));
    TTR_HIP(hipMemcpyAsync(d_order, order.data(), (size_t)count * sizeof(int), hipMemcpyHostToDevice, st));
    TTR_HIP(hipMemcpyAsync(d_prefix, prefix.data(), (size_t)(count + 1) * sizeof(int), hipMemcpyHostToDevice, st));
    for (auto& u : ups) TTR_HIP(hipMemcpyAsync(u.dst, u.bytes.data(), u.bytes.size(), hipMemcpyHostToDevice, st));
    TTR_HIP(hipStreamSynchronize(st));
    grid = std::min(batch_resident_workgroups(), std::max(1, prefix[count]));
}

void BatchPlan::pc_work(int i, const std::vector<double>& info, int64_t& cores, double& bytes,
                        double& flops) const {
    const Shape& s = shapes[i];
    const int d = s.d;
    cores = 0;
    bytes = flops = 0.0;
    const int passes = std::min<int>((int)info[3], kBatchMaxPasses);
    for (int p = 0; p < passes; ++p) {
        const int k1 = (int)info[8 + 2 * p];
        const double nc = info[9 + 2 * p];
        for (int k = k1; k <= d; ++k) {
            const double r0 = (double)s.r[k - 1], nk = (double)s.n[k - 1], r1 = (double)s.r[k];
            bytes += 8.0 * r0 * nk * r1 + 8.0 * r0 * nc;
            flops += 2.0 * r0 * nk * r1 * nc + (k < d ? 2.0 * r0 * r1 * nc : 0.0);
            ++cores;
        }
    }
}

void BatchPlan::launch(hipStream_t st) const {
    launch_batch(d_tts, d_order, d_prefix, count, d_zero, d_zero, zwords, grid, st);
}

void BatchPlan::results(hipStream_t st, std::vector<std::vector<int64_t>>& ranks,
                        std::vector<std::vector<double>>& info, std::vector<int>& status) const {
    ranks.assign(count, {});
    info.assign(count, {});
    status.assign(count, 0);
    std::vector<unsigned> z((size_t)zwords);
    TTR_HIP(hipMemcpyAsync(z.data(), d_zero, (size_t)zwords * sizeof(unsigned), hipMemcpyDeviceToHost, st));
    for (int i = 0; i < count; ++i) {
        ranks[i].resize(d_of[i] + 1);
        info[i].resize(kBatchInfo);
        TTR_HIP(hipMemcpyAsync(ranks[i].data(), ranks_dev[i], (d_of[i] + 1) * sizeof(int64_t),
                               hipMemcpyDeviceToHost, st));
        TTR_HIP(hipMemcpyAsync(info[i].data(), info_dev[i], kBatchInfo * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    TTR_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) status[i] = (int)z[1 + 2 * count + i];
}

}  // namespace ttr
