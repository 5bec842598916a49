// Allocation-free fixed-rank rounding: tt_round_fixed with every device
// buffer carved from one file-scope device array instead of the library's
// workspace pool (which grows with hipMalloc).
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that address is handed to kernels.  Each
// GPU holds its own copy of the array until the process ends; every call on
// a GPU reuses it, so calls are serialised per device by a mutex here (two
// processes have separate copies).  Whatever a rounding needs zeroed
// (QR tree counters, reduction counters) is cleared by a fill kernel at the
// start of each call, since the array keeps the previous call's contents.
#include <mutex>

#include "../../include/ttround.h"
#include "runtime.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)TT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_addr_mu;
void* g_addr[kMaxDevices] = {};
std::mutex g_call_mu[kMaxDevices];

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current: the caller's current device).
void* scratch_address(int dev) {
    std::lock_guard<std::mutex> lk(g_addr_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw ttr::Error(TT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_addr[dev] = p;
    }
    return g_addr[dev];
}

}  // namespace

namespace ttr {

void round_fixed_noalloc(const Shape& s, const double* const* cores, const int64_t* target,
                         int64_t ell, uint64_t seed, const Options& o, OutCores& y, RoundInfo& info) {
    // the workspace estimate bounds what the carves below can take; a request
    // over the limit is refused before anything is queued
    const size_t need = workspace_bytes(s, ell, o.prec);
    if (need > kScratchBytes)
        throw Error(TT_ENOMEM, "allocation-free rounding needs up to " + std::to_string(need) +
                                   " bytes of scratch; the limit is " + std::to_string(kScratchBytes));
    int dev = 0;
    TTR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(TT_EUNSUPPORTED, "device index out of range");
    void* base = scratch_address(dev);
    std::lock_guard<std::mutex> lk(g_call_mu[dev]);
    round_fixed_in(base, kScratchBytes, s, cores, target, ell, seed, o, y, info);
}

}  // namespace ttr
