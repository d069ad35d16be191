// noalloc.hip -- device scratch of the allocation-free entry point
// (empp_fields_at_dev_noalloc): the per-chunk field partials of its pair
// pass live in a fixed file-scope device array instead of memory the
// library or the caller allocates.
#include "empp_dev.h"

#include <mutex>

namespace empp {

// 128 MiB on every GPU the library runs on, held until the process ends.
constexpr size_t kScratchBytes = size_t(128) << 20;

// The partials of a call fill it from the start and are overwritten in full
// by the call's pair pass (every target writes every chunk's 12 values), so
// nothing needs clearing between calls.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Device address of `device`'s copy of the scratch array.  In host code the
// array's name is only a stand-in, so its address is taken once per device
// with hipGetSymbolAddress while that device is current, and cached; the
// caller's current device is restored.
hipError_t noalloc_scratch(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices || !out)
        return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess)
            return e;
        if ((e = hipSetDevice(device)) != hipSuccess)
            return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess)
            return e;
        if (e2 != hipSuccess)
            return e2;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace empp
