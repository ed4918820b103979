// The library's one static scratch array (for kw_create_static): the six
// spectral scratch arrays of a simulation whose caller cannot allocate them.
// Each GPU the library runs on holds its own copy of the array, at its own
// address, until the process ends.  Host code never uses the array's name as
// a device address: the address is taken once per device with
// hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kw_internal.h"

namespace kw {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_addr[kMaxDevices];
}  // namespace

// Device address of the scratch array on the current device (looked up on
// the first call for that device).
hipError_t static_scratch(void **out, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

}  // namespace kw
