// Staging memory of the read entry point that allocates nothing
// (tcm_read_noalloc): a file-scope device array, one copy per GPU, looked up
// once per device with hipGetSymbolAddress.  The kernels only ever receive
// the device address returned by that lookup, never the array's host-side
// name.
#include "tcm_internal.h"

#include <mutex>

namespace tcmk {

// 32 MiB: the box of a read through the no-allocation entry point holds at
// most NOALLOC_FLOATS floats.
__device__ __align__(256) float noalloc_scratch[NOALLOC_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
}  // namespace

// Device address of this device's copy of the staging array (the calling
// thread's current device).  Looked up on the first call for each device
// and kept for the life of the process.
hipError_t noalloc_staging(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = (float*)g_ptr[dev];
    return hipSuccess;
}

}  // namespace tcmk
