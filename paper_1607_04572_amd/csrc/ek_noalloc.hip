// ek_noalloc.hip -- fixed device scratch of the allocation-free step
// (ek_step_noalloc): the per-(particle, chunk) partial sums of the particle
// kernels, in a file-scope device array instead of the context's arena.
//
// The array exists once per GPU the library runs on, for the life of the
// process.  Host code cannot use its name as a device address: the address is
// resolved once per device with hipGetSymbolAddress (with that device
// current) and kept in a per-device table.  Every allocation-free step on a
// GPU uses the same array, so such calls must not overlap on one GPU.
#include <mutex>

#include "ek_internal.h"

namespace ek {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};
std::mutex g_scratch_mu;
}  // namespace

// Device address of the current device's scratch array (resolved on the
// first call on that device).  Returns hipSuccess or the HIP error.
hipError_t noalloc_scratch(void** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace ek
