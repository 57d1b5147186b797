// noalloc.hip -- the static device scratch behind ccmg_vcycle_noalloc.
//
// A fixed array in device memory, one copy per device, held from the moment
// the library's code is loaded on that device until the process ends.  Host
// code never uses the array's name as an address (on the host it is only a
// stand-in for the symbol): the device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and kept.
#include <mutex>

#include "internal.h"

namespace ccmg {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int dev, void **ptr, size_t *bytes) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

}  // namespace ccmg
