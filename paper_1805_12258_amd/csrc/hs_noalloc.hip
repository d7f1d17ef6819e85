// Device scratch for the entry points that allocate nothing: a file-scope
// device array (one copy per GPU, held until the process ends) whose
// address is looked up once per device with that device current.  Host
// code uses only the looked-up address, never the array's name.  Every
// call on a GPU shares that GPU's copy: calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hs_internal.h"

namespace hsk {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_mu;
void* g_ptr[64] = {nullptr};
}  // namespace

hipError_t noalloc_scratch(void** ptr)
{
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace hsk
