// Canonical order of a candidate list: ascending CL1 word (row, then plane,
// then bin), i.e. a stable radix sort of the 8-byte entries on their low
// 32 bits (the power in the high half travels with its word).
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "hs_internal.h"

namespace hsk {

namespace {
size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
}

hipError_t sort_workspace(int64_t n, size_t* bytes)
{
    size_t temp = 0;
    rocprim::double_buffer<uint64_t> kb(nullptr, nullptr);
    hipError_t e = rocprim::radix_sort_keys(nullptr, temp, kb, (size_t)n, 0, 32);
    *bytes = align_up((size_t)n * 8) + temp;
    return e;
}

hipError_t sort_candidates(uint64_t* cand, int64_t n, void* work, hipStream_t s)
{
    if (n <= 1) return hipSuccess;
    uint64_t* alt = static_cast<uint64_t*>(work);
    void* temp = static_cast<char*>(work) + align_up((size_t)n * 8);
    size_t temp_bytes = 0;
    rocprim::double_buffer<uint64_t> kb(cand, alt);
    hipError_t e = rocprim::radix_sort_keys(nullptr, temp_bytes, kb, (size_t)n, 0, 32, s);
    if (e != hipSuccess) return e;
    e = rocprim::radix_sort_keys(temp, temp_bytes, kb, (size_t)n, 0, 32, s);
    if (e != hipSuccess) return e;
    if (kb.current() != cand)
        e = hipMemcpyAsync(cand, kb.current(), (size_t)n * 8, hipMemcpyDeviceToDevice, s);
    return e;
}

}  // namespace hsk
