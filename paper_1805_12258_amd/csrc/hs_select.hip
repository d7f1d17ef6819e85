// Per-plane capped candidate lists (Sec. III: the module returns at most
// N_cand candidates for each of the N_hp planes).  Policy: the N_cand
// largest powers of each plane, ties to the smaller CL1 word, listed in that
// order.  Powers are ordered by the IEEE total order of their bits (-0 below
// +0).
//
// Two stable radix passes over a copy of the list: by CL1 word, then by
// (plane, descending power); the first N_cand entries of each plane's run
// are copied out.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "hs_internal.h"

namespace hsk {

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kSelThreads = 256;

// Descending order of fp32 bits as an ascending unsigned key.
__device__ __forceinline__ uint32_t desc_power_key(uint32_t b)
{
    const uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ~asc;
}

// Sort keys of the second pass and the per-plane counts (counted per block
// in LDS, then one global atomic per block and plane: a global atomic per
// entry would serialise on the few counters).
__global__ __launch_bounds__(kSelThreads) void k_sel_keys(const uint64_t* __restrict__ rec, int64_t n, int s_bin,
                                                          uint32_t kmask, uint64_t* __restrict__ key,
                                                          unsigned long long* __restrict__ cnt)
{
    __shared__ unsigned int hist[kMaxH];
    if (threadIdx.x < kMaxH) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSelThreads) {
        const uint64_t w = rec[i];
        const uint32_t k1 = ((uint32_t)w >> s_bin) & kmask;       // plane - 1 (kmask < kMaxH)
        key[i] = ((uint64_t)k1 << 32) | desc_power_key((uint32_t)(w >> 32));
        atomicAdd(&hist[k1], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kMaxH && hist[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
}

__global__ __launch_bounds__(kSelThreads) void k_sel_copy(const uint64_t* __restrict__ sorted,
                                                          const unsigned long long* __restrict__ cnt, int H,
                                                          int n_cand, uint64_t* __restrict__ out,
                                                          int64_t* __restrict__ out_counts)
{
    const int64_t total = (int64_t)H * n_cand;
    for (int64_t e = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kSelThreads) {
        const int k = (int)(e / n_cand);
        const int64_t i = e - (int64_t)k * n_cand;
        int64_t off = 0;
        for (int q = 0; q < k; ++q) off += (int64_t)cnt[q];
        const int64_t c = (int64_t)cnt[k];
        if (i < c) out[e] = sorted[off + i];
        if (i == 0) out_counts[k] = c < n_cand ? c : n_cand;
    }
}

int sel_grid(int64_t n)
{
    const int64_t b = (n + kSelThreads - 1) / kSelThreads;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

struct SelLayout {
    size_t rec_b, key_a, key_b, cnt, temp, total, temp_bytes;
};

hipError_t sel_layout(int64_t n, int end_bit, SelLayout& L)
{
    size_t t1 = 0, t2 = 0;
    rocprim::double_buffer<uint64_t> kb(nullptr, nullptr), vb(nullptr, nullptr);
    hipError_t e = rocprim::radix_sort_keys(nullptr, t1, kb, (size_t)n, 0, 32);
    if (e != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(nullptr, t2, kb, vb, (size_t)n, 0, end_bit);
    if (e != hipSuccess) return e;
    const size_t nb = align_up((size_t)n * 8);
    L.rec_b = nb;                 // record copy A at 0, B here
    L.key_a = 2 * nb;
    L.key_b = 3 * nb;
    L.cnt = 4 * nb;
    L.temp = L.cnt + align_up(kMaxH * 8);
    L.temp_bytes = t1 > t2 ? t1 : t2;
    L.total = L.temp + L.temp_bytes;
    return hipSuccess;
}

}  // namespace

hipError_t select_workspace(int64_t n, int end_bit, size_t* bytes)
{
    SelLayout L;
    const hipError_t e = sel_layout(n, end_bit, L);
    *bytes = L.total;
    return e;
}

hipError_t select_top(const uint64_t* cand, int64_t n, int H, int s_bin, int s_k, int n_cand, uint64_t* out,
                      int64_t* out_counts, void* work, hipStream_t s)
{
    const int end_bit = 32 + s_k;
    SelLayout L;
    hipError_t e = sel_layout(n, end_bit, L);
    if (e != hipSuccess) return e;
    char* w = static_cast<char*>(work);
    uint64_t* rec_a = reinterpret_cast<uint64_t*>(w);
    uint64_t* rec_b = reinterpret_cast<uint64_t*>(w + L.rec_b);
    uint64_t* key_a = reinterpret_cast<uint64_t*>(w + L.key_a);
    uint64_t* key_b = reinterpret_cast<uint64_t*>(w + L.key_b);
    int64_t* cnt = reinterpret_cast<int64_t*>(w + L.cnt);
    void* temp = w + L.temp;
    size_t temp_bytes = L.temp_bytes;

    e = launch_zero_i64(cnt, kMaxH, s);
    if (e != hipSuccess) return e;
    const uint64_t* sorted = rec_a;
    if (n > 0) {
        e = hipMemcpyAsync(rec_a, cand, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        rocprim::double_buffer<uint64_t> rb(rec_a, rec_b);
        e = rocprim::radix_sort_keys(temp, temp_bytes, rb, (size_t)n, 0, 32, s);   // by CL1 word
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sel_keys, dim3(sel_grid(n)), dim3(kSelThreads), 0, s, rb.current(), n, s_bin,
                           (uint32_t)((1u << s_k) - 1u), key_a,
                           reinterpret_cast<unsigned long long*>(cnt));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        rocprim::double_buffer<uint64_t> kb(key_a, key_b);
        rocprim::double_buffer<uint64_t> vb(rb.current(), rb.current() == rec_a ? rec_b : rec_a);
        temp_bytes = L.temp_bytes;
        e = rocprim::radix_sort_pairs(temp, temp_bytes, kb, vb, (size_t)n, 0, end_bit, s);   // stable
        if (e != hipSuccess) return e;
        sorted = vb.current();
    }
    hipLaunchKernelGGL(k_sel_copy, dim3(sel_grid((int64_t)H * n_cand)), dim3(kSelThreads), 0, s, sorted,
                       reinterpret_cast<const unsigned long long*>(cnt), H, n_cand, out, out_counts);
    return hipGetLastError();
}

}  // namespace hsk
