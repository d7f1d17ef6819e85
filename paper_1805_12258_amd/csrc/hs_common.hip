// Dtype-independent parts of the fused kernels: LDS sizing, dispatch on the
// storage type, the counter-clearing kernel and the per-plane counting pass.
#include <hip/hip_runtime.h>

#include "hs_internal.h"

namespace hsk {

#define HS_DECL_GROUP(n, g)                                                                     \
    hipError_t launch_fused_##n##_g##g(int mode, int H, const TileArgs& a, int64_t nt, int grid,  \
                                       int lds, hipStream_t s);                                  \
    hipError_t launch_batched_##n##_g##g(int H, const BatchArgs& b, int grid, int lds, hipStream_t s);
#define HS_DECL_TYPE(n) HS_DECL_GROUP(n, 0) HS_DECL_GROUP(n, 1) HS_DECL_GROUP(n, 2) HS_DECL_GROUP(n, 3)
HS_DECL_TYPE(f32)
HS_DECL_TYPE(f16)
HS_DECL_TYPE(bf16)
#define HS_DECL_STAT(g)                                                                          \
    hipError_t launch_stat_f32_g##g(int mode, int H, const TileArgs& a, int64_t nt, int grid,     \
                                    int lds, hipStream_t s);
HS_DECL_STAT(0)
HS_DECL_STAT(1)
HS_DECL_STAT(2)
HS_DECL_STAT(3)

__global__ void k_zero_i64(int64_t* p, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0;
}

// Per-plane counts of the candidates a detection stored.  The detection
// kernels reserve list positions with one atomic per flush and count per
// plane only the entries dropped for lack of capacity; this pass adds a
// histogram of the plane field over the first min(total, capacity) entries
// of each list.  Grid (x, lists); a list whose total is ~0 (a FOP the
// batched detection rejected) is left as it is.  The list is short (a few
// MB at most) and latency-bound: each thread keeps kPcU loads in flight (48
// blocks cover 384 K entries in one round), every entry is one LDS atomic on
// the block's histogram, and each block adds its H counts with one global
// atomic per plane.
constexpr int kPcThreads = 1024;
constexpr int kPcU = 8;
constexpr int kPcMaxBlocks = 48;

__global__ __launch_bounds__(kPcThreads) void k_plane_counts(const uint64_t* out, const int64_t* out_offsets,
                                                             const int64_t* caps, int64_t cap1,
                                                             unsigned long long* counts, int H, int s_bin,
                                                             uint32_t kmask)
{
    __shared__ unsigned int hist[kMaxH];
    const int f = blockIdx.y;
    const uint64_t* o = out + (out_offsets ? out_offsets[f] : 0);
    const int64_t cap = caps ? caps[f] : cap1;
    unsigned long long* c = counts + (int64_t)f * (H + 1);
    const unsigned long long tot = c[H];   // the same for the whole block
    if (tot == ~0ull) return;
    const int64_t n = (int64_t)tot < cap ? (int64_t)tot : cap;
    if (threadIdx.x < kMaxH) hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kPcThreads;
    for (int64_t e0 = blockIdx.x * (int64_t)kPcThreads + threadIdx.x; e0 < n; e0 += stride * kPcU) {
        // unconditional loads (indexes clamped into the list), so that all
        // kPcU are in flight together; entries past the end are not counted
        uint32_t w[kPcU];
#pragma unroll
        for (int u = 0; u < kPcU; ++u) {
            const int64_t e = e0 + u * stride;
            w[u] = (uint32_t)o[e < n ? e : n - 1];
        }
#pragma unroll
        for (int u = 0; u < kPcU; ++u)
            if (e0 + u * stride < n) atomicAdd(&hist[(w[u] >> s_bin) & kmask], 1u);
    }
    __syncthreads();
    if (threadIdx.x < H && hist[threadIdx.x]) atomicAdd(&c[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
}

hipError_t launch_plane_counts(const hs_cand* out, const int64_t* out_offsets, const int64_t* caps, int64_t cap,
                               unsigned long long* counts, int n_lists, int H, int s_bin, uint32_t kmask,
                               hipStream_t s)
{
    if (n_lists < 1 || n_lists > 65535 || H < 1 || H > kMaxH) return hipErrorInvalidValue;
    // one list: enough blocks for its capacity, at most kPcMaxBlocks; a
    // batch: one block per list
    int64_t bx = 1;
    if (n_lists == 1) {
        bx = (cap + (int64_t)kPcThreads * kPcU - 1) / ((int64_t)kPcThreads * kPcU);
        bx = bx < 1 ? 1 : (bx > kPcMaxBlocks ? kPcMaxBlocks : bx);
    }
    hipLaunchKernelGGL(k_plane_counts, dim3((unsigned)bx, (unsigned)n_lists), dim3(kPcThreads), 0, s,
                       reinterpret_cast<const uint64_t*>(out), out_offsets, caps, cap, counts, H, s_bin, kmask);
    return hipGetLastError();
}

int fused_lds_bytes(int T, int R, int H, int mode, int elem_bytes)
{
    (void)mode;
    return fused_stage_bytes(H, elem_bytes) + smem_tail_bytes(T, R, H);
}

#define HS_GROUP_CASES(call)                                                                    \
    switch ((H - 1) / 4) {                                                                      \
    case 0: return call(0);                                                                     \
    case 1: return call(1);                                                                     \
    case 2: return call(2);                                                                     \
    case 3: return call(3);                                                                     \
    }                                                                                           \
    return hipErrorInvalidValue;

hipError_t launch_fused(int mode, int dtype, int H, const TileArgs& a, int64_t n_tiles, int grid,
                        int lds_bytes, hipStream_t s)
{
    if (H < 1 || H > kMaxH) return hipErrorInvalidValue;
    if (mode == kModeLse) {
        if (dtype != HS_DTYPE_F32) return hipErrorInvalidValue;
#define HS_CALL(g) launch_stat_f32_g##g(mode, H, a, n_tiles, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    switch (dtype) {
    case HS_DTYPE_F32: {
#define HS_CALL(g) launch_fused_f32_g##g(mode, H, a, n_tiles, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    case HS_DTYPE_F16: {
#define HS_CALL(g) launch_fused_f16_g##g(mode, H, a, n_tiles, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    case HS_DTYPE_BF16: {
#define HS_CALL(g) launch_fused_bf16_g##g(mode, H, a, n_tiles, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batched(int dtype, int H, const BatchArgs& b, int grid, int lds_bytes, hipStream_t s)
{
    if (H < 1 || H > kMaxH) return hipErrorInvalidValue;
    switch (dtype) {
    case HS_DTYPE_F32: {
#define HS_CALL(g) launch_batched_f32_g##g(H, b, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    case HS_DTYPE_F16: {
#define HS_CALL(g) launch_batched_f16_g##g(H, b, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    case HS_DTYPE_BF16: {
#define HS_CALL(g) launch_batched_bf16_g##g(H, b, grid, lds_bytes, s)
        HS_GROUP_CASES(HS_CALL)
#undef HS_CALL
    }
    }
    return hipErrorInvalidValue;
}

// Streaming read of n16 16-byte words: block b sums its words (grid-stride,
// four loads in flight per thread) and writes one float, sink[b].  The
// bandwidth ceiling the detection kernels are measured against.
__global__ __launch_bounds__(256) void k_stream_read(const float4* __restrict__ p, int64_t n16,
                                                     float* __restrict__ sink)
{
    constexpr int U = 4;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float acc = 0.0f;
    for (; i + (U - 1) * stride < n16; i += U * stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (; i < n16; i += stride) {
        const float4 v = p[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    __shared__ float part[4];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

hipError_t launch_stream_read(const void* src, int64_t bytes, float* sink, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, s, static_cast<const float4*>(src), bytes / 16,
                       sink);
    return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace hsk
