// Dtype-independent parts of the fused kernels: LDS sizing, dispatch on the
// storage type, the counter-clearing kernel.
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
    if (mode == kModeLse || mode == kModeWeights) {
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

hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace hsk
