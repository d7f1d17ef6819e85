// Dtype-independent parts of the fused kernels: LDS sizing, dispatch on the
// storage type, the counter-clearing kernel.
#include <hip/hip_runtime.h>

#include "hs_internal.h"

namespace hsk {

hipError_t launch_fused_f32(int mode, int H, const TileArgs& a, int64_t n, int g, int lds, hipStream_t s);
hipError_t launch_fused_f16(int mode, int H, const TileArgs& a, int64_t n, int g, int lds, hipStream_t s);
hipError_t launch_fused_bf16(int mode, int H, const TileArgs& a, int64_t n, int g, int lds, hipStream_t s);
hipError_t launch_batched_f32(int H, const BatchArgs& b, int grid, int lds, hipStream_t s);
hipError_t launch_batched_f16(int H, const BatchArgs& b, int grid, int lds, hipStream_t s);
hipError_t launch_batched_bf16(int H, const BatchArgs& b, int grid, int lds, hipStream_t s);

__global__ void k_zero_i64(int64_t* p, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0;
}

int fused_stage_words(int T, int R, int H)
{
    const int c = T / 2;
    int worst = 0;
    for (int r0 = 0; r0 < T; r0 += R) {
        const int r1 = r0 + R < T ? r0 + R : T;
        int tot = 0;
        for (int m = 2; m <= H; ++m) {
            const int nrow = (int)(floordiv(r1 - 1 - c, m) - floordiv(r0 - c, m) + 1);
            tot += nrow * stage_pitch(m);
        }
        tot = (tot + 3) & ~3;      // the row table after it is read as float4
        if (tot > worst) worst = tot;
    }
    return worst;
}

int fused_lds_bytes(int T, int R, int H, int mode)
{
    (void)mode;
    return 2 * fused_stage_words(T, R, H) * 4 + smem_tail_bytes(T, R, H);
}

hipError_t launch_fused(int mode, int dtype, int H, const TileArgs& a, int64_t n_tiles, int grid,
                        int lds_bytes, hipStream_t s)
{
    switch (dtype) {
    case HS_DTYPE_F32: return launch_fused_f32(mode, H, a, n_tiles, grid, lds_bytes, s);
    case HS_DTYPE_F16: return launch_fused_f16(mode, H, a, n_tiles, grid, lds_bytes, s);
    case HS_DTYPE_BF16: return launch_fused_bf16(mode, H, a, n_tiles, grid, lds_bytes, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batched(int dtype, int H, const BatchArgs& b, int grid, int lds_bytes, hipStream_t s)
{
    switch (dtype) {
    case HS_DTYPE_F32: return launch_batched_f32(H, b, grid, lds_bytes, s);
    case HS_DTYPE_F16: return launch_batched_f16(H, b, grid, lds_bytes, s);
    case HS_DTYPE_BF16: return launch_batched_bf16(H, b, grid, lds_bytes, s);
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
