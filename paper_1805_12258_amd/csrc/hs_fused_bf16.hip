// Fused kernels instantiated for bf16_t FOP storage.
#include "hs_fused_impl.h"

namespace hsk {

template <int H>
static hipError_t fused_one(int mode, const TileArgs& a, int64_t n, int g, int lds, hipStream_t s)
{
    return launch_fused_t<bf16_t, H>(mode, a, n, g, lds, s);
}

template <int H>
static hipError_t batched_one(const BatchArgs& b, int grid, int lds, hipStream_t s)
{
    return launch_batched_t<bf16_t, H>(b, grid, lds, s);
}

hipError_t launch_fused_bf16(int mode, int H, const TileArgs& a, int64_t n, int g, int lds, hipStream_t s)
{
    HS_H_CASES(fused_one, mode, a, n, g, lds, s)
}

hipError_t launch_batched_bf16(int H, const BatchArgs& b, int grid, int lds, hipStream_t s)
{
    HS_H_CASES(batched_one, b, grid, lds, s)
}

}  // namespace hsk
