// Launchers of the fused kernels for one storage type and one group of four
// plane counts.  Each including translation unit defines HS_INST_T (storage
// type), HS_INST_NAME (its short name) and HS_INST_GROUP (H in
// 4 * group + 1 .. 4 * group + 4), so the kernel sets compile in parallel;
// with HS_INST_STAT defined it holds the statistic's modes of fp32 storage
// instead.
#include "hs_fused_impl.h"

#define HS_PASTE3(a, b, c) a##_##b##_g##c
#define HS_NAMED(base, n, g) HS_PASTE3(base, n, g)

namespace hsk {

#ifdef HS_INST_STAT
// the statistic's modes (fp32 storage)
hipError_t HS_NAMED(launch_stat, HS_INST_NAME, HS_INST_GROUP)(int mode, int H, const TileArgs& a, int64_t n,
                                                              int g, int lds, hipStream_t s)
{
    switch (H - 4 * HS_INST_GROUP) {
    case 1: return launch_stat_t<4 * HS_INST_GROUP + 1>(mode, a, n, g, lds, s);
    case 2: return launch_stat_t<4 * HS_INST_GROUP + 2>(mode, a, n, g, lds, s);
    case 3: return launch_stat_t<4 * HS_INST_GROUP + 3>(mode, a, n, g, lds, s);
    case 4: return launch_stat_t<4 * HS_INST_GROUP + 4>(mode, a, n, g, lds, s);
    }
    return hipErrorInvalidValue;
}
#else
hipError_t HS_NAMED(launch_fused, HS_INST_NAME, HS_INST_GROUP)(int mode, int H, const TileArgs& a,
                                                               int64_t n, int g, int lds, hipStream_t s)
{
    switch (H - 4 * HS_INST_GROUP) {
    case 1: return launch_fused_t<HS_INST_T, 4 * HS_INST_GROUP + 1>(mode, a, n, g, lds, s);
    case 2: return launch_fused_t<HS_INST_T, 4 * HS_INST_GROUP + 2>(mode, a, n, g, lds, s);
    case 3: return launch_fused_t<HS_INST_T, 4 * HS_INST_GROUP + 3>(mode, a, n, g, lds, s);
    case 4: return launch_fused_t<HS_INST_T, 4 * HS_INST_GROUP + 4>(mode, a, n, g, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t HS_NAMED(launch_batched, HS_INST_NAME, HS_INST_GROUP)(int H, const BatchArgs& b, int grid,
                                                                 int lds, hipStream_t s)
{
    switch (H - 4 * HS_INST_GROUP) {
    case 1: return launch_batched_t<HS_INST_T, 4 * HS_INST_GROUP + 1>(b, grid, lds, s);
    case 2: return launch_batched_t<HS_INST_T, 4 * HS_INST_GROUP + 2>(b, grid, lds, s);
    case 3: return launch_batched_t<HS_INST_T, 4 * HS_INST_GROUP + 3>(b, grid, lds, s);
    case 4: return launch_batched_t<HS_INST_T, 4 * HS_INST_GROUP + 4>(b, grid, lds, s);
    }
    return hipErrorInvalidValue;
}
#endif

}  // namespace hsk
