// Launcher of the strip-walk kernels for one storage type, one number of
// bins per lane and one group of four plane counts.  Each including
// translation unit defines HS_WALK_T (storage type), HS_WALK_NAME (its short
// name), HS_WALK_V (bins per lane) and HS_WALK_GROUP (H in 4 * group + 1 ..
// 4 * group + 4), so the kernel sets compile in parallel.
#include "hs_walk_impl.h"

#define HS_WPASTE4(a, b, v, c) a##_##b##_v##v##_g##c
#define HS_WNAMED(base, n, v, g) HS_WPASTE4(base, n, v, g)

namespace hsk {

hipError_t HS_WNAMED(launch_walk, HS_WALK_NAME, HS_WALK_V, HS_WALK_GROUP)(int H, const WalkArgs& a, int grid, int lds,
                                                                          hipStream_t s)
{
    switch (H - 4 * HS_WALK_GROUP) {
    case 1: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 1, HS_WALK_V>(a, grid, lds, s);
    case 2: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 2, HS_WALK_V>(a, grid, lds, s);
    case 3: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 3, HS_WALK_V>(a, grid, lds, s);
    case 4: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 4, HS_WALK_V>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hsk
