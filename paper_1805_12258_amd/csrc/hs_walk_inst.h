// Launcher of the strip-walk kernels for one storage type and one group of
// four plane counts.  Each including translation unit defines HS_WALK_T
// (storage type), HS_WALK_NAME (its short name) and HS_WALK_GROUP (H in
// 4 * group + 1 .. 4 * group + 4), so the kernel sets compile in parallel.
#include "hs_walk_impl.h"

#define HS_WPASTE3(a, b, c) a##_##b##_g##c
#define HS_WNAMED(base, n, g) HS_WPASTE3(base, n, g)

namespace hsk {

hipError_t HS_WNAMED(launch_walk, HS_WALK_NAME, HS_WALK_GROUP)(int H, const WalkArgs& a, int grid, int lds,
                                                               hipStream_t s)
{
    switch (H - 4 * HS_WALK_GROUP) {
    case 1: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 1>(a, grid, lds, s);
    case 2: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 2>(a, grid, lds, s);
    case 3: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 3>(a, grid, lds, s);
    case 4: return launch_walk_t<HS_WALK_T, 4 * HS_WALK_GROUP + 4>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hsk
