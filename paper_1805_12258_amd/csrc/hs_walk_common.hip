// Dtype-independent parts of the strip-walk kernels: LDS sizing and dispatch
// on the storage type, the bins per lane and the plane count.
#include "hs_walk_impl.h"

namespace hsk {

#define HS_WDECL(n, v, g) \
    hipError_t launch_walk_##n##_v##v##_g##g(int H, const WalkArgs& a, int grid, int lds, hipStream_t s);
#define HS_WDECL_V(n, v) HS_WDECL(n, v, 0) HS_WDECL(n, v, 1) HS_WDECL(n, v, 2) HS_WDECL(n, v, 3)
#define HS_WDECL_TYPE(n) HS_WDECL_V(n, 2) HS_WDECL_V(n, 4) HS_WDECL_V(n, 8)
HS_WDECL_TYPE(f32)
HS_WDECL_TYPE(f16)
HS_WDECL_TYPE(bf16)

static_assert(walk::kWDmax == kWalkDepth, "pipeline depth");

bool walk_supported(int T, int H)
{
    return T >= walk::kWDmax && (int64_t)T * walk::thr_stride(H) * 4 <= walk::kWThrBytes && H >= 1 && H <= kMaxH;
}

bool walk_v_ok(int V) { return V == 2 || V == 4 || V == 8; }

int walk_lds_bytes(int T, int H, int dtype, int V)
{
    const int EB = dtype == HS_DTYPE_F32 ? 4 : 2;
    return walk::kWWaves * walk::wave_bytes(H, EB, V) + walk::kWBookBytes + T * walk::thr_stride(H) * 4;
}

#define HS_WCASES(n, v)                                                   \
    switch ((H - 1) / 4) {                                                \
    case 0: return launch_walk_##n##_v##v##_g0(H, a, grid, lds, s);       \
    case 1: return launch_walk_##n##_v##v##_g1(H, a, grid, lds, s);       \
    case 2: return launch_walk_##n##_v##v##_g2(H, a, grid, lds, s);       \
    case 3: return launch_walk_##n##_v##v##_g3(H, a, grid, lds, s);       \
    }                                                                     \
    return hipErrorInvalidValue;

#define HS_WCASES_V(n)                        \
    switch (V) {                              \
    case 2: { HS_WCASES(n, 2) }               \
    case 4: { HS_WCASES(n, 4) }               \
    case 8: { HS_WCASES(n, 8) }               \
    }                                         \
    return hipErrorInvalidValue;

hipError_t launch_walk(int dtype, int H, int V, const WalkArgs& a, int grid, int lds, hipStream_t s)
{
    if (H < 1 || H > kMaxH) return hipErrorInvalidValue;
    switch (dtype) {
    case HS_DTYPE_F32: { HS_WCASES_V(f32) }
    case HS_DTYPE_F16: { HS_WCASES_V(f16) }
    case HS_DTYPE_BF16: { HS_WCASES_V(bf16) }
    }
    return hipErrorInvalidValue;
}

}  // namespace hsk
