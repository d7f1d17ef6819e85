// Dtype-independent parts of the strip-walk kernels: LDS sizing and dispatch
// on the storage type and plane count.
#include "hs_walk_impl.h"

namespace hsk {

#define HS_WDECL(n, g) hipError_t launch_walk_##n##_g##g(int H, const WalkArgs& a, int grid, int lds, hipStream_t s);
#define HS_WDECL_TYPE(n) HS_WDECL(n, 0) HS_WDECL(n, 1) HS_WDECL(n, 2) HS_WDECL(n, 3)
HS_WDECL_TYPE(f32)
HS_WDECL_TYPE(f16)
HS_WDECL_TYPE(bf16)

namespace {
constexpr int wave_bytes_of(int H, int EB)
{
    return walk::wave_bytes(H, EB);
}
}  // namespace

static_assert(walk::kWBins == kWalkStripBins, "strip width");
static_assert(walk::kWDmax == kWalkDepth, "pipeline depth");

bool walk_supported(int T, int H)
{
    return T >= walk::kWDmax && (int64_t)T * walk::thr_stride(H) * 4 <= walk::kWThrBytes && H >= 1 && H <= kMaxH;
}

int walk_lds_bytes(int T, int H, int dtype)
{
    const int EB = dtype == HS_DTYPE_F32 ? 4 : 2;
    return walk::kWWaves * wave_bytes_of(H, EB) + walk::kWBookBytes + T * walk::thr_stride(H) * 4;
}

#define HS_WCASES(n)                                                  \
    switch ((H - 1) / 4) {                                            \
    case 0: return launch_walk_##n##_g0(H, a, grid, lds, s);         \
    case 1: return launch_walk_##n##_g1(H, a, grid, lds, s);         \
    case 2: return launch_walk_##n##_g2(H, a, grid, lds, s);         \
    case 3: return launch_walk_##n##_g3(H, a, grid, lds, s);         \
    }                                                                 \
    return hipErrorInvalidValue;

hipError_t launch_walk(int dtype, int H, const WalkArgs& a, int grid, int lds, hipStream_t s)
{
    if (H < 1 || H > kMaxH) return hipErrorInvalidValue;
    switch (dtype) {
    case HS_DTYPE_F32: { HS_WCASES(f32) }
    case HS_DTYPE_F16: { HS_WCASES(f16) }
    case HS_DTYPE_BF16: { HS_WCASES(bf16) }
    }
    return hipErrorInvalidValue;
}

}  // namespace hsk
