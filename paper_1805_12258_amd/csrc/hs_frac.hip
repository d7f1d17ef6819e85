// Harmonic planes under the fractional mapping,
//     HPF_k(i, j) = sum_{m=1..k} FOP(floor(m i / k), floor(m j / k)),
// the FOP at the fractions m/k of each point (i = r - T/2 signed, floor
// division), terms added in the order m = 1..k in fp32 (each partial sum
// rounded, no contraction): the incoherent-sum reading of the harmonic sum
// of Sec. III.  Unlike Eq. 1-2 the planes are not cumulative: plane k reads
// k source points of its own, sum_k k = H (H + 1) / 2 of them per point.
//
// Layout of the work: a wave forms one row of a 256-bin strip (four
// consecutive bins per lane), a block four consecutive rows of one strip,
// so that the four rows' source rows (floor(m i / k) for nearby i) and
// source bins share the L1 and L2; every source value is read with a
// plain cached load (the fractions m/k spread the sources of a strip over
// the whole plane, so a staged window would be reused little).  Bins per
// lane are consecutive, so the source bins of one term advance by m/k <= 1
// per bin: one division per term and lane, the other three by carry.
//
// Detection: the candidates of each (row, plane) are compacted with wave
// ballots into a per-wave LDS buffer, written out with one atomic per
// flush (positions reserved in the list) and one atomic per block at the
// end; per-plane counts of the stored entries come from the counting pass
// that follows (only entries dropped for lack of capacity are counted
// here).
#include <hip/hip_runtime.h>

#include "hs_internal.h"

namespace hsk {

namespace {

constexpr int kFWaves = 4;
constexpr int kFThreads = 64 * kFWaves;
constexpr int kFV = 4;                     // bins per lane
constexpr int kFBins = 64 * kFV;           // bins per strip
constexpr int kFCandCap = 320;             // per-wave LDS candidate buffer (>= kFBins)

template <typename TIn> struct FIo;
template <> struct FIo<float> {
    __device__ static float ld(const void* p, int64_t e) { return static_cast<const float*>(p)[e]; }
};
template <> struct FIo<_Float16> {
    __device__ static float ld(const void* p, int64_t e) { return (float)static_cast<const _Float16*>(p)[e]; }
};
struct bf16_raw {
    uint16_t bits;
};
template <> struct FIo<bf16_raw> {
    __device__ static float ld(const void* p, int64_t e)
    {
        return __uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[e] << 16);
    }
};

// floor(x / k) for 0 <= x < 2^32 / 15 and 1 <= k <= 16: x * ceil(2^32 / k)
// >> 32 (the rounding error x e / (k 2^32), e < k, stays below 1/k).  The
// plan keeps N <= 2^24, so m j < 16 (2^24 + 256) is in range.
__device__ __forceinline__ uint32_t div_k(uint32_t x, uint64_t magic)
{
    return (uint32_t)(((uint64_t)x * magic) >> 32);
}

// floor(a / k) for signed a (template indices) and 1 <= k <= 16.
__device__ __forceinline__ int floordiv_k(int a, int k, uint64_t magic)
{
    return a >= 0 ? (int)div_k((uint32_t)a, magic) : -(int)div_k((uint32_t)(-a + k - 1), magic);
}

template <typename TIn, bool DETECT>
__global__ __launch_bounds__(kFThreads) void k_frac(FracArgs a)
{
    __shared__ uint64_t cand[DETECT ? kFWaves * kFCandCap : 1];
    __shared__ int book[2 * kFWaves + 2];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n_rg = (a.T + kFWaves - 1) / kFWaves;
    const int64_t b = blockIdx.x;
    const int rg = (int)(b % n_rg);
    const int64_t strip = b / n_rg;
    const int r = rg * kFWaves + wave;
    const bool row_ok = r < a.T;
    const int i = r - a.c;
    const uint32_t jl = (uint32_t)(strip * kFBins) + (uint32_t)(kFV * lane);   // first bin of the lane
    uint64_t* wbuf = cand + (DETECT ? wave * kFCandCap : 0);
    int ncand = 0;

    auto flush = [&]() {
        if (ncand == 0) return;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.counts[a.H], (unsigned long long)ncand);
        base = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)base);
        for (int e0 = 0; e0 < ncand; e0 += 64) {
            const int e = e0 + lane;
            if (e < ncand) {
                const uint64_t c = wbuf[e];
                if ((int64_t)(base + e) < a.cap) reinterpret_cast<uint64_t*>(a.out)[base + e] = c;
                else atomicAdd(&a.counts[((uint32_t)c >> a.s_bin) & ((1u << (a.s_row - a.s_bin)) - 1u)], 1ull);
            }
        }
        ncand = 0;
    };

    if (row_ok) {
        for (int k = 1; k <= a.H; ++k) {
            const uint64_t mk = a.magic[k];
            float acc[kFV];
            for (int m = 1; m <= k; ++m) {
                const int srow = floordiv_k(m * i, k, mk) + a.c;
                const int64_t rowoff = (int64_t)srow * a.ld;
                const uint32_t base = (uint32_t)m * jl;
                uint32_t q = div_k(base, mk);
                int rem = (int)(base - q * (uint32_t)k);
#pragma unroll
                for (int v = 0; v < kFV; ++v) {
                    if (v > 0) {
                        rem += m;                  // m <= k: at most one carry
                        if (rem >= k) {
                            rem -= k;
                            ++q;
                        }
                    }
                    const float x = jl + v < (uint32_t)a.N ? FIo<TIn>::ld(a.fop, rowoff + q) : 0.0f;
                    acc[v] = m == 1 ? x : acc[v] + x;
                }
            }
            if constexpr (DETECT) {
                const float t = a.ta[(int64_t)(k - 1) * a.T + r] * a.scale;
                bool hit[kFV];
                bool anyl = false;
#pragma unroll
                for (int v = 0; v < kFV; ++v) {
                    hit[v] = jl + v < (uint32_t)a.N && acc[v] > t;
                    anyl |= hit[v];
                }
                const uint64_t any = __builtin_amdgcn_ballot_w64(anyl);
                if (any) {
                    if (ncand + kFV * __builtin_popcountll(any) > kFCandCap) flush();
                    const uint32_t hi = ((uint32_t)r << a.s_row) | ((uint32_t)(k - 1) << a.s_bin);
#pragma unroll
                    for (int v = 0; v < kFV; ++v) {
                        const uint64_t mv = __builtin_amdgcn_ballot_w64(hit[v]);
                        if (mv) {
                            const int pre = (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(mv >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mv, 0));
                            if (hit[v])
                                wbuf[ncand + pre] = ((uint64_t)__float_as_uint(acc[v] * a.inv_scale) << 32) |
                                                    (hi | (jl + v));
                            ncand += __builtin_popcountll(mv);
                        }
                    }
                }
            } else {
                float* dst = a.hp + ((int64_t)(k - 1) * a.T + r) * a.N + jl;
#pragma unroll
                for (int v = 0; v < kFV; ++v)
                    if (jl + v < (uint32_t)a.N) dst[v] = acc[v] * a.inv_scale;
            }
        }
    }

    if constexpr (DETECT) {
        // the block's last candidates with one atomic (idle waves take part
        // with none)
        __syncthreads();
        if (lane == 0) book[wave] = ncand;
        __syncthreads();
        if (threadIdx.x == 0) {
            int s = 0;
            for (int w = 0; w < kFWaves; ++w) {
                book[kFWaves + w] = s;
                s += book[w];
            }
            const unsigned long long bb = s ? atomicAdd(&a.counts[a.H], (unsigned long long)s) : 0ull;
            book[2 * kFWaves] = (int)(uint32_t)bb;
            book[2 * kFWaves + 1] = (int)(uint32_t)(bb >> 32);
        }
        __syncthreads();
        const unsigned long long base =
            (((unsigned long long)(uint32_t)book[2 * kFWaves + 1] << 32) | (uint32_t)book[2 * kFWaves]) +
            (unsigned long long)book[kFWaves + wave];
        for (int e0 = 0; e0 < ncand; e0 += 64) {
            const int e = e0 + lane;
            if (e < ncand) {
                const uint64_t c = wbuf[e];
                if ((int64_t)(base + e) < a.cap) reinterpret_cast<uint64_t*>(a.out)[base + e] = c;
                else atomicAdd(&a.counts[((uint32_t)c >> a.s_bin) & ((1u << (a.s_row - a.s_bin)) - 1u)], 1ull);
            }
        }
    }
}

template <typename TIn>
hipError_t launch_frac_t(bool detect, const FracArgs& a, hipStream_t s)
{
    const int64_t n_rg = (a.T + kFWaves - 1) / kFWaves;
    const int64_t blocks = n_rg * ((a.N + kFBins - 1) / kFBins);
    if (blocks < 1 || blocks > INT32_MAX) return hipErrorInvalidValue;
    if (detect)
        hipLaunchKernelGGL((k_frac<TIn, true>), dim3((unsigned)blocks), dim3(kFThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_frac<TIn, false>), dim3((unsigned)blocks), dim3(kFThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace

void frac_magic(FracArgs& a)
{
    a.magic[0] = 0;
    for (int k = 1; k <= kMaxH; ++k) a.magic[k] = (((uint64_t)1 << 32) + (uint64_t)k - 1) / (uint64_t)k;
}

hipError_t launch_frac(int dtype, bool detect, const FracArgs& a, hipStream_t s)
{
    if (a.H < 1 || a.H > kMaxH || a.T < 1 || a.N < 1) return hipErrorInvalidValue;
    switch (dtype) {
    case HS_DTYPE_F32: return launch_frac_t<float>(detect, a, s);
    case HS_DTYPE_F16: return launch_frac_t<_Float16>(detect, a, s);
    case HS_DTYPE_BF16: return launch_frac_t<bf16_raw>(detect, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hsk
