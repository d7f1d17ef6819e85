// Fused harmonic-summing kernels for gfx950: harmonic planes (Eq. 1-2 of
// arXiv:1805.12258, Sec. III) with threshold detection, or materialised.
//
// Work decomposition (the paper's MultipleHP idea, Sec. IV-C, rebuilt for a
// GPU): a tile is a block of template rows x kTileBins consecutive bins.  For
// each stretch factor m >= 2 the tile reads only the shrunken source range
// rows floor(i/m), bins [floor(j0/m), floor((j0+B-1)/m)] of the FOP; these
// ranges are staged in LDS once per tile (for fp32 straight from global
// memory with LDS-DMA loads).  Each lane owns kV consecutive bins of one row
// at a time and keeps the kV partial sums in registers; HP_k is formed for
// k = 1..H in order (Eq. 2), compared with its row threshold and, in the
// materialising mode, stored.  No intermediate plane goes to memory in the
// detection mode.
//
// Candidates are compacted through a per-block LDS buffer (wave-aggregated
// LDS atomics) and written out with one global atomic per block; a buffer
// overflow spills straight to global memory with per-wave atomics.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "hs_internal.h"

namespace hsk {

struct bf16_t {
    uint16_t bits;
};

template <typename TIn> struct Io;

template <> struct Io<float> {
    using T = float;
    static __device__ __forceinline__ float one(const T* p) { return *p; }
    static __device__ __forceinline__ void four(const T* p, float* v)
    {
        const float4 x = *reinterpret_cast<const float4*>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
};

template <> struct Io<_Float16> {
    using T = _Float16;
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ float one(const T* p) { return (float)*p; }
    static __device__ __forceinline__ void four(const T* p, float* v)
    {
        const h4 x = *reinterpret_cast<const h4*>(p);
        v[0] = (float)x.x; v[1] = (float)x.y; v[2] = (float)x.z; v[3] = (float)x.w;
    }
};

template <> struct Io<bf16_t> {
    using T = bf16_t;
    static __device__ __forceinline__ float one(const T* p)
    {
        return __uint_as_float((uint32_t)p->bits << 16);
    }
    static __device__ __forceinline__ void four(const T* p, float* v)
    {
        const uint2 x = *reinterpret_cast<const uint2*>(p);
        v[0] = __uint_as_float(x.x << 16);
        v[1] = __uint_as_float(x.x & 0xffff0000u);
        v[2] = __uint_as_float(x.y << 16);
        v[3] = __uint_as_float(x.y & 0xffff0000u);
    }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Compile-time loop: f(integral_constant<int, I>) for I = B..E.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B <= E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Shared-memory carve-up of one block.
struct Smem {
    float* stage;                 // staged source rows, all m >= 2
    float* thr;                   // [R][H] thresholds * scale
    uint2* cand;                  // [kCandCap]
    int* cnt;                     // [0]: buffered candidates, [k]: plane k
    unsigned long long* base;     // global slot of the buffer
};

template <int H>
__device__ __forceinline__ Smem carve(float* lds, int stage_words, int R)
{
    Smem s;
    s.stage = lds;
    s.thr = lds + stage_words;
    const int thr_words = (R * H + 3) & ~3;
    s.cand = reinterpret_cast<uint2*>(s.thr + thr_words);
    s.base = reinterpret_cast<unsigned long long*>(s.cand + kCandCap);
    s.cnt = reinterpret_cast<int*>(s.base + 1);
    return s;
}


template <int H>
__device__ __forceinline__ void push_cand(const Smem& sh, hs_cand* out, int64_t cap,
                                          unsigned long long* counts, uint32_t key, float pw, int k)
{
    const int pos = atomicAdd(&sh.cnt[0], 1);
    if (pos < kCandCap) {
        sh.cand[pos] = make_uint2(key, __float_as_uint(pw));
    } else {
        const unsigned long long g = atomicAdd(&counts[H], 1ull);
        if ((int64_t)g < cap) {
            reinterpret_cast<uint2*>(out)[g] = make_uint2(key, __float_as_uint(pw));
        }
    }
    atomicAdd(&sh.cnt[k], 1);
}

// Write the block's buffered candidates and per-plane counts to global memory
// and reset the buffer.  Called by the whole block, after a barrier.
template <int H>
__device__ __forceinline__ void flush_cands(const Smem& sh, hs_cand* out, int64_t cap,
                                            unsigned long long* counts)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        const int n = min(sh.cnt[0], kCandCap);
        *sh.base = n ? atomicAdd(&counts[H], (unsigned long long)n) : 0ull;
        sh.cnt[0] = n;
    }
    if (tid >= 1 && tid <= H) {
        const int n = sh.cnt[tid];
        if (n) atomicAdd(&counts[tid - 1], (unsigned long long)n);
    }
    __syncthreads();
    const int n = sh.cnt[0];
    const unsigned long long base = *sh.base;
    for (int e = tid; e < n; e += kThreads) {
        if ((int64_t)(base + e) < cap) reinterpret_cast<uint2*>(out)[base + e] = sh.cand[e];
    }
    __syncthreads();
    if (tid <= H) sh.cnt[tid] = 0;
}

// One tile: stage, form the planes, detect or store.
template <typename TIn, int H, int MODE>
__device__ __forceinline__ void run_tile(const TileArgs& a, int64_t tile, const Smem& sh)
{
    using Ld = Io<TIn>;
    using T = typename Ld::T;
    const T* __restrict__ fop = reinterpret_cast<const T*>(a.fop);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int rb = (int)(tile % a.row_blocks);
    const int64_t j0 = (tile / a.row_blocks) * kTileBins;
    const int r0 = rb * a.R;
    const int r1 = min(r0 + a.R, a.T);
    const int nr = r1 - r0;
    const int c = a.c;
    const int64_t N = a.N;
    const int64_t ld = a.ld;
    const int i_lo = r0 - c, i_hi = r1 - 1 - c;
    const int64_t jend = min(j0 + (int64_t)kTileBins, N);   // one past the tile's last bin

    // Source ranges of every stretch factor (scalar).
    int a_lo[H + 1], nrow[H + 1], offm[H + 1], span[H + 1];
    int64_t blo[H + 1];
    int tot = 0;
#pragma unroll
    for (int m = 2; m <= H; ++m) {
        a_lo[m] = (int)floordiv(i_lo, m);
        nrow[m] = (int)floordiv(i_hi, m) - a_lo[m] + 1;
        blo[m] = j0 / m;
        span[m] = (int)((jend - 1) / m - blo[m] + 1);
        offm[m] = tot;
        tot += nrow[m] * stage_pitch(m);
    }

    // Stage the shrunken source ranges.
#pragma unroll
    for (int m = 2; m <= H; ++m) {
        for (int row = wave; row < nrow[m]; row += kWaves) {
            const T* src = fop + (int64_t)(a_lo[m] + row + c) * ld + blo[m];
            float* dst = sh.stage + offm[m] + row * stage_pitch(m);
            for (int ch = 0; ch * 64 < span[m]; ++ch) {
                const int col = ch * 64 + lane;
                if constexpr (sizeof(T) == 4) {
                    if (col < span[m]) {
                        __builtin_amdgcn_global_load_lds(src + col, (lds_ptr_t)(dst + ch * 64), 4, 0, 0);
                    }
                } else {
                    if (col < span[m]) dst[col] = Ld::one(src + col);
                }
            }
        }
    }
    if constexpr (MODE == kModeDetect) {
        for (int e = threadIdx.x; e < nr * H; e += kThreads) {
            const int rr = e / H, k = e - rr * H;
            sh.thr[e] = a.ta[(int64_t)k * a.T + r0 + rr] * a.scale;
        }
    }

    // Per-lane view of the staged rows.
    const int64_t jb = j0 + kV * lane;
    bool valid[kV];
#pragma unroll
    for (int v = 0; v < kV; ++v) valid[v] = jb + v < N;
    int loff[H + 1], sig[H + 1];
#pragma unroll
    for (int m = 2; m <= H; ++m) {
        const int rho = (int)(j0 - blo[m] * m);       // j0 mod m
        const int t = rho + kV * lane;
        loff[m] = offm[m] + t / m;
        sig[m] = t % m;
    }

    // First row's m = 1 values (overlaps the staging loads).
    auto load_row = [&](int r, float* x) {
        const T* p = fop + (int64_t)r * ld + jb;
        if (jb + kV <= N) {
            Ld::four(p, x);
        } else {
#pragma unroll
            for (int v = 0; v < kV; ++v) x[v] = valid[v] ? Ld::one(p + v) : 0.0f;
        }
    };
    float xn[kV];
    if (wave < nr) load_row(r0 + wave, xn);

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int rr = wave; rr < nr; rr += kWaves) {
        const int r = r0 + rr;
        const int i = r - c;
        float acc[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) acc[v] = xn[v];
        if (rr + kWaves < nr) load_row(r + kWaves, xn);

        float thr[H];
        if constexpr (MODE == kModeDetect) {
#pragma unroll
            for (int k = 0; k < H; ++k) thr[k] = sh.thr[rr * H + k];
        }

        auto emit = [&](int k) {
            if constexpr (MODE == kModeDetect) {
                const float t = thr[k - 1];
                bool hit[kV];
                bool any = false;
#pragma unroll
                for (int v = 0; v < kV; ++v) {
                    hit[v] = valid[v] && (acc[v] > t);
                    any |= hit[v];
                }
                if (any) {
                    const uint32_t hi = (uint32_t)(((uint64_t)r << a.s_row) | ((uint64_t)(k - 1) << a.s_bin));
#pragma unroll
                    for (int v = 0; v < kV; ++v) {
                        if (hit[v]) {
                            push_cand<H>(sh, a.out, a.cap, a.counts, hi | (uint32_t)(jb + v),
                                         acc[v] * a.inv_scale, k);
                        }
                    }
                }
            } else {
                float* dst = a.hp + ((int64_t)(k - 1) * a.T + r) * N + jb;
                float y[kV];
#pragma unroll
                for (int v = 0; v < kV; ++v) y[v] = acc[v] * a.inv_scale;
                if (jb + kV <= N && (N & 3) == 0) {
                    *reinterpret_cast<float4*>(dst) = make_float4(y[0], y[1], y[2], y[3]);
                } else {
#pragma unroll
                    for (int v = 0; v < kV; ++v)
                        if (valid[v]) dst[v] = y[v];
                }
            }
        };

        emit(1);
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int srow = (int)floordiv(i, m) - a_lo[m];
            const float* p = sh.stage + loff[m] + srow * stage_pitch(m);
            if constexpr (kV % m == 0) {
                float w[kV / m];
#pragma unroll
                for (int q = 0; q < kV / m; ++q) w[q] = p[q];
#pragma unroll
                for (int v = 0; v < kV; ++v) acc[v] = acc[v] + w[v / m];
            } else if constexpr (m % kV == 0) {
                const float w0 = p[0];
#pragma unroll
                for (int v = 0; v < kV; ++v) acc[v] = acc[v] + w0;
            } else {
                // lane's kV bins span two source words: bin jb+v reads word
                // floor((sig + v)/m) of the lane's window
                const float w0 = p[0], w1 = p[1];
#pragma unroll
                for (int v = 0; v < kV; ++v) {
                    const int q = v / m, s = v % m;
                    float val;
                    if (s == 0) val = q ? w1 : w0;
                    else val = (sig[m] >= m - s) ? w1 : w0;
                    acc[v] = acc[v] + val;
                }
            }
            emit(m);
        });
    }
}

template <typename TIn, int H, int MODE>
__global__ __launch_bounds__(kThreads) void k_fused(TileArgs a, int stage_words)
{
    extern __shared__ __align__(16) float lds[];
    const Smem sh = carve<H>(lds, stage_words, a.R);
    if constexpr (MODE == kModeDetect) {
        if (threadIdx.x <= H) sh.cnt[threadIdx.x] = 0;
    }
    run_tile<TIn, H, MODE>(a, blockIdx.x, sh);
    if constexpr (MODE == kModeDetect) {
        __syncthreads();
        flush_cands<H>(sh, a.out, a.cap, a.counts);
    }
}

// Batched persistent kernel: a fixed grid walks the tiles of every FOP.
template <typename TIn, int H>
__global__ __launch_bounds__(kThreads) void k_batched(BatchArgs b, int stage_words)
{
    extern __shared__ __align__(16) float lds[];
    const Smem sh = carve<H>(lds, stage_words, b.R);
    if (threadIdx.x <= H) sh.cnt[threadIdx.x] = 0;
    constexpr int align_elems = sizeof(typename Io<TIn>::T) == 4 ? 4 : 8;

    int f = 0;
    int64_t t = blockIdx.x;
    // first FOP holding tile t (binary search over the prefix of tile counts)
    {
        int lo = 0, hi = b.n_fops - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.tile_prefix[mid] <= t) lo = mid; else hi = mid - 1;
        }
        f = lo;
    }
    for (; t < b.tiles_total; t += gridDim.x) {
        while (t >= b.tile_prefix[f + 1]) ++f;
        f = __builtin_amdgcn_readfirstlane(f);
        TileArgs a;
        a.fop = b.fops[f];
        a.ld = b.lds[f];
        a.N = b.n_chans[f];
        a.T = b.T;
        a.c = b.c;
        a.R = b.R;
        a.row_blocks = b.row_blocks;
        a.scale = b.scale;
        a.inv_scale = b.inv_scale;
        a.ta = b.ta;
        a.out = b.out + b.out_offsets[f];
        a.cap = b.caps[f];
        a.counts = b.counts + (int64_t)f * (H + 1);
        a.s_row = b.s_row;
        a.s_bin = b.s_bin;
        a.hp = nullptr;
        const bool ok = ((reinterpret_cast<uintptr_t>(a.fop) & 15) == 0) &&
                        (a.ld % align_elems == 0) && a.ld >= a.N;
        if (!ok) {
            if (threadIdx.x == 0 && t == b.tile_prefix[f]) a.counts[H] = ~0ull;
            continue;
        }
        run_tile<TIn, H, kModeDetect>(a, t - b.tile_prefix[f], sh);
        __syncthreads();
        flush_cands<H>(sh, a.out, a.cap, a.counts);
    }
}

template <typename TIn, int H>
static hipError_t launch_fused_t(int mode, const TileArgs& a, int64_t n_tiles, int lds_bytes,
                                 hipStream_t s)
{
    const int stage_words = (lds_bytes - smem_tail_bytes(a.R, H)) / 4;
    if (mode == kModeDetect) {
        auto k = k_fused<TIn, H, kModeDetect>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        hipLaunchKernelGGL(k, dim3((unsigned)n_tiles), dim3(kThreads), lds_bytes, s, a, stage_words);
    } else {
        auto k = k_fused<TIn, H, kModeSum>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        hipLaunchKernelGGL(k, dim3((unsigned)n_tiles), dim3(kThreads), lds_bytes, s, a, stage_words);
    }
    return hipGetLastError();
}

template <typename TIn, int H>
static hipError_t launch_batched_t(const BatchArgs& b, int grid, int lds_bytes, hipStream_t s)
{
    const int stage_words = (lds_bytes - smem_tail_bytes(b.R, H)) / 4;
    auto k = k_batched<TIn, H>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds_bytes, s, b, stage_words);
    return hipGetLastError();
}

#define HS_H_CASES(F, ...)                                                                        \
    switch (H) {                                                                                  \
    case 1: return F<1>(__VA_ARGS__);   case 2: return F<2>(__VA_ARGS__);                         \
    case 3: return F<3>(__VA_ARGS__);   case 4: return F<4>(__VA_ARGS__);                         \
    case 5: return F<5>(__VA_ARGS__);   case 6: return F<6>(__VA_ARGS__);                         \
    case 7: return F<7>(__VA_ARGS__);   case 8: return F<8>(__VA_ARGS__);                         \
    case 9: return F<9>(__VA_ARGS__);   case 10: return F<10>(__VA_ARGS__);                       \
    case 11: return F<11>(__VA_ARGS__); case 12: return F<12>(__VA_ARGS__);                       \
    case 13: return F<13>(__VA_ARGS__); case 14: return F<14>(__VA_ARGS__);                       \
    case 15: return F<15>(__VA_ARGS__); case 16: return F<16>(__VA_ARGS__);                       \
    default: return hipErrorInvalidValue;                                                         \
    }

}  // namespace hsk
