// Fused harmonic-summing kernels for gfx950: harmonic planes (Eq. 1-2 of
// arXiv:1805.12258, Sec. III) with threshold detection, or materialised.
//
// Work decomposition (the paper's MultipleHP idea, Sec. IV-C, rebuilt for a
// GPU): a tile is a block of at most kMaxTileRows template rows x kTileBins
// consecutive bins.  For each stretch factor m >= 2 the tile reads only the
// shrunken source range (rows floor(i/m), bins [floor(j0/m),
// floor((j0+B-1)/m)]); these ranges are staged in LDS once per tile, for fp32
// straight from global memory with LDS-DMA loads.  Each lane owns kV
// consecutive bins of one row at a time and keeps the kV partial sums in
// registers; HP_k is formed for k = 1..H in order (Eq. 2), compared with its
// row threshold and, in the materialising mode, stored.  No intermediate
// plane goes to memory in the detection mode.
//
// Latency: all loads a wave needs for a tile (its share of the staging and
// the m = 1 values of all its rows) are issued together at the start of the
// tile, so a tile costs one memory round trip; several blocks per compute
// unit overlap one another's round trips.  The grid is persistent: block b
// walks a contiguous chunk of tiles.
//
// Candidates: each wave appends its hits to a private LDS buffer (ballot +
// mbcnt, no atomics) and keeps per-plane counts in scalar registers.  A full
// buffer is written out with one global atomic per wave; per-plane counts
// are reduced through LDS and added to global memory once per block and FOP.
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

// Reduced-precision storage holds power * scale with scale a power of two;
// converting each stored value to fp32 and multiplying by 1/scale is exact,
// and power-of-two scaling commutes with every fp32 rounding of the sums, so
// the planes come out in power units, bitwise equal to the scaled-storage
// sums divided by scale.
template <typename TIn> struct Scaled { static constexpr bool value = !std::is_same<TIn, float>::value; };

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
    uint2* cand;                  // [kWaves][kWaveCandCap] per-wave candidate buffers
    int* cnt;                     // [kMaxH] per-plane counts of the block
};

__device__ __forceinline__ Smem carve(float* lds, int stage_words, int R, int H)
{
    Smem s;
    (void)R;
    (void)H;
    s.stage = lds;
    s.cand = reinterpret_cast<uint2*>(lds + stage_words);
    s.cnt = reinterpret_cast<int*>(s.cand + kWaves * kWaveCandCap);
    return s;
}

// Per-wave detection state (a wave-uniform value).
template <int H>
struct WaveState {
    int n;          // entries in the wave's LDS buffer
};

__device__ __forceinline__ uint64_t read_first_u64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Write a wave's buffered candidates to global memory (one atomic per wave)
// and count them per plane in the block's LDS counters (the plane is read
// back from each candidate word).
__device__ __forceinline__ void flush_wave(const uint2* wbuf, int n, hs_cand* out, int64_t cap,
                                           unsigned long long* total, int* block_cnt, int s_bin,
                                           uint32_t kmask)
{
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(total, (unsigned long long)n);
    base = read_first_u64(base);
    for (int e = lane; e < n; e += 64) {
        const uint2 c = wbuf[e];
        atomicAdd(&block_cnt[(c.x >> s_bin) & kmask], 1);
        if ((int64_t)(base + e) < cap) reinterpret_cast<uint2*>(out)[base + e] = c;
    }
}

// Add the block's per-plane counts to global memory and clear them.  Called
// by the whole block; contains barriers.
template <int H>
__device__ __forceinline__ void flush_counts(const Smem& sh, unsigned long long* counts)
{
    __syncthreads();
    if (threadIdx.x < H) {
        const int v = sh.cnt[threadIdx.x];
        if (v) atomicAdd(&counts[threadIdx.x], (unsigned long long)v);
        sh.cnt[threadIdx.x] = 0;
    }
    __syncthreads();
}

// One tile: stage, form the planes, detect or store.  Starts and ends with a
// barrier so the staging buffer is free when it is refilled.
template <typename TIn, int H, int MODE>
__device__ __forceinline__ void run_tile(const TileArgs& a, int64_t tile, const Smem& sh,
                                         WaveState<H>& ws)
{
    using Ld = Io<TIn>;
    using T = typename Ld::T;
    const T* __restrict__ fop = reinterpret_cast<const T*>(a.fop);
    // thresholds are read-only for the whole launch: read them through the
    // constant address space so uniform reads become scalar loads
    const __attribute__((address_space(4))) float* ta =
        (const __attribute__((address_space(4))) float*)a.ta;
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
        a_lo[m] = floordiv32(i_lo, m);
        nrow[m] = floordiv32(i_hi, m) - a_lo[m] + 1;
        blo[m] = j0 / m;
        span[m] = (int)((jend - 1) / m - blo[m] + 1);
        offm[m] = tot;
        tot += nrow[m] * stage_pitch(m);
    }

    __syncthreads();   // the previous tile is done with the staging buffer

    // 1. Stage the shrunken source ranges (this wave's rows of each region).
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
                    if (col < span[m]) dst[col] = Ld::one(src + col) * a.inv_scale;
                }
            }
        }
    }

    // 2. The m = 1 values of every row this wave owns.
    const int64_t jb = j0 + kV * lane;
    bool valid[kV];
#pragma unroll
    for (int v = 0; v < kV; ++v) valid[v] = jb + v < N;
    const bool tile_full = j0 + kTileBins <= N;        // wave-uniform
    float x[kRowsPerWave][kV];
    if (tile_full) {
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) {
            const int rr = wave + kWaves * q;
            if (rr < nr) Ld::four(fop + (int64_t)(r0 + rr) * ld + jb, x[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) {
            const int rr = wave + kWaves * q;
            const T* p = fop + (int64_t)(r0 + rr) * ld + jb;
#pragma unroll
            // bins past the end start at -inf: no sum of them can pass a
            // threshold (-inf + x is -inf or NaN)
            for (int v = 0; v < kV; ++v)
                x[q][v] = (rr < nr && valid[v]) ? Ld::one(p + v) : -__builtin_inff();
        }
    }

    // Per-lane view of the staged rows.
    int loff[H + 1], sig[H + 1];
#pragma unroll
    for (int m = 2; m <= H; ++m) {
        const int rho = (int)(j0 - blo[m] * m);       // j0 mod m
        const int t = rho + kV * lane;
        loff[m] = offm[m] + t / m;
        sig[m] = t % m;
    }

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    uint2* wbuf = sh.cand + wave * kWaveCandCap;
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
        const int rr = wave + kWaves * q;
        if (rr >= nr) break;
        const int r = r0 + rr;
        const int i = r - c;
        // All LDS reads of the row first (thresholds and staged source
        // words), so their latencies overlap; the candidate writes below
        // could otherwise alias them and serialise every read.
        float thr[H];
        if constexpr (MODE == kModeDetect) {
#pragma unroll
            for (int k = 0; k < H; ++k) thr[k] = ta[k * a.T + r];
        }
        float w[H + 1][2];
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int srow = floordiv32(i, m) - a_lo[m];
            const float* p = sh.stage + loff[m] + srow * stage_pitch(m);
            if constexpr (kV % m == 0) {
#pragma unroll
                for (int u = 0; u < kV / m; ++u) w[m][u] = p[u];
            } else if constexpr (m % kV == 0) {
                w[m][0] = p[0];
            } else {
                w[m][0] = p[0];
                w[m][1] = p[1];
            }
        });

        float acc[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) acc[v] = Scaled<TIn>::value ? x[q][v] * a.inv_scale : x[q][v];

        auto emit = [&](int k) {
            if constexpr (MODE == kModeDetect) {
                const float t = thr[k - 1];
                bool hit[kV];
                uint64_t mk[kV];
                uint64_t mall = 0;
#pragma unroll
                for (int v = 0; v < kV; ++v) {
                    hit[v] = acc[v] > t;
                    mk[v] = __builtin_amdgcn_ballot_w64(hit[v]);
                    mall |= mk[v];
                }
                if (mall) {
                    // room for every hit of this (row, plane): at most kV per lane
                    if (ws.n > kWaveCandCap - kV * 64) {
                        flush_wave(wbuf, ws.n, a.out, a.cap, &a.counts[H], sh.cnt, a.s_bin, a.kmask);
                        ws.n = 0;
                    }
                    const uint32_t hi =
                        (uint32_t)(((uint64_t)r << a.s_row) | ((uint64_t)(k - 1) << a.s_bin));
#pragma unroll
                    for (int v = 0; v < kV; ++v) {
                        if (mk[v]) {
                            if (hit[v]) {
                                const int pos = ws.n + (int)__builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(mk[v] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk[v], 0));
                                wbuf[pos] = make_uint2(hi | (uint32_t)(jb + v), __float_as_uint(acc[v]));
                            }
                            ws.n += __builtin_popcountll(mk[v]);
                        }
                    }
                }
            } else {
                float* dst = a.hp + ((int64_t)(k - 1) * a.T + r) * N + jb;
                const float* y = acc;
                if (tile_full && (N & 3) == 0) {
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
            if constexpr (kV % m == 0) {
#pragma unroll
                for (int v = 0; v < kV; ++v) acc[v] = acc[v] + w[m][v / m];
            } else if constexpr (m % kV == 0) {
#pragma unroll
                for (int v = 0; v < kV; ++v) acc[v] = acc[v] + w[m][0];
            } else {
                // the lane's kV bins span two source words: bin jb+v reads
                // word floor((sig + v)/m) of the lane's window
#pragma unroll
                for (int v = 0; v < kV; ++v) {
                    const int qv = v / m, s = v % m;
                    float val;
                    if (s == 0) val = qv ? w[m][1] : w[m][0];
                    else val = (sig[m] >= m - s) ? w[m][1] : w[m][0];
                    acc[v] = acc[v] + val;
                }
            }
            emit(m);
        });
    }
}

// Tiles [t_begin, t_end) of block b for a grid of g blocks over n tiles.
__device__ __forceinline__ void block_chunk(int64_t n, int64_t& t_begin, int64_t& t_end)
{
    const int64_t g = gridDim.x, b = blockIdx.x;
    const int64_t q = n / g, r = n % g;
    t_begin = b * q + (b < r ? b : r);
    t_end = t_begin + q + (b < r ? 1 : 0);
}

template <typename TIn, int H, int MODE>
__global__ __launch_bounds__(kThreads) void k_fused(TileArgs a, int stage_words, int64_t n_tiles)
{
    extern __shared__ __align__(16) float lds[];
    const Smem sh = carve(lds, stage_words, a.R, H);
    WaveState<H> ws;
    ws.n = 0;
    if (threadIdx.x < kMaxH) sh.cnt[threadIdx.x] = 0;

    int64_t t0, t1;
    block_chunk(n_tiles, t0, t1);
    for (int64_t t = t0; t < t1; ++t) run_tile<TIn, H, MODE>(a, t, sh, ws);

    if constexpr (MODE == kModeDetect) {
        if (ws.n) flush_wave(sh.cand + (threadIdx.x >> 6) * kWaveCandCap, ws.n, a.out, a.cap,
                             &a.counts[H], sh.cnt, a.s_bin, a.kmask);
        flush_counts<H>(sh, a.counts);
    }
}

// Batched persistent kernel: the grid walks the tiles of every FOP.
template <typename TIn, int H>
__global__ __launch_bounds__(kThreads) void k_batched(BatchArgs b, int stage_words)
{
    extern __shared__ __align__(16) float lds[];
    const Smem sh = carve(lds, stage_words, b.R, H);
    WaveState<H> ws;
    ws.n = 0;
    if (threadIdx.x < kMaxH) sh.cnt[threadIdx.x] = 0;
    constexpr int align_elems = sizeof(typename Io<TIn>::T) == 4 ? 4 : 8;

    int64_t t0, t1;
    block_chunk(b.tiles_total, t0, t1);
    if (t0 >= t1) return;
    // FOP holding tile t0 (binary search over the prefix of tile counts)
    int f;
    {
        int lo = 0, hi = b.n_fops - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.tile_prefix[mid] <= t0) lo = mid; else hi = mid - 1;
        }
        f = __builtin_amdgcn_readfirstlane(lo);
    }
    for (int64_t tf = t0; tf < t1; ++f) {
        const int64_t fb = b.tile_prefix[f], fe = min(b.tile_prefix[f + 1], t1);
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
        a.kmask = b.kmask;
        a.hp = nullptr;
        const bool ok = ((reinterpret_cast<uintptr_t>(a.fop) & 15) == 0) &&
                        (a.ld % align_elems == 0) && a.ld >= a.N;
        if (!ok) {
            if (threadIdx.x == 0 && tf == fb) a.counts[H] = ~0ull;
        } else {
            for (int64_t t = tf; t < fe; ++t) run_tile<TIn, H, kModeDetect>(a, t - fb, sh, ws);
            if (ws.n) {
                flush_wave(sh.cand + (threadIdx.x >> 6) * kWaveCandCap, ws.n, a.out, a.cap,
                           &a.counts[H], sh.cnt, a.s_bin, a.kmask);
                ws.n = 0;
            }
            flush_counts<H>(sh, a.counts);
        }
        tf = fe;
    }
}

template <typename TIn, int H>
static hipError_t launch_fused_t(int mode, const TileArgs& a, int64_t n_tiles, int grid,
                                 int lds_bytes, hipStream_t s)
{
    const int stage_words = (lds_bytes - smem_tail_bytes(a.R, H)) / 4;
    if (mode == kModeDetect) {
        auto k = k_fused<TIn, H, kModeDetect>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds_bytes, s, a, stage_words, n_tiles);
    } else {
        auto k = k_fused<TIn, H, kModeSum>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds_bytes, s, a, stage_words, n_tiles);
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
