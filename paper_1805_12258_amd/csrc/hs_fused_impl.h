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
// the m = 1 values of all its rows) are issued together, one tile ahead of
// the tile being summed.  The grid is persistent.
//
// Reuse: the staged ranges of a tile at bin tile x are the m = 1 data of bin
// tiles near x/m, read earlier by some other tile.  They come from the L2 of
// the reading XCD only if the same XCD read them shortly before.  Halving a
// tile index keeps the bits after its leading one, so the plan deals the bin
// tiles to the eight XCDs by those three bits and orders each XCD's list by
// the position inside that sub-range of the octave: x, x/2, x/4 and x/8 then
// fall on one XCD at nearly the same time, and the ranges of m = 2, 4, 8 are
// L2 hits.  Without a schedule, block b walks a contiguous chunk of tiles.
//
// Candidates: each wave appends its hits to a private LDS buffer (ballot +
// mbcnt, no atomics).  A full buffer is written out with one global atomic
// per wave that reserves its positions in the list, and the block's last
// buffers with one atomic for the whole block.  Per-plane counts are formed
// by a counting pass over the list afterwards (only candidates dropped for
// lack of capacity are counted here).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "hs_internal.h"

namespace hsk {

struct bf16_t {
    uint16_t bits;
};

template <typename TIn> struct Io;

// Storage access.  one(): a stored value as fp32 (exact).  Prefetched m = 1
// values stay in registers as raw storage bits (kV fp32 words, or kV halves
// packed two per word) and are decoded when the tile is summed, so their
// loads are not waited for at issue: four_raw() loads them, bits() gives one
// element's storage bits, decode() one value, kNegInf the bits of -inf.
template <> struct Io<float> {
    using T = float;
    static constexpr int kWords = kV;
    static constexpr uint32_t kNegInf = 0xff800000u;
    static __device__ __forceinline__ float one(const T* p) { return *p; }
    static __device__ __forceinline__ uint32_t bits(const T* p) { return __float_as_uint(*p); }
    static __device__ __forceinline__ void four_raw(const T* p, uint32_t* r)
    {
        const uint4 x = *reinterpret_cast<const uint4*>(p);
        r[0] = x.x; r[1] = x.y; r[2] = x.z; r[3] = x.w;
    }
    static __device__ __forceinline__ void put(uint32_t* r, int v, uint32_t b) { r[v] = b; }
    static __device__ __forceinline__ float decode(const uint32_t* r, int v) { return __uint_as_float(r[v]); }
};

template <> struct Io<_Float16> {
    using T = _Float16;
    static constexpr int kWords = kV / 2;
    static constexpr uint32_t kNegInf = 0xfc00u;
    static __device__ __forceinline__ float one(const T* p) { return (float)*p; }
    static __device__ __forceinline__ uint32_t bits(const T* p) { return *reinterpret_cast<const uint16_t*>(p); }
    static __device__ __forceinline__ void four_raw(const T* p, uint32_t* r)
    {
        const uint2 x = *reinterpret_cast<const uint2*>(p);
        r[0] = x.x; r[1] = x.y;
    }
    static __device__ __forceinline__ void put(uint32_t* r, int v, uint32_t b)
    {
        r[v >> 1] = (v & 1) ? (r[v >> 1] | (b << 16)) : b;
    }
    static __device__ __forceinline__ float decode(const uint32_t* r, int v)
    {
        const uint16_t b = (uint16_t)(r[v >> 1] >> (16 * (v & 1)));
        _Float16 h;
        __builtin_memcpy(&h, &b, 2);
        return (float)h;
    }
};

// Reduced-precision storage holds power * scale with scale a power of two.
// Sums are formed in storage units; the thresholds are scaled and the
// reported powers unscaled, both exactly, and power-of-two scaling commutes
// with every fp32 rounding of the sums, so planes and candidates equal those
// of the stored values converted to fp32 and divided by scale.
template <typename TIn> struct Scaled { static constexpr bool value = !std::is_same<TIn, float>::value; };

template <> struct Io<bf16_t> {
    using T = bf16_t;
    static constexpr int kWords = kV / 2;
    static constexpr uint32_t kNegInf = 0xff80u;
    static __device__ __forceinline__ float one(const T* p)
    {
        return __uint_as_float((uint32_t)p->bits << 16);
    }
    static __device__ __forceinline__ uint32_t bits(const T* p) { return p->bits; }
    static __device__ __forceinline__ void four_raw(const T* p, uint32_t* r)
    {
        const uint2 x = *reinterpret_cast<const uint2*>(p);
        r[0] = x.x; r[1] = x.y;
    }
    static __device__ __forceinline__ void put(uint32_t* r, int v, uint32_t b)
    {
        r[v >> 1] = (v & 1) ? (r[v >> 1] | (b << 16)) : b;
    }
    static __device__ __forceinline__ float decode(const uint32_t* r, int v)
    {
        return __uint_as_float((v & 1) ? (r[v >> 1] & 0xffff0000u) : (r[v >> 1] << 16));
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

// Shared-memory carve-up of one block.  The staging buffer and (when it
// covers only one tile) the row table are double-buffered: the loads of the
// next tile land in one copy while the current tile is summed from the other.
struct Smem {
    float* stage[2];              // staged source rows of all m >= 2 (fp32); 16-bit
                                  // storage uses stage[0] only
    uint16_t* raw[2];             // 16-bit storage: raw staged halves (DMA targets)
    float* rowtab[2];             // per row: staged-row offsets of m = 2..H, then
                                  // the H thresholds (both entries alias when the
                                  // table covers the whole plane)
    uint64_t* cand;               // [kWaves][kWaveCandCap] per-wave candidate buffers
                                  // (bin word in the low half, power bits high)
    int* cnt;                     // [kCntWords] bookkeeping of the block's candidate flush
    struct FlushParams* fp;       // where flushed candidates go
};

// Candidate output of the FOP being processed, kept in LDS so that the
// out-of-line flush needs only LDS pointers (few registers at the call).
struct FlushParams {
    hs_cand* out;
    int64_t cap;
    unsigned long long* counts;   // [H+1]: per-plane counts, then the total
    int32_t H;
    int32_t s_bin;
    uint32_t kmask;
};
static_assert(sizeof(FlushParams) <= kFlushParamBytes, "flush parameters");

template <int H, int EB>
__device__ __forceinline__ Smem carve(float* lds, int T, int R, bool whole)
{
    Smem s;
    float* tab;
    if constexpr (EB == 4) {
        s.stage[0] = lds;
        s.stage[1] = lds + stage_words(H);
        s.raw[0] = s.raw[1] = nullptr;
        tab = lds + 2 * stage_words(H);
    } else {
        constexpr int raw_bytes = (raw_halves(H) * 2 + 15) & ~15;
        s.stage[0] = s.stage[1] = lds;
        s.raw[0] = reinterpret_cast<uint16_t*>(lds + stage_words(H));
        s.raw[1] = reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(s.raw[0]) + raw_bytes);
        tab = reinterpret_cast<float*>(reinterpret_cast<char*>(s.raw[1]) + raw_bytes);
    }
    s.rowtab[0] = tab;
    const int trows = whole ? T : R;
    s.rowtab[1] = whole ? s.rowtab[0] : s.rowtab[0] + trows * row_table_stride(H);
    s.cand = reinterpret_cast<uint64_t*>(s.rowtab[1] + trows * row_table_stride(H));
    s.cnt = reinterpret_cast<int*>(s.cand + kWaves * kWaveCandCap);
    s.fp = reinterpret_cast<FlushParams*>(s.cnt + kCntWords);
    return s;
}

// Per-wave detection state (a wave-uniform value).
template <int H>
struct WaveState {
    int n;          // detection: entries in the wave's LDS buffer (wave-uniform)
    float lm[H];    // log-sum-exp: the lane's running maximum of each plane
    float ls[H];    //   and the sum of exp2((x - lm) * lse_c) over its values
};

// Merge two (max, sum) pairs of the log-sum-exp in fp32.  A pair with max
// -inf holds no value; the shift by the larger max keeps every term <= 1.
__device__ __forceinline__ void lse_pair_merge(float& M, float& S, float M2, float S2, float c)
{
    const float nm = fmaxf(M, M2);
    const float base = nm == -__builtin_inff() ? 0.0f : nm;
    S = S * __builtin_amdgcn_exp2f((M - base) * c) + S2 * __builtin_amdgcn_exp2f((M2 - base) * c);
    M = nm;
}

// Add the lane's kV values of one plane (storage units) to its pair.  The
// sum is rescaled only when some lane's maximum grows (a wave-uniform
// branch); otherwise the rescale factor would be exp2(0) = 1 and the result
// is the same, bitwise.  Called by the whole wave.
template <int V>
__device__ __forceinline__ void lse_add(const float (&x)[V], float& M, float& S, float c)
{
    const float xm = fmaxf(fmaxf(x[0], x[1]), fmaxf(x[2], x[3]));
    if (__builtin_amdgcn_ballot_w64(xm > M)) {
        const float nm = fmaxf(xm, M);
        const float base = nm == -__builtin_inff() ? 0.0f : nm;
        float t = 0.0f;
#pragma unroll
        for (int v = 0; v < V; ++v) t = t + __builtin_amdgcn_exp2f((x[v] - base) * c);
        S = S * __builtin_amdgcn_exp2f((M - base) * c) + t;
        M = nm;
    } else {
        const float base = M == -__builtin_inff() ? 0.0f : M;
        float t = 0.0f;
#pragma unroll
        for (int v = 0; v < V; ++v) t = t + __builtin_amdgcn_exp2f((x[v] - base) * c);
        S = S + t;
    }
}

__device__ __forceinline__ uint64_t read_first_u64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Write a wave's buffered candidates to global memory (one atomic per wave
// reserves their positions in the list).  The per-plane counts of the
// entries that fit are formed afterwards from the list itself (a counting
// pass); entries past the capacity are dropped, and only those are counted
// here, per plane.
__device__ __forceinline__ void store_cands(const uint64_t* wbuf, int n, unsigned long long base, hs_cand* out,
                                            int64_t cap, unsigned long long* counts, int s_bin, uint32_t kmask)
{
    const int lane = threadIdx.x & 63;
    for (int e0 = 0; e0 < n; e0 += 64) {   // uniform trip count
        const int e = e0 + lane;
        if (e < n) {
            const uint64_t c = wbuf[e];
            if ((int64_t)(base + e) < cap) reinterpret_cast<uint64_t*>(out)[base + e] = c;
            else atomicAdd(&counts[((uint32_t)c >> s_bin) & kmask], 1ull);
        }
    }
}

__device__ __forceinline__ void flush_wave(const uint64_t* wbuf, int n, hs_cand* out, int64_t cap,
                                           unsigned long long* counts, int H, int s_bin, uint32_t kmask)
{
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&counts[H], (unsigned long long)n);
    base = read_first_u64(base);
    store_cands(wbuf, n, base, out, cap, counts, s_bin, kmask);
}

// Flush every wave's buffer with one atomic for the whole block (called by
// the whole block; contains barriers).  `n` is the calling wave's fill; the
// block's bookkeeping uses the LDS words at sh.cnt.
template <int H>
__device__ __forceinline__ void flush_block(const Smem& sh, int n, unsigned long long* counts, hs_cand* out,
                                            int64_t cap, int s_bin, uint32_t kmask)
{
    int* bf = sh.cnt;   // [0, kWaves): fills; [kWaves, 2 kWaves): offsets; then the base (2 words)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) bf[wave] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < kWaves; ++w) {
            bf[kWaves + w] = acc;
            acc += bf[w];
        }
        const unsigned long long b = acc ? atomicAdd(&counts[H], (unsigned long long)acc) : 0ull;
        bf[2 * kWaves] = (int)(uint32_t)b;
        bf[2 * kWaves + 1] = (int)(uint32_t)(b >> 32);
    }
    __syncthreads();
    const unsigned long long base = ((unsigned long long)(uint32_t)bf[2 * kWaves + 1] << 32) |
                                    (uint32_t)bf[2 * kWaves];
    store_cands(sh.cand + wave * kWaveCandCap, n, base + (unsigned long long)bf[kWaves + wave], out, cap, counts,
                s_bin, kmask);
    __syncthreads();
}

// Out-of-line flush of the calling wave's buffer (n entries): the rare path
// inside the row loop, kept out of line so the loop stays small.
__device__ __noinline__ void flush_call(int n, const uint64_t* wbuf, const FlushParams* fp)
{
    flush_wave(wbuf, n, fp->out, fp->cap, fp->counts, fp->H, fp->s_bin, fp->kmask);
}

__device__ __forceinline__ void set_flush_params(const Smem& sh, hs_cand* out, int64_t cap,
                                                 unsigned long long* counts, int H, int s_bin, uint32_t kmask)
{
    if (threadIdx.x == 0) {
        sh.fp->out = out;
        sh.fp->cap = cap;
        sh.fp->counts = counts;
        sh.fp->H = H;
        sh.fp->s_bin = s_bin;
        sh.fp->kmask = kmask;
    }
}

// Append the hits of one (row, plane) to the wave's LDS buffer.  Called by
// the whole wave (uniform control flow): positions come from wave ballots.
// `lanes` is the number of lanes with a hit: the call adds at most V * lanes
// entries.  The buffer is written out only when that many might not fit, so
// that a flush carries a nearly full buffer (each flush costs one atomic on
// the list's shared counter).
template <int V, int H>
__device__ __forceinline__ void emit_hits(const float* acc, float t, int r, int k, int64_t jb, int lanes,
                                          const TileArgs& a, const Smem& sh, WaveState<H>& ws,
                                          uint64_t* wbuf)
{
    const uint32_t hi = (uint32_t)(((uint64_t)r << a.s_row) | ((uint64_t)(k - 1) << a.s_bin));
    static_assert(kWaveCandCap >= V * 64, "candidate buffer");
    if (__builtin_expect(ws.n + V * lanes > kWaveCandCap, 0)) {
        flush_call(ws.n, wbuf, sh.fp);
        ws.n = 0;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const bool hit = acc[v] > t;
        const uint64_t mk = __builtin_amdgcn_ballot_w64(hit);
        if (mk) {
            const int pre = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
            // sums are in storage units: the reported power is unscaled
            if (hit)
                wbuf[ws.n + pre] = ((uint64_t)__float_as_uint(acc[v] * a.inv_scale) << 32) | (hi | (uint32_t)(jb + v));
            ws.n += __builtin_popcountll(mk);
        }
    }
}

// Row block of a tile: rows [r0, r0 + nr) of the plane.
struct RowGeo {
    int rb, r0, nr;
};

__device__ __forceinline__ void row_geo(const TileArgs& a, int rb, RowGeo& g)
{
    g.rb = rb;
    g.r0 = rb * a.R;
    g.nr = min(g.r0 + a.R, a.T) - g.r0;
}

// First source row staged for stretch factor m in the row block starting at
// plane row r0: floor((r0 - c) / m) + c (Eq. 1 with the template index i = r - c).
template <int m>
__device__ __forceinline__ int src_row_lo(int r0, int c)
{
    return floordiv32(r0 - c, m) + c;
}

// First source word staged for stretch factor m in the bin tile starting at j0.
template <int m>
__device__ __forceinline__ uint32_t src_col_lo(int j0)
{
    const uint32_t blo = (uint32_t)j0 / (uint32_t)m;
    return stage_aligned(m) ? blo : (blo & ~3u);
}

// Per-lane byte offsets of this wave's LDS-DMA pieces, relative to the first
// staged element of the piece's stretch factor (they depend on the row pitch
// ld only, so they are computed once per launch or FOP): fp32 pieces (EB = 4)
// of the fp32 staging, or raw pieces (EB = 2) of 16-bit storage.  Lanes past
// the end of a region get 0xffffffff, which every row limit rejects.
template <int H, int EB>
__device__ __forceinline__ void dma_offsets(int64_t ld, uint32_t (&voff)[dma_slot_regs(H, EB)])
{
    const uint32_t lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t ldb = (uint32_t)ld * (uint32_t)EB;
#pragma unroll
    for (int s = 0; s < dma_slots(H, EB); ++s) {
        const int g = s * kWaves + wave;
        uint32_t off = 0xffffffffu;
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr int RW = EB == 4 ? stage_row_words(m) : raw_row_halves(m);
            constexpr int REG = EB == 4 ? stage_region_words(m) : raw_region_halves(m);
            constexpr int CB = EB == 4 ? stage_chunk_begin(m) : raw_chunk_begin(m);
            constexpr int CE = EB == 4 ? stage_chunk_begin(m + 1) : raw_chunk_begin(m + 1);
            if (g >= CB && g < CE) {
                const uint32_t w = ((uint32_t)(g - CB) * 64u + lane) * (16u / EB);
                if (w < (uint32_t)REG) {
                    const uint32_t row = w / RW, col = w - row * RW;
                    off = row * ldb + col * (uint32_t)EB;
                }
            }
        });
        voff[s] = off;
    }
    if (dma_slots(H, EB) == 0) voff[0] = 0xffffffffu;
}

// LDS-DMA of the pieces of wave W for the tile (r0, j0): piece g = s kWaves + W
// of region m copies 64 x 16 bytes of source rows src_row_lo<m> + .. into the
// staging buffer (fp32, EB = 4) or the raw buffer (16-bit, EB = 2, rows
// starting at floor(j0/m) rounded down to 8 halves).  Source rows past the
// plane are masked (row limit); the columns of a full bin tile all lie inside
// the plane's rows.
template <int H, int W, int EB>
__device__ __forceinline__ void dma_wave(const TileArgs& a, int r0, int j0, void* dst,
                                         const uint32_t (&voff)[dma_slot_regs(H, EB)])
{
    static_for<0, dma_slots(H, EB) - 1>([&](auto sc) {   // empty for H = 1
        constexpr int s = decltype(sc)::value;
        constexpr int g = s * kWaves + W;
        constexpr int total = EB == 4 ? stage_total_chunks(H) : raw_total_chunks(H);
        if constexpr (g < total) {
            constexpr int m = EB == 4 ? stage_chunk_m(g) : raw_chunk_m(g);
            constexpr int c = g - (EB == 4 ? stage_chunk_begin(m) : raw_chunk_begin(m));
            const int lo = src_row_lo<m>(r0, a.c);
            const uint32_t col0 = EB == 4 ? src_col_lo<m>(j0) : (((uint32_t)j0 / (uint32_t)m) & ~7u);
            const char* base = reinterpret_cast<const char*>(a.fop) + ((int64_t)lo * a.ld + col0) * EB;
            const uint64_t lim64 = (uint64_t)(a.T - lo) * (uint64_t)a.ld * (uint64_t)EB;
            const uint32_t lim = lim64 > 0xffffffffull ? 0xffffffffu : (uint32_t)lim64;
            char* d = reinterpret_cast<char*>(dst) +
                      (EB == 4 ? (stage_offset(m) + c * kDmaWords) * 4 : (raw_offset(m) + c * kDmaHalves) * 2);
            if (voff[s] < lim)
                __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(base + voff[s]), (lds_ptr_t)d,
                                                 16, 0, 0);
        }
    });
}

// 16-bit storage: the raw staged halves of a tile (all DMA pieces landed)
// to the fp32 staging layout, four words per thread and step.  The sums stay
// in storage units (power * scale): the thresholds are scaled to match and
// the emitted powers are unscaled, all exactly, since scale is a power of
// two.  Raw reads go through 64-bit integers (LDS accesses with type-based
// alias information are not ordered after the DMA of the next tile).
template <typename TIn, int H>
__device__ __forceinline__ void convert_tile(const uint16_t* raw, float* stage, int j0)
{
    static_for<2, H>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        constexpr int RW = stage_row_words(m);
        constexpr int RH = raw_row_halves(m);
        const int shift = stage_aligned(m) ? 0 : (int)(((uint32_t)j0 / (uint32_t)m) & 4u);
        for (int q = threadIdx.x; q < stage_rows(m) * RW / 4; q += kThreads) {
            const int w = 4 * q;
            const int row = w / RW, col = w - row * RW;
            const uint64_t h4 = *reinterpret_cast<const uint64_t*>(raw + raw_offset(m) + row * RH + col + shift);
            float* o = stage + stage_offset(m) + w;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint16_t bits = (uint16_t)(h4 >> (16 * v));
                if constexpr (std::is_same<TIn, bf16_t>::value) {
                    o[v] = __uint_as_float((uint32_t)bits << 16);
                } else {
                    _Float16 hv;
                    __builtin_memcpy(&hv, &bits, 2);
                    o[v] = (float)hv;
                }
            }
        }
    });
}

// Start every load of tile (g.rb, bt): the shrunken source ranges into the
// staging buffer `stage` (fp32) or `raw` (16-bit storage, full tiles), the
// m = 1 values of the wave's rows into `x`, and (when the row table does not
// cover the whole plane) the tile's row table into `rowtab`.  Nothing is
// waited for here.  All values stay in storage units (power * scale).
template <typename TIn, int H, int MODE, bool FULL>
__device__ __forceinline__ void issue_tile(const TileArgs& a, const RowGeo& g, int bt,
                                           float* stage, uint16_t* raw, float* rowtab,
                                           const uint32_t (&voff)[dma_slot_regs(H, sizeof(typename Io<TIn>::T))],
                                           uint32_t (&x)[kRowsPerWave][kV])
{
    using Ld = Io<TIn>;
    using T = typename Ld::T;
    constexpr int EB = sizeof(T);
    const T* __restrict__ fop = reinterpret_cast<const T*>(a.fop);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = (int)a.N;
    // Bin arithmetic is 32-bit (N < 2^31).
    const int j0 = bt * kTileBins;
    const int64_t ld = a.ld;

    // 1. Source ranges.  Full tiles (j0 + kTileBins <= N): LDS-DMA pieces
    // with precomputed lane offsets, into the fp32 staging (fp32) or the raw
    // buffer (16-bit, converted later).  Partial tiles: every thread converts
    // words one at a time, with bounds checks.
    if constexpr (FULL) {
        void* dst = EB == 4 ? static_cast<void*>(stage) : static_cast<void*>(raw);
        switch (wave) {
        case 0: dma_wave<H, 0, EB>(a, g.r0, j0, dst, voff); break;
        case 1: dma_wave<H, 1, EB>(a, g.r0, j0, dst, voff); break;
        case 2: dma_wave<H, 2, EB>(a, g.r0, j0, dst, voff); break;
        case 3: dma_wave<H, 3, EB>(a, g.r0, j0, dst, voff); break;
        case 4: dma_wave<H, 4, EB>(a, g.r0, j0, dst, voff); break;
        case 5: dma_wave<H, 5, EB>(a, g.r0, j0, dst, voff); break;
        case 6: dma_wave<H, 6, EB>(a, g.r0, j0, dst, voff); break;
        default: dma_wave<H, 7, EB>(a, g.r0, j0, dst, voff); break;
        }
    } else {
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr int RW = stage_row_words(m);
            const int lo = src_row_lo<m>(g.r0, a.c);
            const int cb = (int)src_col_lo<m>(j0);
            for (int e = threadIdx.x; e < stage_region_words(m); e += kThreads) {
                const int row = e / RW, col = e - row * RW;
                float v = 0.0f;
                if (lo + row < a.T && cb + col < N) v = Ld::one(fop + (int64_t)(lo + row) * ld + cb + col);
                stage[stage_offset(m) + e] = v;
            }
        });
    }

    // 2. The m = 1 values of every row this wave owns.
    if constexpr (FULL) {
        // unconditional loads (rows past the tile re-read its last row and
        // are ignored) land straight in their registers, so nothing waits
        // for them before the tile is summed
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) {
            const int rr = min(wave + kWaves * q, g.nr - 1);
            const T* rowp = fop + (int64_t)(g.r0 + rr) * ld + j0;
            Ld::four_raw(rowp + kV * lane, x[q]);
        }
    } else {
        const int jb = j0 + kV * lane;
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) {
            const int rr = wave + kWaves * q;
            const T* p = fop + (int64_t)(g.r0 + rr) * ld + jb;
            // bins past the end start at -inf: no sum of them can pass a
            // threshold (-inf + x is -inf or NaN)
#pragma unroll
            for (int v = 0; v < kV; ++v)
                Ld::put(x[q], v, (rr < g.nr && jb + v < N) ? Ld::bits(p + v) : Ld::kNegInf);
        }
    }

    // 3. Row table of the tile (large planes only): per tile row, where each
    // stretch factor's source row sits in the staging buffer, and the row's
    // thresholds.  Per-row scalar work would otherwise dominate the row loop.
    if (!a.table_whole) {
        constexpr int RS = row_table_stride(H);
        constexpr int SO = row_table_thr_offset(H);
        for (int e = threadIdx.x; e < g.nr * RS; e += kThreads) {
            const int rr = e / RS, col = e - rr * RS;
            const int r = g.r0 + rr;
            float val = 0.0f;
            if (col < H - 1) {
                int off = 0;
                static_for<2, H>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if (col == m - 2)
                        off = stage_offset(m) +
                              (src_row_lo<m>(r, a.c) - src_row_lo<m>(g.r0, a.c)) * stage_row_words(m);
                });
                val = __int_as_float(off);
            } else if (MODE == kModeDetect && col >= SO && col < SO + H) {
                // thresholds exist only in the detection mode (a.ta is null otherwise)
                val = a.ta[(int64_t)(col - SO) * a.T + r] * a.scale;   // storage units (exact)
            }
            rowtab[e] = val;
        }
    }
}

// Form the planes of one tile whose loads have completed (after a barrier):
// HP_k for k = 1..H in the order of Eq. 2, detected or stored.
template <typename TIn, int H, int MODE, bool FULL>
__device__ __forceinline__ void compute_tile(const TileArgs& a, const RowGeo& g, int bt,
                                             const Smem& sh, const float* stage,
                                             const float* rowtab,
                                             const uint32_t (&x)[kRowsPerWave][kV], WaveState<H>& ws)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j0 = bt * kTileBins;
    const int r0 = g.r0;
    const int nr = g.nr;
    const int N = (int)a.N;
    const int jb = j0 + kV * lane;
    constexpr int RS = row_table_stride(H);
    constexpr int SO = row_table_thr_offset(H);
    const int trow0 = a.table_whole ? r0 : 0;          // table row of tile row 0

    // Per-lane view of the staged rows: the lane's first source word of each
    // stretch factor (relative to the staged row, which starts at
    // src_col_lo) and where its kV bins cross to the next word.
    int loff[H + 1], sig[H + 1];
#pragma unroll
    for (int m = 2; m <= H; ++m) {
        const int blo = (int)((uint32_t)j0 / (uint32_t)m);
        const int t = (j0 - blo * m) + kV * lane;     // (j0 mod m) + kV * lane
        loff[m] = t / m + (stage_aligned(m) ? 0 : (blo & 3));
        sig[m] = t % m;
    }

    uint64_t* wbuf = sh.cand + wave * kWaveCandCap;
    // rows unrolled with static register indices (a dynamic index into the
    // prefetched rows would make every load complete before the tile starts)
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
        const int rr = wave + kWaves * q;
        if (rr >= nr) break;
        const int r = r0 + rr;
        // All LDS reads of the row first (row table and staged source words),
        // so their latencies overlap; the candidate writes below could
        // otherwise alias them and serialise every read.
        const float* rt = rowtab + (trow0 + rr) * RS;
        // plain float reads (merged into 16-byte reads): LDS accesses through
        // aggregate types carry no type-based alias information, and the
        // compiler then orders them after every LDS-DMA in flight
        float tab[RS];
#pragma unroll
        for (int u = 0; u < RS; ++u) tab[u] = rt[u];
        float w[H + 1][2];
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const float* p = stage + loff[m] + __float_as_int(tab[m - 2]);
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
        for (int v = 0; v < kV; ++v) acc[v] = Io<TIn>::decode(x[q], v);

        auto emit = [&](int k) {
            if constexpr (MODE == kModeDetect) {
                const float t = tab[SO + k - 1];
                // cheap wave test first: the largest of the lane's kV sums
                // (NaN operands are ignored by max and fail the compare)
                const float mx = fmaxf(fmaxf(acc[0], acc[1]), fmaxf(acc[2], acc[3]));
                const uint64_t any = __builtin_amdgcn_ballot_w64(mx > t);
                if (__builtin_expect(any != 0, 0))
                    emit_hits<kV, H>(acc, t, r, k, jb, __builtin_popcountll(any), a, sh, ws, wbuf);
            } else if constexpr (MODE == kModeLse) {
                float xv[kV];
#pragma unroll
                for (int v = 0; v < kV; ++v) xv[v] = (FULL || jb + v < N) ? acc[v] : -__builtin_inff();
                lse_add<kV>(xv, ws.lm[k - 1], ws.ls[k - 1], a.lse_c);
            } else {
                float* dst = a.hp + ((int64_t)(k - 1) * a.T + r) * N + jb;
                float o[kV];
#pragma unroll
                for (int v = 0; v < kV; ++v) o[v] = Scaled<TIn>::value ? acc[v] * a.inv_scale : acc[v];
                if (FULL && (N & 3) == 0) {
                    *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
                } else {
#pragma unroll
                    for (int v = 0; v < kV; ++v)
                        if (jb + v < N) dst[v] = o[v];
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

// Meet the other waves after this wave's LDS accesses are done, without
// waiting for its loads in flight (no release fence, which would wait for
// every load); the empty asm statements keep the compiler from moving memory
// accesses across the barrier.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt and expcnt not waited for
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// The full bin tiles one block visits: `count` tiles, either entries
// ids[0], ids[stride], ... of a schedule list ((rb << 24) | bt), or, with
// ids null, the row-block-major numbers first, first + 1, ... (tile number
// t = rb * n_full + bt).
struct TileSeq {
    const uint32_t* ids;
    int64_t stride;
    int64_t first;
    int64_t count;
};

__device__ __forceinline__ void seq_tile(const TileSeq& q, int n_full, int64_t k, int& rb, int& bt)
{
    if (q.ids) {
        const uint32_t id = q.ids[k * q.stride];
        rb = (int)(id >> 24);
        bt = (int)(id & 0xffffffu);
    } else {
        const int64_t t = q.first + k;
        rb = (int)(t / n_full);
        bt = (int)(t - (int64_t)rb * n_full);
    }
}

// Full tiles of a sequence, processed with the loads of the next tile in
// flight while the current one is summed; the two halves of the loop body
// use the two buffers with static register indices, so no wait on the
// in-flight loads is implied.  16-bit storage converts the landed raw tile
// into the one fp32 staging buffer first.
template <typename TIn, int H, int MODE>
__device__ __forceinline__ void run_full(const TileArgs& a, const TileSeq& q, const Smem& sh,
                                         const uint32_t (&voff)[dma_slot_regs(H, sizeof(typename Io<TIn>::T))],
                                         WaveState<H>& ws)
{
    constexpr bool RAW = sizeof(typename Io<TIn>::T) == 2;
    const int n_full = (int)(a.N / kTileBins);
    if (q.count <= 0) return;
    uint32_t xa[kRowsPerWave][kV], xb[kRowsPerWave][kV];   // raw storage bits
    int rb, bt;
    seq_tile(q, n_full, 0, rb, bt);
    RowGeo gc, gn;                    // row geometry of the current / next tile
    row_geo(a, rb, gc);
    gn = gc;
    __syncthreads();   // the previous run is done with every buffer
    issue_tile<TIn, H, MODE, true>(a, gc, bt, sh.stage[0], sh.raw[0], sh.rowtab[0], voff, xa);
    int64_t k = 0;
    // one tile from buffer set B (0 or 1), the next tile's loads into 1 - B
    auto step = [&](auto bc) {
        constexpr int B = decltype(bc)::value;
        auto& xc = B == 0 ? xa : xb;
        auto& xn = B == 0 ? xb : xa;
        const bool more = k + 1 < q.count;
        int rb1 = gc.rb, bt1 = bt;
        if (more) {
            if (q.ids) {
                seq_tile(q, n_full, k + 1, rb1, bt1);
            } else if (++bt1 == n_full) {
                bt1 = 0;
                ++rb1;
            }
            if (rb1 != gc.rb) row_geo(a, rb1, gn);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (more)
            issue_tile<TIn, H, MODE, true>(a, gn, bt1, sh.stage[1 - B], sh.raw[1 - B], sh.rowtab[1 - B], voff, xn);
        if constexpr (RAW) {
            convert_tile<TIn, H>(sh.raw[B], sh.stage[0], bt * kTileBins);
            lds_barrier();
        }
        compute_tile<TIn, H, MODE, true>(a, gc, bt, sh, RAW ? sh.stage[0] : sh.stage[B], sh.rowtab[B], xc, ws);
        gc = gn; bt = bt1;
        return ++k < q.count;
    };
    for (;;) {
        if (!step(std::integral_constant<int, 0>{})) break;
        if (!step(std::integral_constant<int, 1>{})) break;
    }
}

// The partial last bin tile of row blocks [begin, end) (N not a multiple of
// kTileBins): a plain load-wait-compute loop with bounds checks.
template <typename TIn, int H, int MODE>
__device__ __forceinline__ void run_partial(const TileArgs& a, int64_t begin, int64_t end, const Smem& sh,
                                            const uint32_t (&voff)[dma_slot_regs(H, sizeof(typename Io<TIn>::T))],
                                            WaveState<H>& ws)
{
    const int n_full = (int)(a.N / kTileBins);
    uint32_t xa[kRowsPerWave][kV];
    for (int64_t t = begin; t < end; ++t) {
        RowGeo g;
        row_geo(a, (int)t, g);
        __syncthreads();   // every load in flight has landed; the buffers are free
        issue_tile<TIn, H, MODE, false>(a, g, n_full, sh.stage[0], sh.raw[0], sh.rowtab[0], voff, xa);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        compute_tile<TIn, H, MODE, false>(a, g, n_full, sh, sh.stage[0], sh.rowtab[0], xa, ws);
    }
}

// Tiles [begin, end) of the numbering that puts the full bin tiles first,
// row-block-major, then the partial last bin tile of every row block.
template <typename TIn, int H, int MODE>
__device__ __forceinline__ void run_tiles(const TileArgs& a, int64_t begin, int64_t end, const Smem& sh,
                                          const uint32_t (&voff)[dma_slot_regs(H, sizeof(typename Io<TIn>::T))],
                                          WaveState<H>& ws)
{
    const int64_t full_total = (int64_t)a.row_blocks * (a.N / kTileBins);
    const int64_t fend = end < full_total ? end : full_total;
    const TileSeq q{nullptr, 1, begin, fend - begin};
    run_full<TIn, H, MODE>(a, q, sh, voff, ws);
    run_partial<TIn, H, MODE>(a, (begin > full_total ? begin : full_total) - full_total, end - full_total,
                              sh, voff, ws);
}

// Row table for every row of the plane, built once per launch by the whole
// block: entries of row r refer to the staging layout of r's row block.
template <int H, int MODE>
__device__ __forceinline__ void build_whole_table(int T, int R, int c, const float* ta, float scale,
                                                  float* rowtab)
{
    constexpr int RS = row_table_stride(H);
    constexpr int SO = row_table_thr_offset(H);
    for (int e = threadIdx.x; e < T * RS; e += kThreads) {
        const int r = e / RS, col = e - r * RS;
        float val = 0.0f;
        if (col < H - 1) {
            const int r0 = (r / R) * R;
            int off = 0;
            static_for<2, H>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                if (col == m - 2)
                    off = stage_offset(m) + (src_row_lo<m>(r, c) - src_row_lo<m>(r0, c)) * stage_row_words(m);
            });
            val = __int_as_float(off);
        } else if (MODE == kModeDetect && col >= SO && col < SO + H) {
            val = ta[(int64_t)(col - SO) * T + r] * scale;   // storage units (exact)
        }
        rowtab[e] = val;
    }
}

// The block's (max, sum) pair of every plane: the 64 lanes of a wave are
// merged with xor shuffles (both partners of a step compute the same pair,
// fp32 addition being commutative), the waves in order through LDS (the
// candidate buffers, unused in this mode); thread k writes plane k.
template <int H>
__device__ __forceinline__ void lse_block_pairs(const Smem& sh, WaveState<H>& ws, const TileArgs& a)
{
    float* buf = reinterpret_cast<float*>(sh.cand);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        float M = ws.lm[k], S = ws.ls[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float M2 = __shfl_xor(M, off, 64), S2 = __shfl_xor(S, off, 64);
            lse_pair_merge(M, S, M2, S2, a.lse_c);
        }
        if (lane == 0) {
            buf[(wave * H + k) * 2] = M;
            buf[(wave * H + k) * 2 + 1] = S;
        }
    }
    __syncthreads();
    if (threadIdx.x < H) {
        const int k = threadIdx.x;
        float M = buf[k * 2], S = buf[k * 2 + 1];
        for (int w = 1; w < kWaves; ++w) lse_pair_merge(M, S, buf[(w * H + k) * 2], buf[(w * H + k) * 2 + 1], a.lse_c);
        a.lse_part[((int64_t)blockIdx.x * H + k) * 2] = M;
        a.lse_part[((int64_t)blockIdx.x * H + k) * 2 + 1] = S;
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

// Occupancy asked of the compiler: four waves per SIMD (at most 128 VGPRs)
// where that needs no scratch, otherwise its own choice.
template <int H> constexpr int fused_min_waves() { return H <= 8 ? 4 : 1; }
template <int H> constexpr int batched_min_waves() { return H <= 4 ? 4 : 1; }

template <typename TIn, int H, int MODE>
__global__ __launch_bounds__(kThreads, fused_min_waves<H>()) void k_fused(TileArgs a, int64_t n_tiles)
{
    extern __shared__ __align__(16) float lds[];
    constexpr int EB = sizeof(typename Io<TIn>::T);
    const Smem sh = carve<H, EB>(lds, a.T, a.R, a.table_whole != 0);
    WaveState<H> ws;
    ws.n = 0;
    if constexpr (MODE == kModeLse) {
#pragma unroll
        for (int k = 0; k < H; ++k) {
            ws.lm[k] = -__builtin_inff();
            ws.ls[k] = 0.0f;
        }
    }
    if (a.table_whole) build_whole_table<H, MODE>(a.T, a.R, a.c, a.ta, a.scale, sh.rowtab[0]);

    uint32_t voff[dma_slot_regs(H, EB)];
    dma_offsets<H, EB>(a.ld, voff);

    if (MODE == kModeDetect) set_flush_params(sh, a.out, a.cap, a.counts, H, a.s_bin, a.kmask);

    if (a.sched) {
        // full tiles from the list of this block's XCD (blocks are dealt to
        // the eight XCDs in turn), partial tiles in contiguous chunks
        const int x = blockIdx.x & 7;
        const int64_t i = blockIdx.x >> 3;
        const int64_t per = ((int64_t)gridDim.x - x + 7) >> 3;   // blocks on list x
        const int64_t lo = a.sched[x], len = (int64_t)a.sched[x + 1] - lo;
        const TileSeq q{a.sched + 9 + lo + i, per, 0, len > i ? (len - i + per - 1) / per : 0};
        run_full<TIn, H, MODE>(a, q, sh, voff, ws);
        int64_t p0, p1;
        block_chunk((a.N % kTileBins) ? a.row_blocks : 0, p0, p1);
        run_partial<TIn, H, MODE>(a, p0, p1, sh, voff, ws);
    } else {
        int64_t t0, t1;
        block_chunk(n_tiles, t0, t1);
        run_tiles<TIn, H, MODE>(a, t0, t1, sh, voff, ws);
    }

    if constexpr (MODE == kModeDetect) flush_block<H>(sh, ws.n, a.counts, a.out, a.cap, a.s_bin, a.kmask);
    if constexpr (MODE == kModeLse) lse_block_pairs<H>(sh, ws, a);
}

// Batched persistent kernel: the grid walks the tiles of every FOP.
template <typename TIn, int H>
__global__ __launch_bounds__(kThreads, batched_min_waves<H>()) void k_batched(BatchArgs b)
{
    extern __shared__ __align__(16) float lds[];
    constexpr int EB = sizeof(typename Io<TIn>::T);
    const Smem sh = carve<H, EB>(lds, b.T, b.R, b.table_whole != 0);
    WaveState<H> ws;
    ws.n = 0;
    constexpr int align_elems = sizeof(typename Io<TIn>::T) == 4 ? 4 : 8;

    int64_t t0, t1;
    block_chunk(b.tiles_total, t0, t1);
    if (t0 >= t1) return;
    if (b.table_whole) build_whole_table<H, kModeDetect>(b.T, b.R, b.c, b.ta, b.scale, sh.rowtab[0]);
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
        a.table_whole = b.table_whole;
        a.hp = nullptr;
        a.sched = nullptr;
        constexpr int eb = sizeof(typename Io<TIn>::T);
        const bool ok = ((reinterpret_cast<uintptr_t>(a.fop) & 15) == 0) &&
                        (a.ld % align_elems == 0) && a.ld >= a.N &&
                        (a.ld * stage_rows(2) + kTileBins) * eb < ((int64_t)1 << 32);
        if (!ok) {
            if (threadIdx.x == 0 && tf == fb) a.counts[H] = ~0ull;
        } else {
            uint32_t voff[dma_slot_regs(H, EB)];
            dma_offsets<H, EB>(a.ld, voff);
            set_flush_params(sh, a.out, a.cap, a.counts, H, a.s_bin, a.kmask);
            // tiles of this FOP segment, numbered from the FOP's first tile
            run_tiles<TIn, H, kModeDetect>(a, tf - fb, fe - fb, sh, voff, ws);
            flush_block<H>(sh, ws.n, a.counts, a.out, a.cap, a.s_bin, a.kmask);
            ws.n = 0;
        }
        tf = fe;
    }
}

// Persistent grid: as many blocks as the device holds at once (occupancy of
// this kernel at this LDS size), at most one per tile.  A positive `grid`
// overrides.
template <typename K>
static int resident_grid(K kernel, int lds_bytes, int64_t n_tiles, int grid)
{
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kernel, kThreads,
                                                         lds_bytes) != hipSuccess || per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if (grid > n_tiles) grid = (int)n_tiles;
    return grid < 1 ? 1 : grid;
}

template <typename TIn, int H>
static hipError_t launch_fused_t(int mode, const TileArgs& a, int64_t n_tiles, int grid,
                                 int lds_bytes, hipStream_t s)
{
    // a schedule needs a block on each of its eight lists
    TileArgs b = a;
    if (mode == kModeDetect) {
        auto k = k_fused<TIn, H, kModeDetect>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        const int g = resident_grid(k, lds_bytes, n_tiles, grid);
        if (g < 8) b.sched = nullptr;
        hipLaunchKernelGGL(k, dim3(g), dim3(kThreads), lds_bytes, s, b, n_tiles);
    } else if (mode == kModeSum) {
        auto k = k_fused<TIn, H, kModeSum>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        const int g = resident_grid(k, lds_bytes, n_tiles, grid);
        if (g < 8) b.sched = nullptr;
        hipLaunchKernelGGL(k, dim3(g), dim3(kThreads), lds_bytes, s, b, n_tiles);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The statistic's mode (fp32 storage only; its own translation units).
template <int H>
static hipError_t launch_stat_t(int mode, const TileArgs& a, int64_t n_tiles, int grid, int lds_bytes,
                                hipStream_t s)
{
    TileArgs b = a;
    if (mode == kModeLse) {
        // the caller fixes the grid (one partial pair per block)
        auto k = k_fused<float, H, kModeLse>;
        if (grid < 1 || grid > kLseMaxBlocks || grid > n_tiles) return hipErrorInvalidValue;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (grid < 8) b.sched = nullptr;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds_bytes, s, b, n_tiles);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TIn, int H>
static hipError_t launch_batched_t(const BatchArgs& b, int grid, int lds_bytes, hipStream_t s)
{
    auto k = k_batched<TIn, H>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    const int g = resident_grid(k, lds_bytes, b.tiles_total, grid);
    hipLaunchKernelGGL(k, dim3(g), dim3(kThreads), lds_bytes, s, b);
    return hipGetLastError();
}

}  // namespace hsk
