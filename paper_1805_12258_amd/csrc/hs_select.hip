// Per-plane capped candidate lists (Sec. III: the module returns at most
// N_cand candidates for each of the N_hp planes), under three policies:
//   top      the N_cand largest powers of each plane, ties to the smaller
//            CL1 word, listed in that order (powers in the IEEE total order
//            of their bits, -0 below +0);
//   last     the N_cand candidates met last when the loops run in Algorithm
//            2 order (bin, template, plane: ascending (j, row) within a
//            plane) or Algorithm 1 order (plane, template, bin: ascending
//            (row, j)), listed oldest first (Sec. IV-A).
// Each policy is "the N_cand largest of a unique 64-bit key per plane".
//
// Bounded selection, no full sort, in five passes over the list: (1) per
// block, the count and key range of each plane; (2) per block, a histogram
// over 1024 (512 above eight planes) bins of equal width spanning each
// plane's key range; (3) per plane, the summed histogram's suffix scan gives
// the bin holding the N_cand-th largest key; (4) entries above that bin are
// kept, entries in it set aside; (5) per plane, the bin's largest keys
// complete the list (ranked in LDS; a bin too large for LDS is split again
// over its own range first) and the kept entries are ranked in the
// policy's order.  Caps above kSelLdsCand fall back (top policy
// only) to two stable rocPRIM radix passes over a copy of the list: by CL1
// word, then by (plane, descending power).
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "hs_internal.h"

namespace hsk {

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kSelThreads = 256;

// Descending order of fp32 bits as an ascending unsigned key.
__device__ __forceinline__ uint32_t desc_power_key(uint32_t b)
{
    const uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ~asc;
}

// Sort keys of the second pass and the per-plane counts (counted per block
// in LDS, then one global atomic per block and plane: a global atomic per
// entry would serialise on the few counters).
__global__ __launch_bounds__(kSelThreads) void k_sel_keys(const uint64_t* __restrict__ rec, int64_t n, int s_bin,
                                                          uint32_t kmask, uint64_t* __restrict__ key,
                                                          unsigned long long* __restrict__ cnt)
{
    __shared__ unsigned int hist[kMaxH];
    if (threadIdx.x < kMaxH) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSelThreads) {
        const uint64_t w = rec[i];
        const uint32_t k1 = ((uint32_t)w >> s_bin) & kmask;       // plane - 1 (kmask < kMaxH)
        key[i] = ((uint64_t)k1 << 32) | desc_power_key((uint32_t)(w >> 32));
        atomicAdd(&hist[k1], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kMaxH && hist[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
}

__global__ __launch_bounds__(kSelThreads) void k_sel_copy(const uint64_t* __restrict__ sorted,
                                                          const unsigned long long* __restrict__ cnt, int H,
                                                          int n_cand, uint64_t* __restrict__ out,
                                                          int64_t* __restrict__ out_counts)
{
    const int64_t total = (int64_t)H * n_cand;
    for (int64_t e = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kSelThreads) {
        const int k = (int)(e / n_cand);
        const int64_t i = e - (int64_t)k * n_cand;
        int64_t off = 0;
        for (int q = 0; q < k; ++q) off += (int64_t)cnt[q];
        const int64_t c = (int64_t)cnt[k];
        if (i < c) out[e] = sorted[off + i];
        if (i == 0) out_counts[k] = c < n_cand ? c : n_cand;
    }
}

int sel_grid(int64_t n)
{
    const int64_t b = (n + kSelThreads - 1) / kSelThreads;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

struct SelLayout {
    size_t rec_b, key_a, key_b, cnt, temp, total, temp_bytes;
};

hipError_t sel_layout(int64_t n, int end_bit, SelLayout& L)
{
    size_t t1 = 0, t2 = 0;
    rocprim::double_buffer<uint64_t> kb(nullptr, nullptr), vb(nullptr, nullptr);
    hipError_t e = rocprim::radix_sort_keys(nullptr, t1, kb, (size_t)n, 0, 32);
    if (e != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(nullptr, t2, kb, vb, (size_t)n, 0, end_bit);
    if (e != hipSuccess) return e;
    const size_t nb = align_up((size_t)n * 8);
    L.rec_b = nb;                 // record copy A at 0, B here
    L.key_a = 2 * nb;
    L.key_b = 3 * nb;
    L.cnt = 4 * nb;
    L.temp = L.cnt + align_up(kMaxH * 8);
    L.temp_bytes = t1 > t2 ? t1 : t2;
    L.total = L.temp + L.temp_bytes;
    return hipSuccess;
}

// ---- bounded selection -----------------------------------------------------

constexpr int kST = 1024;               // threads per block of the selection passes
constexpr int kMaxSelBlocks = 64;       // blocks of the passes over the whole list
constexpr int kSelLdsBnd = 2048;        // boundary entries sorted in LDS at once
constexpr int kSelU = 8;                // loads in flight per thread (the passes are latency-bound)
constexpr int kHistWords = 8192;        // per-block LDS histogram: H planes x bins(H)

__host__ __device__ constexpr int sel_bins(int H) { return H <= 8 ? 1024 : 512; }

__device__ __forceinline__ uint32_t total_order_key(uint32_t b)
{
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

struct KeyCfg {
    int policy, s_bin, s_row;
};

// The policy's unique 64-bit key of a candidate (larger = kept first).
__device__ __forceinline__ uint64_t sel_key(uint64_t e, const KeyCfg& c)
{
    const uint32_t w = (uint32_t)e;
    if (c.policy == HS_SELECT_TOP) return ((uint64_t)total_order_key((uint32_t)(e >> 32)) << 32) | (uint32_t)~w;
    // last N_cand: (bin, row) for Algorithm 2, (row, bin) for Algorithm 1,
    // packed without the plane field and left-aligned, so that the leading
    // bits (the ones the range bins split first) are the leading loop index;
    // bit 0 set so that no key is 0
    const int rbits = 32 - c.s_row;
    const int width = c.s_bin + rbits;              // <= 32
    if (width == 0) return 1u;
    const uint64_t j = w & ((1u << c.s_bin) - 1u);
    const uint64_t r = c.s_row < 32 ? (w >> c.s_row) : 0u;
    const uint64_t v = c.policy == HS_SELECT_LAST_ALG1 ? ((r << c.s_bin) | j) : ((j << rbits) | r);
    return (v << (64 - width)) | 1u;
}

// Bin width 2^shift covering [lo, hi] with `bins` bins.
__device__ __forceinline__ int range_shift(uint64_t lo, uint64_t hi, int bins)
{
    const uint64_t span = hi - lo;
    const int lb = bins == 1024 ? 10 : 9;
    return span < (uint64_t)bins ? 0 : (64 - lb) - __builtin_clzll(span);
}

// Per-plane summary shared by the passes.
struct alignas(128) PlaneInfo {   // one cache line each: the passes' atomics on different planes do not meet
    uint64_t lo, hi;          // key range of the plane
    uint32_t start, count;    // its run in the partitioned list
    int32_t shift, cut;       // bin width; the bin holding the n_cand-th largest key (-1: keep all)
    uint32_t above, inbin;    // entries in bins above the cut; in the cut bin
    uint32_t n_sel, n_bnd;    // collected so far (global counters)
};

// Blocks over a list of n entries: one round of kSelU loads per thread
// covers kSelU * kST entries, so up to 64 such chunks each pass takes a
// single round of loads.
int sel_blocks(int64_t n)
{
    const int64_t b = (n + (int64_t)kSelU * kST - 1) / ((int64_t)kSelU * kST);
    return (int)(b < 1 ? 1 : (b > kMaxSelBlocks ? kMaxSelBlocks : b));
}

__device__ __forceinline__ void chunk_of(int64_t n, int64_t& e0, int64_t& e1)
{
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    e0 = (int64_t)blockIdx.x * per;
    e1 = e0 + per < n ? e0 + per : n;
}

// Unrolled loop over [e0, e1) with kSelU loads in flight per thread; body(x)
// for each entry.
template <typename F>
__device__ __forceinline__ void for_entries(const uint64_t* __restrict__ a, int64_t e0, int64_t e1, F body)
{
    for (int64_t b = e0 + threadIdx.x; b < e1; b += (int64_t)kSelU * kST) {
        uint64_t x[kSelU];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) {
            const int64_t e = b + (int64_t)u * kST;
            x[u] = a[e < e1 ? e : e1 - 1];
        }
#pragma unroll
        for (int u = 0; u < kSelU; ++u)
            if (b + (int64_t)u * kST < e1) body(x[u]);
    }
}

// Pass 1: per block and plane, the number of candidates and the range of
// the keys' upper 32 bits (widened to whole keys: [min << 32, max << 32 |
// ones]).  Each thread accumulates in registers and the block reduces with
// wave shuffles: atomics on a handful of LDS words would serialise.
// HP: plane slots tracked per thread (4, 8 or 16, at least H).
template <int HP>
__global__ __launch_bounds__(kST) void k_sel_stats(const uint64_t* __restrict__ cand, int64_t n, KeyCfg cfg,
                                                   uint32_t kmask, int H, uint32_t* __restrict__ cnt,
                                                   uint64_t* __restrict__ kmin, uint64_t* __restrict__ kmax)
{
    __shared__ uint32_t red[3][kST / 64][HP];
    uint32_t c[HP], lo[HP], hi[HP];
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        c[q] = 0;
        lo[q] = ~0u;
        hi[q] = 0;
    }
    int64_t e0, e1;
    chunk_of(n, e0, e1);
    for_entries(cand, e0, e1, [&](uint64_t x) {
        const uint32_t k = ((uint32_t)x >> cfg.s_bin) & kmask;
        const uint32_t kh = (uint32_t)(sel_key(x, cfg) >> 32);
#pragma unroll
        for (int q = 0; q < HP; ++q) {
            if (k == (uint32_t)q) {
                ++c[q];
                lo[q] = kh < lo[q] ? kh : lo[q];
                hi[q] = kh > hi[q] ? kh : hi[q];
            }
        }
    });
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        if (q >= H) break;
        for (int d = 32; d >= 1; d >>= 1) {
            c[q] += (uint32_t)__shfl_xor((int)c[q], d, 64);
            const uint32_t a = (uint32_t)__shfl_xor((int)lo[q], d, 64);
            const uint32_t b = (uint32_t)__shfl_xor((int)hi[q], d, 64);
            lo[q] = a < lo[q] ? a : lo[q];
            hi[q] = b > hi[q] ? b : hi[q];
        }
        if (lane == 0) {
            red[0][w][q] = c[q];
            red[1][w][q] = lo[q];
            red[2][w][q] = hi[q];
        }
    }
    __syncthreads();
    if (threadIdx.x < H) {
        const int q = threadIdx.x;
        uint32_t sc = 0, sl = ~0u, sh = 0;
        for (int v = 0; v < kST / 64; ++v) {
            sc += red[0][v][q];
            sl = red[1][v][q] < sl ? red[1][v][q] : sl;
            sh = red[2][v][q] > sh ? red[2][v][q] : sh;
        }
        const int64_t o = (int64_t)blockIdx.x * H + q;
        cnt[o] = sc;
        kmin[o] = (uint64_t)sl << 32;
        kmax[o] = ((uint64_t)sh << 32) | 0xFFFFFFFFull;
    }
}

// The planes' ranges and runs from the blocks' statistics into `pi` (LDS):
// every (block, plane) record is loaded by its own thread (one round of
// loads), then thread q < H works out plane q from LDS.  Called by the
// whole block (contains barriers).
__device__ void plane_infos(const uint32_t* __restrict__ cnt, const uint64_t* __restrict__ kmin,
                            const uint64_t* __restrict__ kmax, int G, int H, PlaneInfo* pi)
{
    __shared__ uint32_t sc[kMaxSelBlocks * kMaxH];
    __shared__ uint64_t sl[kMaxSelBlocks * kMaxH], sh[kMaxSelBlocks * kMaxH];
    __shared__ uint32_t tot[kMaxH];
    const int t = threadIdx.x;
    if (t < G * H) {
        sc[t] = cnt[t];
        sl[t] = kmin[t];
        sh[t] = kmax[t];
    }
    __syncthreads();
    const int q = t;
    uint32_t total = 0;
    uint64_t lo = ~0ull, hi = 0;
    if (q < H) {
        for (int b = 0; b < G; ++b) {
            const int o = b * H + q;
            total += sc[o];
            if (sc[o]) {
                lo = sl[o] < lo ? sl[o] : lo;
                hi = sh[o] > hi ? sh[o] : hi;
            }
        }
        tot[q] = total;
    }
    __syncthreads();
    if (q < H) {
        uint32_t before = 0;
        for (int p = 0; p < q; ++p) before += tot[p];
        PlaneInfo x{};
        x.lo = lo;
        x.hi = hi;
        x.start = before;
        x.count = total;
        x.shift = total ? range_shift(lo, hi, sel_bins(H)) : 0;
        pi[q] = x;
    }
}

// Pass 2: per block, the histogram of its entries over each plane's bins
// (bins of equal width spanning the plane's key range); block 0 records the
// planes' ranges and runs.
__global__ __launch_bounds__(kST) void k_sel_hist(const uint64_t* __restrict__ cand, int64_t n, KeyCfg cfg,
                                                  uint32_t kmask, int H, const uint32_t* __restrict__ cnt,
                                                  const uint64_t* __restrict__ kmin,
                                                  const uint64_t* __restrict__ kmax, uint32_t* __restrict__ ph,
                                                  PlaneInfo* __restrict__ info)
{
    __shared__ uint32_t hist[kHistWords];
    __shared__ PlaneInfo pi[kMaxH];
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    const int bins = sel_bins(H);
    for (int i = t; i < H * bins; i += kST) hist[i] = 0;
    plane_infos(cnt, kmin, kmax, G, H, pi);
    __syncthreads();
    if (b == 0 && t < H) info[t] = pi[t];
    int64_t e0, e1;
    chunk_of(n, e0, e1);
    for_entries(cand, e0, e1, [&](uint64_t x) {
        const uint32_t k = ((uint32_t)x >> cfg.s_bin) & kmask;
        const uint64_t d = (sel_key(x, cfg) - pi[k].lo) >> pi[k].shift;   // < bins by the range
        atomicAdd(&hist[k * bins + (int)(d < (uint64_t)bins ? d : (uint64_t)(bins - 1))], 1u);
    });
    __syncthreads();
    for (int i = t; i < H * bins; i += kST) ph[(int64_t)b * H * bins + i] = hist[i];
}

// Pass 3: one block per plane: the plane's histogram (the blocks' partial
// histograms summed), a suffix scan, and the bin holding the n_cand-th
// largest key.
__global__ __launch_bounds__(kST) void k_sel_cut(const uint32_t* __restrict__ ph, int G, int H, int n_cand,
                                                 PlaneInfo* __restrict__ info)
{
    __shared__ uint32_t h[1024];
    const int k = blockIdx.x, t = threadIdx.x;
    const int bins = sel_bins(H);
    __shared__ uint32_t wsum[kST / 64];
    // the blocks' counts of bin t, sixteen loads in flight at a time
    uint32_t own = 0;
    if (t < bins) {
        constexpr int U = 16;
        for (int b0 = 0; b0 < G; b0 += U) {
            uint32_t x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = b0 + u < G ? ph[((int64_t)(b0 + u) * H + k) * bins + t] : 0u;
#pragma unroll
            for (int u = 0; u < U; ++u) own += x[u];
        }
    }
    // suffix sums over the bins: within each wave by shuffles, then across
    // the waves
    const int lane = t & 63, w = t >> 6;
    uint32_t suf = own;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_down((int)suf, d, 64);
        if (lane + d < 64) suf += y;
    }
    if (lane == 0) wsum[w] = suf;
    __syncthreads();
    for (int v = w + 1; v < kST / 64; ++v) suf += wsum[v];
    h[t] = suf;
    __syncthreads();
    const uint32_t m = info[k].count;
    if (t == 0) {
        info[k].n_sel = 0;
        info[k].n_bnd = 0;
    }
    if (m <= (uint32_t)n_cand) {
        if (t == 0) {
            info[k].cut = -1;                     // every entry is kept
            info[k].above = m;
            info[k].inbin = 0;
        }
        return;
    }
    const uint32_t next = t < 1023 ? h[t + 1] : 0u;   // suf: entries in bins t..end
    if (suf >= (uint32_t)n_cand && next < (uint32_t)n_cand) {
        info[k].cut = t;
        info[k].above = next;
        info[k].inbin = own;
    }
}

// Pass 4: blocks over the whole list: entries above their plane's cut go to
// the plane's kept list, entries in the cut bin to its boundary list (at
// the plane's run offset); per block and list one atomic reserves the
// positions.
__global__ __launch_bounds__(kST) void k_sel_collect(const uint64_t* __restrict__ cand, int64_t n, KeyCfg cfg,
                                                     uint32_t kmask, int H, int n_cand,
                                                     PlaneInfo* __restrict__ info, uint64_t* __restrict__ sel,
                                                     uint64_t* __restrict__ bnd)
{
    __shared__ PlaneInfo pi[kMaxH];
    __shared__ unsigned int na[kMaxH], nb[kMaxH], ia[kMaxH], ib[kMaxH];
    __shared__ uint32_t base_a[kMaxH], base_b[kMaxH];
    const int t = threadIdx.x;
    if (t < H) {
        pi[t] = info[t];
        na[t] = nb[t] = ia[t] = ib[t] = 0;
    }
    __syncthreads();
    int64_t e0, e1;
    chunk_of(n, e0, e1);
    auto bin_of = [&](uint64_t x, uint32_t k) { return (int64_t)((sel_key(x, cfg) - pi[k].lo) >> pi[k].shift); };
    auto count = [&](uint64_t x) {
        const uint32_t k = ((uint32_t)x >> cfg.s_bin) & kmask;
        const int64_t d = bin_of(x, k);
        if (d > pi[k].cut) atomicAdd(&na[k], 1u);
        else if (d == pi[k].cut) atomicAdd(&nb[k], 1u);
    };
    auto place = [&](uint64_t x) {
        const uint32_t k = ((uint32_t)x >> cfg.s_bin) & kmask;
        const int64_t d = bin_of(x, k);
        if (d > pi[k].cut) {
            const uint32_t p = base_a[k] + atomicAdd(&ia[k], 1u);
            if (p < (uint32_t)n_cand) sel[(int64_t)k * n_cand + p] = x;
        } else if (d == pi[k].cut) {
            const uint32_t p = base_b[k] + atomicAdd(&ib[k], 1u);
            if (p < pi[k].count) bnd[pi[k].start + p] = x;
        }
    };
    auto reserve = [&]() {
        __syncthreads();
        if (t < H) {
            base_a[t] = na[t] ? atomicAdd(&info[t].n_sel, na[t]) : 0u;
            base_b[t] = nb[t] ? atomicAdd(&info[t].n_bnd, nb[t]) : 0u;
        }
        __syncthreads();
    };
    if (e1 - e0 <= (int64_t)kSelU * kST) {
        // one round of loads: the entries stay in registers for both passes
        uint64_t x[kSelU];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) {
            const int64_t e = e0 + t + (int64_t)u * kST;
            x[u] = e < e1 ? cand[e] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kSelU; ++u)
            if (e0 + t + (int64_t)u * kST < e1) count(x[u]);
        reserve();
#pragma unroll
        for (int u = 0; u < kSelU; ++u)
            if (e0 + t + (int64_t)u * kST < e1) place(x[u]);
    } else {
        for_entries(cand, e0, e1, count);
        reserve();
        for_entries(cand, e0, e1, place);
    }
}

// Rank of each of n distinct keys in LDS (descending: the number of larger
// keys; ascending: of smaller ones), by comparison with every other key
// (the reads are LDS broadcasts); n is at most a few thousand.
__device__ __forceinline__ int key_rank(const uint64_t* k, int n, int i, bool desc)
{
    const uint64_t me = k[i];
    int r = 0;
    for (int j = 0; j < n; ++j) r += desc ? (k[j] > me) : (k[j] < me);
    return r;
}

// Pass 5: one block per plane: the kept entries and the largest keys of the
// boundary bin (a bin too large for LDS is first split again over its own
// range), ranked in the policy's order and written out.
static_assert(kST == 1024, "one histogram bin per thread");
__global__ __launch_bounds__(kST) void k_sel_final(const uint64_t* __restrict__ sel, const uint64_t* __restrict__ bnd,
                                                   const PlaneInfo* __restrict__ info, KeyCfg cfg, int n_cand,
                                                   uint64_t* __restrict__ out, int64_t* __restrict__ out_counts)
{
    __shared__ uint32_t hist[1024];
    __shared__ uint64_t in_k[kSelLdsCand], in_v[kSelLdsCand];
    __shared__ uint64_t bd_k[kSelLdsBnd], bd_v[kSelLdsBnd];
    __shared__ int n_in_s, n_bd_s, cut_s, above_s, inbin_s;
    const int k = blockIdx.x, t = threadIdx.x;
    const PlaneInfo pi = info[k];
    const int keep = (int)(pi.count < (uint32_t)n_cand ? pi.count : (uint32_t)n_cand);
    const int n_above = (int)(pi.above < (uint32_t)n_cand ? pi.above : (uint32_t)n_cand);
    for (int i = t; i < n_above; i += kST) {
        in_v[i] = sel[(int64_t)k * n_cand + i];
        in_k[i] = sel_key(in_v[i], cfg);
    }
    if (t == 0) n_in_s = n_above;
    __syncthreads();
    int need = keep - n_above;
    const uint64_t* run = bnd + pi.start;
    const int64_t m = pi.cut >= 0 ? (int64_t)pi.inbin : 0;
    // the boundary entries lie in [lo, hi]; split further while they do not
    // fit in LDS (keys are distinct, so each round narrows the range)
    uint64_t lo = pi.lo + ((uint64_t)(pi.cut < 0 ? 0 : pi.cut) << pi.shift);
    uint64_t hi = lo + ((((uint64_t)1) << pi.shift) - 1);
    hi = hi < pi.hi ? hi : pi.hi;
    int64_t in_range = m;
    while (need > 0 && in_range > kSelLdsBnd) {
        if (hi - lo < 1024) break;   // one key per bin already (only repeated entries get here)
        const int shift = range_shift(lo, hi, 1024);
        hist[t] = 0;
        __syncthreads();
        for_entries(run, 0, m, [&](uint64_t x) {
            const uint64_t key = sel_key(x, cfg);
            if (key >= lo && key <= hi) {
                const uint64_t d = (key - lo) >> shift;
                atomicAdd(&hist[d < 1024 ? d : 1023], 1u);
            }
        });
        __syncthreads();
        const uint32_t own = hist[t];
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const uint32_t add = t + d < 1024 ? hist[t + d] : 0u;
            __syncthreads();
            hist[t] += add;
            __syncthreads();
        }
        const uint32_t suf = hist[t], next = t < 1023 ? hist[t + 1] : 0u;
        if ((int)suf >= need && (int)next < need) {
            cut_s = t;
            above_s = (int)next;
            inbin_s = (int)own;
        }
        __syncthreads();
        const int cut = cut_s;
        for_entries(run, 0, m, [&](uint64_t x) {
            const uint64_t key = sel_key(x, cfg);
            if (key < lo || key > hi) return;
            if ((int64_t)((key - lo) >> shift) > cut) {
                const int p = atomicAdd(&n_in_s, 1);
                if (p < kSelLdsCand) {
                    in_k[p] = key;
                    in_v[p] = x;
                }
            }
        });
        __syncthreads();
        need -= above_s;
        in_range = inbin_s;
        const uint64_t nlo = lo + ((uint64_t)cut << shift);
        const uint64_t nhi = nlo + ((((uint64_t)1) << shift) - 1);
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
        __syncthreads();
    }
    if (need > 0) {
        if (t == 0) n_bd_s = 0;
        __syncthreads();
        for_entries(run, 0, m, [&](uint64_t x) {
            const uint64_t key = sel_key(x, cfg);
            if (key < lo || key > hi) return;
            const int p = atomicAdd(&n_bd_s, 1);
            if (p < kSelLdsBnd) {
                bd_k[p] = key;
                bd_v[p] = x;
            }
        });
        __syncthreads();
        // the `need` largest boundary keys complete the list
        const int nb = n_bd_s < kSelLdsBnd ? n_bd_s : kSelLdsBnd;
        const int base = n_in_s;
        for (int i = t; i < nb; i += kST) {
            const int r = key_rank(bd_k, nb, i, true);
            if (r < need && base + r < kSelLdsCand) {
                in_k[base + r] = bd_k[i];
                in_v[base + r] = bd_v[i];
            }
        }
        __syncthreads();
    }
    // the kept entries in the policy's order
    for (int i = t; i < keep; i += kST) {
        const int r = key_rank(in_k, keep, i, cfg.policy == HS_SELECT_TOP);
        out[(int64_t)k * n_cand + r] = in_v[i];
    }
    if (t == 0) out_counts[k] = keep;
}

struct BoundedLayout {
    size_t bnd, sel, cnt, kmin, kmax, ph, info, total;
};

BoundedLayout bounded_layout(int64_t n, int H, int n_cand)
{
    BoundedLayout L;
    const size_t nn = align_up((size_t)(n > 0 ? n : 1) * 8);
    L.bnd = 0;
    L.sel = nn;
    L.cnt = L.sel + align_up((size_t)H * n_cand * 8);
    L.kmin = L.cnt + align_up((size_t)kMaxSelBlocks * kMaxH * 4);
    L.kmax = L.kmin + align_up((size_t)kMaxSelBlocks * kMaxH * 8);
    L.ph = L.kmax + align_up((size_t)kMaxSelBlocks * kMaxH * 8);
    L.info = L.ph + align_up((size_t)kMaxSelBlocks * kHistWords * 4);
    L.total = L.info + align_up((size_t)kMaxH * sizeof(PlaneInfo));
    return L;
}

}  // namespace

hipError_t select_bounded(const uint64_t* cand, int64_t n, int H, int s_bin, int s_k, int policy, int n_cand,
                          uint64_t* out, int64_t* out_counts, void* work, hipStream_t s)
{
    if (n_cand < 1 || n_cand > kSelLdsCand || n < 0 || n > (int64_t)UINT32_MAX || H < 1 || H > kMaxH)
        return hipErrorInvalidValue;
    const BoundedLayout L = bounded_layout(n, H, n_cand);
    char* w = static_cast<char*>(work);
    uint64_t* bnd = reinterpret_cast<uint64_t*>(w + L.bnd);
    uint64_t* sel = reinterpret_cast<uint64_t*>(w + L.sel);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(w + L.cnt);
    uint64_t* kmin = reinterpret_cast<uint64_t*>(w + L.kmin);
    uint64_t* kmax = reinterpret_cast<uint64_t*>(w + L.kmax);
    uint32_t* ph = reinterpret_cast<uint32_t*>(w + L.ph);
    PlaneInfo* info = reinterpret_cast<PlaneInfo*>(w + L.info);
    const uint32_t kmask = (1u << s_k) - 1u;
    const KeyCfg cfg{policy, s_bin, s_bin + s_k};
    const int G = sel_blocks(n);
    if (H <= 4)
        hipLaunchKernelGGL(k_sel_stats<4>, dim3(G), dim3(kST), 0, s, cand, n, cfg, kmask, H, cnt, kmin, kmax);
    else if (H <= 8)
        hipLaunchKernelGGL(k_sel_stats<8>, dim3(G), dim3(kST), 0, s, cand, n, cfg, kmask, H, cnt, kmin, kmax);
    else
        hipLaunchKernelGGL(k_sel_stats<kMaxH>, dim3(G), dim3(kST), 0, s, cand, n, cfg, kmask, H, cnt, kmin, kmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_hist, dim3(G), dim3(kST), 0, s, cand, n, cfg, kmask, H, cnt, kmin, kmax, ph, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_cut, dim3(H), dim3(kST), 0, s, ph, G, H, n_cand, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_collect, dim3(G), dim3(kST), 0, s, cand, n, cfg, kmask, H, n_cand, info, sel, bnd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_final, dim3(H), dim3(kST), 0, s, sel, bnd, info, cfg, n_cand, out, out_counts);
    return hipGetLastError();
}

size_t select_bounded_workspace(int64_t n, int H, int n_cand) { return bounded_layout(n, H, n_cand).total; }

hipError_t select_workspace(int64_t n, int end_bit, size_t* bytes)
{
    SelLayout L;
    const hipError_t e = sel_layout(n, end_bit, L);
    *bytes = L.total;
    return e;
}

hipError_t select_top(const uint64_t* cand, int64_t n, int H, int s_bin, int s_k, int n_cand, uint64_t* out,
                      int64_t* out_counts, void* work, hipStream_t s)
{
    const int end_bit = 32 + s_k;
    SelLayout L;
    hipError_t e = sel_layout(n, end_bit, L);
    if (e != hipSuccess) return e;
    char* w = static_cast<char*>(work);
    uint64_t* rec_a = reinterpret_cast<uint64_t*>(w);
    uint64_t* rec_b = reinterpret_cast<uint64_t*>(w + L.rec_b);
    uint64_t* key_a = reinterpret_cast<uint64_t*>(w + L.key_a);
    uint64_t* key_b = reinterpret_cast<uint64_t*>(w + L.key_b);
    int64_t* cnt = reinterpret_cast<int64_t*>(w + L.cnt);
    void* temp = w + L.temp;
    size_t temp_bytes = L.temp_bytes;

    e = launch_zero_i64(cnt, kMaxH, s);
    if (e != hipSuccess) return e;
    const uint64_t* sorted = rec_a;
    if (n > 0) {
        e = hipMemcpyAsync(rec_a, cand, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        rocprim::double_buffer<uint64_t> rb(rec_a, rec_b);
        e = rocprim::radix_sort_keys(temp, temp_bytes, rb, (size_t)n, 0, 32, s);   // by CL1 word
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sel_keys, dim3(sel_grid(n)), dim3(kSelThreads), 0, s, rb.current(), n, s_bin,
                           (uint32_t)((1u << s_k) - 1u), key_a,
                           reinterpret_cast<unsigned long long*>(cnt));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        rocprim::double_buffer<uint64_t> kb(key_a, key_b);
        rocprim::double_buffer<uint64_t> vb(rb.current(), rb.current() == rec_a ? rec_b : rec_a);
        temp_bytes = L.temp_bytes;
        e = rocprim::radix_sort_pairs(temp, temp_bytes, kb, vb, (size_t)n, 0, end_bit, s);   // stable
        if (e != hipSuccess) return e;
        sorted = vb.current();
    }
    hipLaunchKernelGGL(k_sel_copy, dim3(sel_grid((int64_t)H * n_cand)), dim3(kSelThreads), 0, s, sorted,
                       reinterpret_cast<const unsigned long long*>(cnt), H, n_cand, out, out_counts);
    return hipGetLastError();
}

}  // namespace hsk
