// Strip-walk detection kernel for gfx950: harmonic planes (Eq. 1-2 of
// arXiv:1805.12258, Sec. III) thresholded into packed candidates, with no
// plane written to memory.
//
// Work decomposition.  A unit is a strip of B = 64 V consecutive bins of
// one row band of the plane (V = 2, 4 or 8 bins per lane, a template
// parameter chosen per plan): the rows with negative template index, or the
// rows with non-negative index.  Under the floor of Eq. 1 the two bands read
// disjoint source rows (floor(i/m) keeps the sign of i), so each band only
// stages source rows of its own half (the independent half FOPs of Sec. VI-A).
// One wave owns one unit at a time and walks its rows in increasing order;
// each lane owns V consecutive bins.  Waves are independent: there is no
// block barrier inside the walk.
//
// Loads.  Every global read is an LDS-DMA (global_load_lds_dwordx4) into
// rings private to the wave: the m = 1 row of each walked row (a ring of
// kWDmax rows), and for each stretch factor m >= 2 the shrunken source range
// [floor(j0/m), floor((j0+B-1)/m)] of source row floor(i/m), loaded only
// when floor(i/m) changes, i.e. every m rows.  The loads of row p + D are issued while row p is summed; the wave
// then waits with an exact vmcnt for the loads of the next row (vector memory
// loads complete in issue order), so D rows stay in flight.  Source values
// are read from the ring and selected per bin only when a source row
// changes, and kept in registers for the m rows that use them.
//
// Order.  A host-built schedule lists the units of each XCD (blocks are
// dealt to the XCDs in turn): the bin strips are dealt to eight lists by the
// three bits after the leading one of the strip index, and each list is
// ordered by position inside the octave, so that strips x, x/2, x/4 and x/8
// are summed on one XCD at nearly the same time and the staged ranges of
// m = 2, 4, 8 are L2 hits.  A batch assigns whole FOPs to XCDs instead.
//
// Candidates.  A wave appends its hits to a private LDS buffer (ballot +
// mbcnt); a full buffer is written out with one global atomic per wave that
// reserves its positions in the list, and the last buffers of a block with
// one atomic for the block.  Per-plane counts are formed by a counting pass
// over the list afterwards (only candidates dropped for lack of capacity
// are counted here).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "hs_internal.h"

namespace hsk {
namespace walk {

constexpr int kWDmax = 2;               // rows whose loads are in flight (a power of two)
constexpr int kWWaves = 4;              // waves per block
constexpr int kWThreads = 64 * kWWaves;
constexpr int kWThrBytes = 16384;       // largest threshold table (LDS, per block)

struct bf16 {
    uint16_t bits;
};

template <typename TIn> struct St;
template <> struct St<float> {
    static constexpr int EB = 4;
};
template <> struct St<_Float16> {
    static constexpr int EB = 2;
};
template <> struct St<bf16> {
    static constexpr int EB = 2;
};

// Bins of a strip for V bins per lane.
__host__ __device__ constexpr int strip_bins(int V) { return 64 * V; }
// Per-wave candidate buffer (entries).  One emission call adds at most 64
// hits per bin of the lane group; the buffer is written out before a bin's
// hits when they might not fit, so it need not hold the 64 V hits of a
// whole call.  (128 entries, which would leave more LDS for waves, made fp32
// at H = 8, V = 4 slower: 253 -> 292 us per call on 85 x 2^21.)
__host__ __device__ constexpr int cand_cap(int) { return 320; }

// Elements of one source slot of stretch factor m: the range
// [floor(j0/m), floor((j0+B-1)/m)] (at most floor((B-1)/m) + 2 elements)
// from a start rounded down to a 16-byte piece (3 more fp32 words or 7 more
// halves).
__host__ __device__ constexpr int slot_elems(int m, int EB, int V)
{
    return EB == 4 ? (((strip_bins(V) - 1) / m + 5 + 3) & ~3) : (((strip_bins(V) - 1) / m + 9 + 7) & ~7);
}
// LDS of one wave: a ring of kWDmax rows of m = 1 values (row p in slot
// p mod kWDmax), then a byte ring of source slots: each source row that a
// row needs is given slot_bytes(m) consecutive bytes at the ring's head
// (wrapping to the start when it does not fit before the end), in row order
// and m order within a row; the consuming side walks the same sequence, so
// both sides compute the same slot addresses.  The ring holds the sources of
// the kWDmax rows in flight: per m at most ceil(D/m) + 1 of them (one more
// when a unit starts inside the window), plus the bytes lost to one wrap.
// Then the candidate buffer.  Loads are 16-byte pieces, one per lane and
// DMA instruction: a region of more than 64 pieces takes several.
static_assert((kWDmax & (kWDmax - 1)) == 0, "row slots are indexed by the low bits of the row count");
__host__ __device__ constexpr int x1_bytes(int EB, int V) { return strip_bins(V) * EB; }
__host__ __device__ constexpr int x1_pieces(int EB, int V) { return x1_bytes(EB, V) / 16; }
__host__ __device__ constexpr int slot_bytes(int m, int EB, int V) { return slot_elems(m, EB, V) * EB; }
__host__ __device__ constexpr int slot_pieces(int m, int EB, int V) { return slot_bytes(m, EB, V) / 16; }
__host__ __device__ constexpr int dmas(int pieces) { return (pieces + 63) / 64; }
__host__ __device__ constexpr int src_ring_bytes(int H, int EB, int V)
{
    int b = 0, mx = 0;
    for (int m = 2; m <= H; ++m) {
        b += ((kWDmax + m - 1) / m + 1) * slot_bytes(m, EB, V);
        mx = slot_bytes(m, EB, V) > mx ? slot_bytes(m, EB, V) : mx;
    }
    return b + mx;
}
__host__ __device__ constexpr int src_ring_offset(int EB, int V) { return kWDmax * x1_bytes(EB, V); }
__host__ __device__ constexpr int cand_offset(int H, int EB, int V)
{
    return (src_ring_offset(EB, V) + src_ring_bytes(H, EB, V) + 15) & ~15;
}
__host__ __device__ constexpr int wave_bytes(int H, int EB, int V) { return cand_offset(H, EB, V) + cand_cap(V) * 8; }
// after the waves: the block's flush bookkeeping (2 kWWaves + 2 words), then the thresholds
constexpr int kWBookBytes = ((2 * kWWaves + 2) * 4 + 15) & ~15;
__host__ __device__ constexpr int thr_stride(int H) { return (H + 3) & ~3; }

// Source values a lane keeps per stretch factor m: the lane's V bins start
// at a multiple of V, so when V divides m they share one source element,
// and when m divides V each group of m bins shares one (V/m elements);
// otherwise one value per bin.
__host__ __device__ constexpr int src_vals(int m, int V) { return m % V == 0 ? 1 : (V % m == 0 ? V / m : V); }

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef const __attribute__((address_space(4))) uint32_t* cu32_t;
typedef const __attribute__((address_space(4))) int64_t* ci64_t;

// The value of lane 0 (states a wave-uniform value as such, so that it
// lives in scalar registers and addresses formed from it are scalar).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Wave-uniform loads through the scalar data cache (constant address space).
__device__ __forceinline__ uint32_t sload_u32(const void* p, int64_t i)
{
    return reinterpret_cast<cu32_t>(reinterpret_cast<uintptr_t>(p))[uni64(i)];
}
__device__ __forceinline__ int64_t sload_i64(const void* p, int64_t i)
{
    return reinterpret_cast<ci64_t>(reinterpret_cast<uintptr_t>(p))[uni64(i)];
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B <= E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// f(integral_constant<int, m>) for every m in 2..H whose bit is set in fl,
// in increasing m.  The bits are tested four factors at a time first: most
// rows change few factors, and a group with no change costs one test.
template <int H, typename F>
__device__ __forceinline__ void for_changed(uint32_t fl, F&& f)
{
    static_for<0, (H - 2) / 4>([&](auto gc) {
        constexpr int lo = 2 + 4 * decltype(gc)::value;
        constexpr int hi = lo + 3 < H ? lo + 3 : H;
        constexpr uint32_t gmask = ((2u << hi) - 1u) & ~((1u << lo) - 1u);
        if (fl & gmask) {
            static_for<lo, hi>([&](auto mc) {
                if (fl & (1u << decltype(mc)::value)) f(mc);
            });
        }
    });
}

// Wait until at most n vector-memory operations of this wave are in flight
// (n clamped to 63, the counter's limit, which is a stricter wait).  The
// count of s_waitcnt is an immediate, so this jumps into a table of 64
// waits; the memory clobber keeps every later LDS access below it.
__device__ __forceinline__ void wait_vm(uint32_t n)
{
#define HS_VMW(k) "s_waitcnt vmcnt(" #k ")\n\ts_branch .Lhs_vmw_end%=\n\t"
    asm volatile(
        "s_min_u32 s98, %0, 63\n\t"
        "s_getpc_b64 s[96:97]\n\t"          // address of the next instruction
        "s_lshl_b32 s98, s98, 3\n\t"        // 8 bytes per table entry
        "s_add_u32 s98, s98, 20\n\t"        // the table starts 5 instructions on
        "s_add_u32 s96, s96, s98\n\t"
        "s_addc_u32 s97, s97, 0\n\t"
        "s_setpc_b64 s[96:97]\n\t"
        HS_VMW(0) HS_VMW(1) HS_VMW(2) HS_VMW(3) HS_VMW(4) HS_VMW(5) HS_VMW(6) HS_VMW(7)
        HS_VMW(8) HS_VMW(9) HS_VMW(10) HS_VMW(11) HS_VMW(12) HS_VMW(13) HS_VMW(14) HS_VMW(15)
        HS_VMW(16) HS_VMW(17) HS_VMW(18) HS_VMW(19) HS_VMW(20) HS_VMW(21) HS_VMW(22) HS_VMW(23)
        HS_VMW(24) HS_VMW(25) HS_VMW(26) HS_VMW(27) HS_VMW(28) HS_VMW(29) HS_VMW(30) HS_VMW(31)
        HS_VMW(32) HS_VMW(33) HS_VMW(34) HS_VMW(35) HS_VMW(36) HS_VMW(37) HS_VMW(38) HS_VMW(39)
        HS_VMW(40) HS_VMW(41) HS_VMW(42) HS_VMW(43) HS_VMW(44) HS_VMW(45) HS_VMW(46) HS_VMW(47)
        HS_VMW(48) HS_VMW(49) HS_VMW(50) HS_VMW(51) HS_VMW(52) HS_VMW(53) HS_VMW(54) HS_VMW(55)
        HS_VMW(56) HS_VMW(57) HS_VMW(58) HS_VMW(59) HS_VMW(60) HS_VMW(61) HS_VMW(62) HS_VMW(63)
        ".Lhs_vmw_end%=:"
        :
        : "s"(n)
        : "s96", "s97", "s98", "scc", "memory");
#undef HS_VMW
}

__device__ __forceinline__ void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lgkm_all() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int floordiv_i(int a, int b)
{
    const int q = a / b;
    return (q * b > a) ? q - 1 : q;
}

// Floor division of a (possibly negative) row offset by the constant m:
// shifted into the unsigned range first, so the division is a multiply-high.
template <int m>
__device__ __forceinline__ int floordiv_c(int a)
{
    constexpr uint32_t K = (uint32_t)m * (1u << 20);
    return (int)(((uint32_t)a + K) / (uint32_t)m) - (1 << 20);
}

// One unit as seen by a wave (wave-uniform values).
struct Unit {
    int j0;                     // first bin of the strip
    int r0, r1;                 // rows [r0, r1) of the band
    int f;                      // FOP index within the call
    int N;                      // bins of the FOP
};

// The issue side's view of a unit's FOP: a buffer resource over the whole
// plane (reads past its end return zero) and the row pitch in bytes.
struct Src {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t ldb;
};

// Position of a wave in its XCD's unit sequence: the concatenation of the
// segments [xseg[x], xseg[x+1]) of the schedule, each segment (FOP, first
// entry, first index, end index) a run of one FOP's unit list.
struct Iter {
    int i;          // next index in the XCD's sequence
    int s, s_end;   // current segment, end of the XCD's segments
};

template <typename TIn, int H, int V>
struct Walker {
    static constexpr int EB = St<TIn>::EB;
    static constexpr int EPP = 16 / EB;     // elements per 16-byte piece
    static constexpr int B = strip_bins(V);

    const WalkArgs& a;
    int lane;

    __device__ Walker(const WalkArgs& a_) : a(a_), lane(threadIdx.x & 63) {}

    // The next unit of the sequence (false at its end); `step` is the number
    // of waves on this XCD.  In a batch, the units of a FOP whose address or
    // pitch breaks the alignment rules are skipped (both sides skip the same
    // ones; the consume side marks the FOP with a total count of -1).
    template <bool CONSUME>
    __device__ __forceinline__ bool next_unit(Iter& it, int step, Unit& u, Src* src) const
    {
        for (;;) {
            int f, eoff, pbeg;
            for (;;) {
                if (it.s >= it.s_end) return false;
                f = (int)sload_u32(a.seg, (int64_t)it.s * 4 + 0);
                eoff = (int)sload_u32(a.seg, (int64_t)it.s * 4 + 1);
                pbeg = (int)sload_u32(a.seg, (int64_t)it.s * 4 + 2);
                const int pend = (int)sload_u32(a.seg, (int64_t)it.s * 4 + 3);
                if (it.i < pend) break;
                it.s = uni(it.s + 1);
            }
            const uint32_t e = sload_u32(a.ent, (int64_t)eoff + (it.i - pbeg));
            it.i = uni(it.i + step);
            const int band = (int)(e >> 24);
            u.j0 = uni((int)(e & 0xffffffu) * B);
            u.r0 = band == 0 ? 0 : a.band_split;
            u.r1 = (band == 0 && a.band_split > 0) ? a.band_split : a.T;
            u.f = f;
            const void* fop;
            int64_t ld;
            if (a.n_fops == 0) {
                u.N = a.N;
                fop = a.fop;
                ld = a.ld;
            } else {
                u.N = (int)sload_i64(a.n_chans, f);
                fop = reinterpret_cast<const void*>((uintptr_t)sload_i64(a.fops, f));
                ld = sload_i64(a.lds, f);
                const bool ok = (reinterpret_cast<uintptr_t>(fop) & 15) == 0 && ld % EPP == 0 && ld >= u.N &&
                                (uint64_t)ld * (uint64_t)a.T * EB <= 0xffffffffull;
                if (!ok) {
                    if (CONSUME && lane == 0) a.counts[(int64_t)f * (H + 1) + H] = ~0ull;
                    continue;
                }
            }
            if (src) {
                src->ldb = (uint32_t)(ld * EB);
                src->rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(fop), 0,
                                                              (int)((uint64_t)ld * (uint64_t)a.T * EB - 1) + 1,
                                                              0x00020000);
            }
            return true;
        }
    }

    // 16-byte LDS-DMA per lane from plane byte soff + voff (voff includes
    // 16 lane) into LDS at dst + 16 lane.
    __device__ __forceinline__ void dma(const Src& s, unsigned char* dst, uint32_t voff, uint32_t soff) const
    {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(s.rsrc, (lds_ptr_t)dst, 16, voff, soff, 0, 0);
    }

    // Stored element at byte address p of LDS as fp32 (storage units).
    __device__ __forceinline__ float elem(const unsigned char* p, int e) const
    {
        if constexpr (EB == 4) {
            return reinterpret_cast<const float*>(p)[e];
        } else {
            const uint16_t b = reinterpret_cast<const uint16_t*>(p)[e];
            if constexpr (std::is_same<TIn, bf16>::value) {
                return __uint_as_float((uint32_t)b << 16);
            } else {
                _Float16 h;
                __builtin_memcpy(&h, &b, 2);
                return (float)h;
            }
        }
    }

    // The lane's V m = 1 values of the row in the row slot at `slot`.
    __device__ __forceinline__ void x1_vals(const unsigned char* slot, float (&x)[V]) const
    {
        if constexpr (EB == 4) {
            const float* p = reinterpret_cast<const float*>(slot) + V * lane;
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = p[v];
        } else {
            const uint16_t* p = reinterpret_cast<const uint16_t*>(slot) + V * lane;
            uint16_t hb[V];
            __builtin_memcpy(hb, p, sizeof(hb));     // one LDS read of 2V bytes
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if constexpr (std::is_same<TIn, bf16>::value) {
                    x[v] = __uint_as_float((uint32_t)hb[v] << 16);
                } else {
                    _Float16 h;
                    __builtin_memcpy(&h, &hb[v], 2);
                    x[v] = (float)h;
                }
            }
        }
    }
};

}  // namespace walk

// Occupancy asked of the compiler: with 16-bit storage and four bins per
// lane a block's LDS leaves room for six waves per SIMD up to eight planes,
// which holds without scratch.  (Five waves at eight bins per lane would
// spill at seven and eight planes.)
template <typename TIn, int H, int V>
constexpr int walk_min_waves() { return (sizeof(TIn) == 2 && H <= 8 && V == 4) ? 6 : 1; }

// The strip-walk detection kernel (see the top of this file).
template <typename TIn, int H, int V>
__global__ __launch_bounds__(walk::kWThreads, (walk_min_waves<TIn, H, V>())) void k_walk(WalkArgs a)
{
    using namespace walk;
    using Wk = Walker<TIn, H, V>;
    constexpr int EB = Wk::EB;
    constexpr int EPP = Wk::EPP;
    constexpr int B = Wk::B;
    constexpr int HS = thr_stride(H);
    constexpr int D = kWDmax;
    constexpr int SRB = src_ring_bytes(H, EB, V);
    constexpr int WB = wave_bytes(H, EB, V);
    constexpr int CAP = cand_cap(V);
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // thresholds of every row in storage units (exact: the scale is a power
    // of two), and the waves' per-plane counters
    int* const book = reinterpret_cast<int*>(smem + kWWaves * WB);
    float* const thr = reinterpret_cast<float*>(smem + kWWaves * WB + kWBookBytes);
    for (int e = threadIdx.x; e < a.T * HS; e += kWThreads) {
        const int r = e / HS, k = e - r * HS;
        thr[e] = k < H ? a.ta[(int64_t)k * a.T + r] * a.scale : 0.0f;
    }
    unsigned char* const wl = smem + wave * WB;
    __syncthreads();

    const Wk w(a);
    uint64_t* const cbuf = reinterpret_cast<uint64_t*>(wl + cand_offset(H, EB, V));

    // this wave's place in its XCD's unit sequence (blocks are dealt to the
    // eight XCDs in turn); the issue side runs D rows ahead of the consume
    // side over the same sequence
    const int xcd = blockIdx.x & 7;
    const int step = (int)((gridDim.x - xcd + 7) >> 3) * kWWaves;
    Iter ii;
    ii.i = uni((int)(blockIdx.x >> 3) * kWWaves + wave);
    ii.s = (int)sload_u32(a.xseg, xcd);
    ii.s_end = (int)sload_u32(a.xseg, xcd + 1);
    Iter ci = ii;

    // ---- issue side ------------------------------------------------------------
    Unit iu;
    Src isrc;
    // single FOP: the block's waves reserve their last candidates' positions
    // with one atomic (they finish together, so their flushes would all meet)
    auto block_reserve = [&](int n) -> unsigned long long {
        __syncthreads();
        if (lane == 0) book[wave] = n;
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int v = 0; v < kWWaves; ++v) {
                book[kWWaves + v] = acc;
                acc += book[v];
            }
            const unsigned long long b = acc ? atomicAdd(&a.counts[H], (unsigned long long)acc) : 0ull;
            book[2 * kWWaves] = (int)(uint32_t)b;
            book[2 * kWWaves + 1] = (int)(uint32_t)(b >> 32);
        }
        __syncthreads();
        return (((unsigned long long)(uint32_t)book[2 * kWWaves + 1] << 32) | (uint32_t)book[2 * kWWaves]) +
               (unsigned long long)book[kWWaves + wave];
    };
    bool ivalid = w.template next_unit<false>(ii, step, iu, &isrc);
    if (!ivalid) {
        if (a.n_fops == 0) (void)block_reserve(0);
        return;
    }
    int ir = iu.r0;
    int iseq = 0;                         // stream index of the next row to issue
    int ihead = 0;                        // byte offset of the source ring's head
    unsigned char* const x1ring = wl;
    unsigned char* const sring = wl + src_ring_offset(EB, V);
    // byte offsets in a row (wave-uniform, added to the row offset): the
    // strip, and each factor's source range; a lane loads the 16-byte piece
    // lane16 bytes further on
    const uint32_t lane16 = 16u * (uint32_t)lane;
    uint32_t sofs1 = 0;
    uint32_t sofs[H + 1];
    auto issue_unit_start = [&]() {
        sofs1 = uni((int)((uint32_t)iu.j0 * EB));
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const uint32_t base = ((uint32_t)iu.j0 / (uint32_t)m) & ~(uint32_t)(EPP - 1);
            sofs[m] = (uint32_t)uni((int)(base * EB));
        });
    };
    issue_unit_start();

    // loads of the next row of the stream: the new source ranges (each into
    // the next slot of the source ring, by as many lane pieces as it holds,
    // 64 pieces per DMA instruction), then the row's m = 1 values; returns
    // the number of DMA instructions issued
    auto issue_next = [&]() -> int {
        if (!ivalid) return 0;
        if (ir == iu.r1) {
            if (!w.template next_unit<false>(ii, step, iu, &isrc)) {
                ivalid = false;
                return 0;
            }
            ir = iu.r0;
            issue_unit_start();
        }
        constexpr int XP = x1_pieces(EB, V);
        int c = dmas(XP);
        if constexpr (H >= 2) {
            const uint32_t fl = ir == iu.r0 ? 0xffffffffu : sload_u32(a.rowmask, ir);
            for_changed<H>(fl, [&](auto mc) {
                constexpr int m = decltype(mc)::value;
                constexpr int SP = slot_pieces(m, EB, V);
                {
                    const int at = ihead + slot_bytes(m, EB, V) > SRB ? 0 : ihead;
                    ihead = at + slot_bytes(m, EB, V);
                    const int srow = floordiv_c<m>(ir - a.c) + a.c;
                    static_for<0, dmas(SP) - 1>([&](auto gc) {
                        constexpr int g = decltype(gc)::value;
                        if (lane + 64 * g < SP)
                            w.dma(isrc, sring + at + 1024 * g, lane16 + 1024 * g, (uint32_t)srow * isrc.ldb + sofs[m]);
                    });
                    c += dmas(SP);
                }
            });
        }
        static_for<0, dmas(XP) - 1>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            if (XP % 64 == 0 || lane + 64 * g < XP)
                w.dma(isrc, x1ring + (iseq & (D - 1)) * x1_bytes(EB, V) + 1024 * g, lane16 + 1024 * g,
                      (uint32_t)ir * isrc.ldb + sofs1);
        });
        ++ir;
        ++iseq;
        return c;
    };

    // win[i]: vector-memory instructions issued for the row i + 1 after the
    // one being summed
    int win[D - 1];
    {
        const int c0 = issue_next();
        (void)c0;
#pragma unroll
        for (int i = 0; i < D - 1; ++i) win[i] = issue_next();
    }

    // ---- consume side ------------------------------------------------------------
    Unit cu;
    (void)w.template next_unit<true>(ci, step, cu, nullptr);
    int cseq = 0;     // stream index of the row being summed
    int ctail = 0;    // byte offset of the next source slot to read

    // per-unit lane constants
    int jb = 0;
    bool full = true;
    int lofsb[H + 1], rmod[H + 1];
    float sv[H + 1][V];
#pragma unroll
    for (int m = 0; m <= H; ++m) {
        lofsb[m] = rmod[m] = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) sv[m][v] = 0.0f;
    }
    auto unit_setup = [&]() {
        jb = cu.j0 + V * lane;
        full = cu.j0 + B <= cu.N;
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const uint32_t t = (uint32_t)cu.j0 + (uint32_t)(V * lane);
            const uint32_t q = t / (uint32_t)m;
            const uint32_t base = ((uint32_t)cu.j0 / (uint32_t)m) & ~(uint32_t)(EPP - 1);
            rmod[m] = (int)(t - q * (uint32_t)m);
            lofsb[m] = (int)(q - base) * EB;
        });
    };
    unit_setup();

    // candidate output of the current FOP
    int ncand = 0;
    int cur_f = cu.f;
    auto out_of = [&](int f, hs_cand*& out, int64_t& cap, unsigned long long*& cnts) {
        out = a.out;
        cap = a.cap;
        cnts = a.counts;
        if (a.n_fops > 0) {
            out = a.out + sload_i64(a.out_offsets, f);
            cap = sload_i64(a.caps, f);
            cnts = a.counts + (int64_t)f * (H + 1);
        }
    };
    // entries [0, n) of the buffer to positions base + e; those past the
    // capacity are dropped and counted per plane
    auto store = [&](int n, unsigned long long base, hs_cand* out, int64_t cap, unsigned long long* cnts) {
        for (int e0 = 0; e0 < n; e0 += 64) {   // uniform trip count
            const int e = e0 + lane;
            if (e < n) {
                const uint64_t c = cbuf[e];
                if ((int64_t)(base + e) < cap) reinterpret_cast<uint64_t*>(out)[base + e] = c;
                else atomicAdd(&cnts[((uint32_t)c >> a.s_bin) & ((1u << (a.s_row - a.s_bin)) - 1u)], 1ull);
            }
        }
    };
    auto flush = [&]() {
        if (ncand == 0) return;
        hs_cand* out;
        int64_t cap;
        unsigned long long* cnts;
        out_of(cur_f, out, cap, cnts);
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&cnts[H], (unsigned long long)ncand);
        base = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)base);
        store(ncand, base, out, cap, cnts);
        ncand = 0;
        wait_vm_all();   // retire the stores before the next counted wait
    };

    // hits of plane k among the lane's values (the rare path, whole wave);
    // `lanes` lanes have one, so the call adds at most V * lanes entries.
    // The buffer is written out only when that many might not fit (so that a
    // flush carries a nearly full buffer: each flush costs one atomic on the
    // list's shared counter), or, when V * 64 entries exceed the buffer,
    // before a bin whose hits might not fit.
    static_assert(CAP >= 64, "candidate buffer");
    constexpr bool kWhole = V * 64 <= CAP;
    auto emit = [&](auto kc, const float (&acc)[V], float tk, int r, int lanes) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        const uint32_t hi = ((uint32_t)r << a.s_row) | ((uint32_t)(k - 1) << a.s_bin);
        if (kWhole && ncand + V * lanes > CAP) flush();
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool hit = acc[v] > tk;
            const uint64_t mk = __builtin_amdgcn_ballot_w64(hit);
            if (mk) {
                if (!kWhole && ncand + __builtin_popcountll(mk) > CAP) flush();
                const int pre = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
                const float pw = EB == 4 ? acc[v] : acc[v] * a.inv_scale;   // unscaled power
                if (hit) cbuf[ncand + pre] = ((uint64_t)__float_as_uint(pw) << 32) | (hi | (uint32_t)(jb + v));
                ncand = uni(ncand + __builtin_popcountll(mk));
            }
        }
    };

    int cr = cu.r0;
    for (;;) {
        // wave-uniform loop state, stated as such for the compiler
        cr = uni(cr);
        cu.r0 = uni(cu.r0);
        cu.r1 = uni(cu.r1);
        cu.f = uni(cu.f);
        cu.N = uni(cu.N);
        cu.j0 = uni(cu.j0);
        ncand = uni(ncand);
        ctail = uni(ctail);
        ihead = uni(ihead);
        cur_f = uni(cur_f);
        ir = uni(ir);
        ci.i = uni(ci.i);
        ci.s = uni(ci.s);
        ii.i = uni(ii.i);
        ii.s = uni(ii.s);
        if (cr == cu.r1) {
            if (!w.template next_unit<true>(ci, step, cu, nullptr)) break;
            cr = cu.r0;
            if (cu.f != cur_f) {
                flush();
                cur_f = cu.f;
            }
            unit_setup();
        }
        const int r = cr;
        // the loads of this row were issued before those of the D - 1 rows
        // after it
        {
            uint32_t n = 0;
#pragma unroll
            for (int i = 0; i < D - 1; ++i) n += (uint32_t)win[i];
            wait_vm((uint32_t)uni((int)n));
        }

        float t[H];
#pragma unroll
        for (int k = 0; k < H; ++k) t[k] = thr[r * HS + k];

        // new source rows: the lane's values, selected per bin
        if constexpr (H >= 2) {
            const uint32_t fl = r == cu.r0 ? 0xffffffffu : sload_u32(a.rowmask, r);
            for_changed<H>(fl, [&](auto mc) {
                constexpr int m = decltype(mc)::value;
                {
                    const int at = ctail + slot_bytes(m, EB, V) > SRB ? 0 : ctail;
                    ctail = at + slot_bytes(m, EB, V);
                    const unsigned char* p = sring + at + lofsb[m];
                    if constexpr (src_vals(m, V) < V) {
                        // one element per group of m bins (or one for all)
#pragma unroll
                        for (int g = 0; g < src_vals(m, V); ++g) sv[m][g] = w.elem(p, g);
                    } else {
                        // bin v reads element (rmod + v) / m of the lane's
                        // range, which spans (V - 1) / m + 2 elements at most
                        constexpr int NE = (V - 1) / m + 2;
                        float e[NE];
#pragma unroll
                        for (int q = 0; q < NE; ++q) e[q] = w.elem(p, q);
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            float x = e[0];
#pragma unroll
                            for (int q = 1; q < NE; ++q)
                                if (rmod[m] + v >= q * m) x = e[q];
                            sv[m][v] = x;
                        }
                    }
                }
            });
        }

        float x[V];
        w.x1_vals(x1ring + (cseq & (D - 1)) * x1_bytes(EB, V), x);
        float acc[V];
        if (full) {
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = x[v];
        } else {
            // bins past the end start at -inf: no sum of them passes a threshold
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = jb + v < cu.N ? x[v] : -__builtin_inff();
        }

        auto detect = [&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            const float tk = t[k - 1];
            float mx = acc[0];
#pragma unroll
            for (int v = 1; v < V; ++v) mx = fmaxf(mx, acc[v]);
            const uint64_t any = __builtin_amdgcn_ballot_w64(mx > tk);
            if (__builtin_expect(any != 0, 0)) emit(kc, acc, tk, r, __builtin_popcountll(any));
        };
        detect(std::integral_constant<int, 1>{});
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                float s;
                if constexpr (src_vals(m, V) == 1) s = sv[m][0];
                else if constexpr (src_vals(m, V) < V) s = sv[m][v / m];
                else s = sv[m][v];
                acc[v] = acc[v] + s;
            }
            detect(mc);
        });

        // the LDS reads of this row are done before its slot is refilled
        wait_lgkm_all();
        const int cn = issue_next();
#pragma unroll
        for (int i = 0; i < D - 2; ++i) win[i] = win[i + 1];
        win[D - 2] = cn;
        ++cr;
        ++cseq;
    }
    // the wave's last candidates (batched: waves may end on different FOPs)
    if (a.n_fops > 0) {
        flush();
    } else {
        const unsigned long long base = block_reserve(ncand);
        hs_cand* out;
        int64_t cap;
        unsigned long long* cnts;
        out_of(cur_f, out, cap, cnts);
        store(ncand, base, out, cap, cnts);
    }
}

template <typename TIn, int H, int V>
hipError_t launch_walk_t(const WalkArgs& a, int grid, int lds_bytes, hipStream_t s)
{
    auto k = k_walk<TIn, H, V>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, walk::kWThreads, lds_bytes) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if (grid < 8) grid = 8;   // every XCD list needs a block
    hipLaunchKernelGGL(k, dim3(grid), dim3(walk::kWThreads), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace hsk
