// Internal declarations of libhs: plan object, tile geometry, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "hs.h"

namespace hsk {

// Tile geometry of the fused kernels.  A tile is a block of at most
// kMaxTileRows template rows times kTileBins consecutive bins; each lane owns
// kV consecutive bins of one row at a time, and wave w of a block handles the
// tile rows w + q kWaves, q < kRowsPerWave.
constexpr int kLanes = 64;
constexpr int kV = 4;
constexpr int kTileBins = kV * kLanes;   // 256
constexpr int kWaves = 8;
constexpr int kThreads = kWaves * kLanes;
constexpr int kRowsPerWave = 4;
constexpr int kMaxTileRows = kWaves * kRowsPerWave;   // 32
constexpr int kWaveCandCap = 320;        // per-wave LDS candidate buffer (>= kV*64)
constexpr int kMaxH = 16;
constexpr int kCntWords = 32;            // block bookkeeping words of the candidate flush
constexpr int kFlushParamBytes = 48;     // candidate-output parameters kept in LDS

// Source words a tile needs per row of stretch factor m: the largest number
// of distinct floor(j/m) over kTileBins consecutive bins starting at a
// multiple of kTileBins (j0 mod m is then a multiple of gcd(kTileBins, m),
// which for a power-of-two tile width is the lowest set bit of m).
static_assert((kTileBins & (kTileBins - 1)) == 0, "tile width must be a power of two");
__host__ __device__ constexpr int stage_pitch(int m)
{
    return (m - (m & -m) + kTileBins - 1) / m + 1;
}

// Staging layout in LDS, fixed at compile time for tiles of up to
// kMaxTileRows rows.  Region m (m = 2..H) holds stage_rows(m) source rows of
// stage_row_words(m) words.  Rows are loaded in 16-byte pieces (LDS-DMA of
// four words per lane), so a row starts at the source word floor(j0/m)
// rounded down to a multiple of four; when m divides kTileBins / 4 that word
// is already aligned.
__host__ __device__ constexpr bool stage_aligned(int m) { return (kTileBins / 4) % m == 0; }
__host__ __device__ constexpr int stage_row_words(int m)
{
    return (stage_pitch(m) + (stage_aligned(m) ? 0 : 3) + 3) & ~3;
}
// Most distinct floor(i/m) over kMaxTileRows consecutive template indices.
__host__ __device__ constexpr int stage_rows(int m) { return (kMaxTileRows + m - 2) / m + 1; }
__host__ __device__ constexpr int stage_region_words(int m) { return stage_rows(m) * stage_row_words(m); }
__host__ __device__ constexpr int stage_offset(int m)
{
    int o = 0;
    for (int k = 2; k < m; ++k) o += stage_region_words(k);
    return o;
}
// Words of one staging buffer for H planes.
__host__ __device__ constexpr int stage_words(int H) { return stage_offset(H + 1); }

// LDS-DMA pieces: one wave instruction moves 64 lanes x 4 words.  Region m is
// covered by stage_chunks(m) pieces (the last one partly masked); pieces are
// numbered across regions and piece g is issued by wave g % kWaves.
constexpr int kDmaWords = kLanes * 4;
__host__ __device__ constexpr int stage_chunks(int m)
{
    return (stage_region_words(m) + kDmaWords - 1) / kDmaWords;
}
__host__ __device__ constexpr int stage_chunk_begin(int m)
{
    int o = 0;
    for (int k = 2; k < m; ++k) o += stage_chunks(k);
    return o;
}
__host__ __device__ constexpr int stage_total_chunks(int H) { return stage_chunk_begin(H + 1); }
__host__ __device__ constexpr int stage_chunk_m(int g)
{
    int m = 2;
    while (g >= stage_chunk_begin(m + 1)) ++m;
    return m;
}
__host__ __device__ constexpr int stage_slots(int H)
{
    return (stage_total_chunks(H) + kWaves - 1) / kWaves;
}
// Registers holding a wave's piece offsets (at least one, for H = 1).
__host__ __device__ constexpr int stage_slot_regs(int H) { return stage_slots(H) > 0 ? stage_slots(H) : 1; }

// Raw staging of 16-bit FOPs: the same source rectangles as 16-bit halves,
// loaded by the same 16-byte pieces (8 halves per lane) and converted to the
// fp32 layout above inside LDS.  A raw row starts at floor(j0/m) rounded down
// to 8 halves, i.e. (blo & 4) halves before the fp32 row, and holds the fp32
// row's words after that shift.
__host__ __device__ constexpr int raw_row_halves(int m)
{
    return (stage_row_words(m) + (stage_aligned(m) ? 0 : 4) + 7) & ~7;
}
__host__ __device__ constexpr int raw_region_halves(int m) { return stage_rows(m) * raw_row_halves(m); }
__host__ __device__ constexpr int raw_offset(int m)
{
    int o = 0;
    for (int k = 2; k < m; ++k) o += raw_region_halves(k);
    return o;
}
// Halves of one raw staging buffer for H planes.
__host__ __device__ constexpr int raw_halves(int H) { return raw_offset(H + 1); }
constexpr int kDmaHalves = kLanes * 8;
__host__ __device__ constexpr int raw_chunks(int m) { return (raw_region_halves(m) + kDmaHalves - 1) / kDmaHalves; }
__host__ __device__ constexpr int raw_chunk_begin(int m)
{
    int o = 0;
    for (int k = 2; k < m; ++k) o += raw_chunks(k);
    return o;
}
__host__ __device__ constexpr int raw_total_chunks(int H) { return raw_chunk_begin(H + 1); }
__host__ __device__ constexpr int raw_chunk_m(int g)
{
    int m = 2;
    while (g >= raw_chunk_begin(m + 1)) ++m;
    return m;
}
__host__ __device__ constexpr int raw_slots(int H) { return (raw_total_chunks(H) + kWaves - 1) / kWaves; }
// Piece slots of the storage type: raw pieces for 16-bit storage.
__host__ __device__ constexpr int dma_slots(int H, int elem_bytes)
{
    return elem_bytes == 4 ? stage_slots(H) : raw_slots(H);
}
__host__ __device__ constexpr int dma_slot_regs(int H, int elem_bytes)
{
    return dma_slots(H, elem_bytes) > 0 ? dma_slots(H, elem_bytes) : 1;
}

// Row table of a tile: per tile row, the staging offsets of stretch factors
// 2..H (padded to 4 words) followed by the H thresholds (padded to 4).
__host__ __device__ constexpr int row_table_thr_offset(int H) { return ((H - 1) + 3) & ~3; }
__host__ __device__ constexpr int row_table_stride(int H)
{
    return row_table_thr_offset(H) + ((H + 3) & ~3);
}

// The row table covers all T rows (and is built once per launch) when it
// takes at most this many bytes; otherwise it covers one tile's rows.
constexpr int kWholeTableBytes = 12 * 1024;
__host__ __device__ constexpr bool table_whole(int T, int H)
{
    return T * row_table_stride(H) * 4 <= kWholeTableBytes;
}

// LDS bytes after the two staging buffers: the row table (two per-tile
// copies unless it covers the whole plane), the per-wave candidate buffers,
// the per-plane counters of the block and the candidate-output parameters.
__host__ __device__ constexpr int smem_tail_bytes(int T, int R, int H)
{
    return (table_whole(T, H) ? T : 2 * R) * row_table_stride(H) * 4 +
           kWaves * kWaveCandCap * 8 + kCntWords * 4 + kFlushParamBytes;
}

__host__ __device__ inline int64_t floordiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (q * b > a) ? q - 1 : q;
}

__host__ __device__ inline int floordiv32(int a, int b)
{
    int q = a / b;
    return (q * b > a) ? q - 1 : q;
}

// Arguments of one fused launch over one FOP (or one FOP of a batch).
struct TileArgs {
    const void* fop;
    int64_t ld;
    int64_t N;              // bins
    int32_t T;              // rows
    int32_t c;              // centre row: row r holds template index r - c
    int32_t R;              // rows per tile
    int32_t row_blocks;     // tiles across the rows
    float scale;            // stored = power * scale
    float inv_scale;        // applied when a stored value is converted to fp32
    const float* ta;        // [H][T], unscaled
    // detect
    hs_cand* out;
    int64_t cap;
    unsigned long long* counts;   // [H+1]
    int32_t s_row, s_bin;
    uint32_t kmask;               // (1 << s_k) - 1
    int32_t table_whole;          // row table covers all T rows (built once)
    // materialised planes
    float* hp;              // [H][T][N]
    // Full-tile schedule: sched[0..8] are the offsets of eight lists in the
    // entries that follow, each entry (rb << 24) | bt.  Block b walks list
    // b % 8 with a stride of the number of blocks that share it.  Null: every
    // block takes a contiguous chunk of the row-block-major numbering.
    const uint32_t* sched;
    // fused log-sum-exp: per block and plane the pair (max, sum of
    // exp2((x - max) * lse_c)) of the block's values x in storage units
    float* lse_part;        // [gridDim.x][H][2]
    float lse_c;            // inv_scale * log2(e) / tau
};

// Arguments of the batched persistent launch.
struct BatchArgs {
    const void* const* fops;
    const int64_t* lds;
    const int64_t* n_chans;       // device [n_fops]
    const int64_t* tile_prefix;   // device [n_fops + 1]
    int64_t tiles_total;
    int32_t n_fops;
    int32_t T, c, R, row_blocks;
    float scale, inv_scale;
    const float* ta;
    hs_cand* out;
    const int64_t* out_offsets;
    const int64_t* caps;
    unsigned long long* counts;   // [n_fops][H+1]
    int32_t s_row, s_bin;
    uint32_t kmask;
    int32_t table_whole;
};

// Arguments of the strip-walk detection kernel (hs_walk_impl.h), for one FOP
// (n_fops == 0: fop, ld, N, out, cap, counts) or a batch (n_fops >= 1: the
// per-FOP device arrays; out, counts are the bases).
struct WalkArgs {
    const void* fop;
    int64_t ld;
    int32_t N;
    int32_t n_fops;
    const void* const* fops;      // [n_fops] device
    const int64_t* lds;           // [n_fops] device
    const int64_t* n_chans;       // [n_fops] device (plan table)
    const int64_t* out_offsets;   // [n_fops] device
    const int64_t* caps;          // [n_fops] device
    int32_t T, c;                 // rows; row r holds template index r - c
    int32_t band_split;           // bands [0, band_split) and [band_split, T); 0: one band
    float scale, inv_scale;
    const float* ta;              // [H][T] unscaled
    hs_cand* out;
    int64_t cap;
    unsigned long long* counts;   // [H+1] (batch: [n_fops][H+1])
    int32_t s_row, s_bin;
    const uint32_t* rowmask;      // [T]: bit m set when floor((r-c)/m) changes at row r
    const uint32_t* ent;          // schedule entries (band << 24) | strip
    const int32_t* seg;           // [n_seg][4]: FOP, first entry, first index, end index
    const uint32_t* xseg;         // [9]: segments of XCD x are [xseg[x], xseg[x+1])
};

enum Mode { kModeDetect = 0, kModeSum = 1, kModeLse = 2 };

// Fused log-sum-exp: most blocks one launch may use (the partial pairs of
// the workspace are sized for it).
constexpr int kLseMaxBlocks = 4096;

// Static device scratch of the allocation-free entry points: the fused
// statistic's per-block pairs at its largest grid and plane count.
constexpr size_t kNoAllocScratchBytes = (size_t)kLseMaxBlocks * kMaxH * 2 * sizeof(float);
// Address of this GPU's copy (looked up once per device).
hipError_t noalloc_scratch(void** ptr);

// LDS bytes of the fused kernel: fp32 storage double-buffers the fp32
// staging; 16-bit storage double-buffers the raw staging and converts into
// one fp32 staging buffer.
__host__ __device__ constexpr int fused_stage_bytes(int H, int elem_bytes)
{
    return elem_bytes == 4 ? 2 * stage_words(H) * 4 : stage_words(H) * 4 + 2 * ((raw_halves(H) * 2 + 15) & ~15);
}
int fused_lds_bytes(int T, int R, int H, int mode, int elem_bytes);

hipError_t launch_fused(int mode, int dtype, int H, const TileArgs& a, int64_t n_tiles,
                        int grid, int lds_bytes, hipStream_t s);
hipError_t launch_batched(int dtype, int H, const BatchArgs& a, int grid, int lds_bytes,
                          hipStream_t s);
hipError_t launch_stream_read(const void* src, int64_t bytes, float* sink, int grid, hipStream_t s);
hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s);

// Bounded per-plane selection (policies of hs_select, n_cand <= kSelLdsCand).
constexpr int kSelLdsCand = 1024;
hipError_t select_bounded(const uint64_t* cand, int64_t n, int H, int s_bin, int s_k, int policy, int n_cand,
                          uint64_t* out, int64_t* out_counts, void* work, hipStream_t s);
size_t select_bounded_workspace(int64_t n, int H, int n_cand);

// Fractional mapping (HP_k = sum_{m<=k} FOP(floor(m i/k), floor(m j/k))):
// planes (hp) or detection (ta, out, cap, counts), single FOP, N <= 2^24.
constexpr int64_t kFracMaxBins = (int64_t)1 << 24;
struct FracArgs {
    const void* fop;
    int64_t ld;
    int32_t T, c, N, H;
    float scale, inv_scale;
    const float* ta;
    float* hp;
    hs_cand* out;
    int64_t cap;
    unsigned long long* counts;
    int32_t s_row, s_bin;
    uint64_t magic[kMaxH + 1];    // ceil(2^32 / k): floor division by k
};
void frac_magic(FracArgs& a);
hipError_t launch_frac(int dtype, bool detect, const FracArgs& a, hipStream_t s);
// Per-plane counts of stored candidates (after a detection kernel): lists at
// out + out_offsets[f] with capacities caps[f] (or one list of capacity `cap`
// when both are null), counts [n_lists][H+1].
hipError_t launch_plane_counts(const hs_cand* out, const int64_t* out_offsets, const int64_t* caps, int64_t cap,
                               unsigned long long* counts, int n_lists, int H, int s_bin, uint32_t kmask,
                               hipStream_t s);

// Strip-walk detection (hs_walk_*.hip): whether a plane's thresholds fit
// the kernel's LDS table (and the plane has rows enough for its pipeline),
// which bins-per-lane values V it is built for (strips of 64 V bins), the
// LDS bytes of a block, and the launcher (grid <= 0: resident grid).
bool walk_supported(int T, int H);
bool walk_v_ok(int V);
int walk_lds_bytes(int T, int H, int dtype, int V);
constexpr int kWalkDepth = 2;        // rows in flight per wave; every band has at least this many rows
hipError_t launch_walk(int dtype, int H, int V, const WalkArgs& a, int grid, int lds_bytes, hipStream_t s);

// Transpose of the plane map and the log-sum-exp statistic (hs_grad.hip).
int64_t backward_partial_floats(int T, int H, int R, int64_t N);
// The statistic's backward with the weights formed in the transpose's tile
// pass (tiles of lse_backward_tile_rows() rows; `part` holds
// backward_partial_floats(T, H, that, N) floats).
hipError_t launch_lse_backward_fused(int dtype, const void* fop, int64_t ld, int T, int64_t N, int H, float inv_scale,
                                    double tau, const double* lse, const double* gscale, float* dfop, float* part,
                                    hipStream_t s);
int lse_backward_tile_rows();
hipError_t launch_backward(const float* g, float* dfop, float* part, int T, int64_t N, int H, int R,
                           hipStream_t s);
int64_t lse_part_bytes(int H);
hipError_t launch_lse_reduce(const float* hp, int64_t plane, int H, double tau, void* work, double* lse,
                             hipStream_t s);
hipError_t launch_lse_fused_final(const float* part, int nblk, int H, double inv_scale, double tau,
                                  double* lse, hipStream_t s);
hipError_t launch_lse_loss(const double* lse, int H, double tau, double* loss, hipStream_t s);
// Canonical candidate order (hs_sort.hip).
hipError_t sort_workspace(int64_t n, size_t* bytes);
hipError_t sort_candidates(uint64_t* cand, int64_t n, void* work, hipStream_t s);

}  // namespace hsk

struct hs_plan {
    int64_t T = 0;
    int64_t N = 0;          // single FOP: bins; batched: maximum bins
    int H = 0;
    int dtype = 0;
    float scale = 1.0f;
    int n_fops = 0;
    int mapping = HS_MAP_PAPER;
    std::vector<int64_t> n_chans;
    int s_row = 0, s_k = 0, s_bin = 0;
    int tile_rows = 0, row_blocks = 0;
    int lds_bytes = 0;
    int64_t tiles_total = 0;
    int persistent_blocks = 0;
    std::vector<int64_t> tile_prefix;   // batched: tiles before each FOP

    std::vector<uint32_t> sched;         // single FOP: full-tile schedule (empty: chunks)

    // Strip-walk detection: unit schedule and row table, host copy laid out
    // as the device buffer (offsets in bytes), copied once per device.
    bool walk = false;
    int walk_v = 4;                      // bins per lane (strips of 64 walk_v bins)
    int band_split = 0;
    std::vector<unsigned char> walk_tab;
    size_t off_xseg = 0, off_rowmask = 0, off_seg = 0, off_nchan = 0, off_ent = 0;
    int walk_lds = 0;

    // Device copies of the batched tables and of the schedule, made at plan
    // creation on the current device or on first use per device.
    mutable std::mutex mu;
    mutable int64_t* d_tables[64] = {nullptr};
    mutable uint32_t* d_sched[64] = {nullptr};
    mutable unsigned char* d_walk[64] = {nullptr};
};
