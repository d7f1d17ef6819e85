/*
 * hs.h -- C ABI of the MI355X (gfx950) harmonic-summing library (libhs.so).
 *
 * The library computes the harmonic-summing module of Wang, Thiagaraj &
 * Sinnen, "Harmonic-summing Module of SKA on FPGA -- Optimising the
 * Irregular Memory Accesses" (arXiv:1805.12258), Sec. III:
 *
 *   FOP      filter-output plane, N_temp templates (rows) x N_chan bins of
 *            power, resident in device memory before a call (Sec. IV-A
 *            assumes the FOP is already in the accelerator's memory).
 *   SP_m(i,j) = FOP(floor(i/m), floor(j/m))                   (Eq. 1)
 *   HP_1 = FOP,  HP_k = HP_{k-1} + SP_k,  k = 2..N_hp          (Eq. 2)
 *   candidate  HP_k(i,j) > TA(k,i), one threshold per row and plane.
 *   candidate word  CL1 = F << (s_k + s_bin) | (k-1) << s_bin | B,
 *            CL2 = power (fp32)       (Sec. III, candidate list format)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Storage row r in [0, N_temp) holds template index i = r - N_temp/2
 *    (integer division): for odd N_temp the paper's range
 *    [-(N_temp-1)/2, (N_temp-1)/2]; for even N_temp [-N_temp/2, N_temp/2-1].
 *    floor() is the mathematical floor, also for negative i.
 *  * Partial sums are fp32 and formed in the order of Eq. 2 (m = 1, 2, ...,
 *    k), each rounded: results are bitwise those of a sequential fp32 loop.
 *  * The FOP is row-major [N_temp][ld] with ld >= N_chan elements of the
 *    plan's storage type.  The base pointer must be 16-byte aligned and ld a
 *    multiple of 4 (fp32) or 8 (fp16, bf16) elements; HS_ERR_INVALID
 *    otherwise.  Reduced-precision storage holds power * input_scale;
 *    thresholds and reported powers are in unscaled units.
 *  * Every pointer argument except hs_plan_desc.n_chans, the host count
 *    array of hs_check_counts and the output of hs_plan_schedule is DEVICE
 *    memory owned by the caller.  The library never frees caller memory.
 *  * `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work and return without waiting; the status covers argument checks and
 *    the launch only.  Output is valid once the stream has been synchronised.
 *  * A plan's results do not change after creation and it may be used from
 *    several streams and threads at once: all per-call state lives in caller
 *    buffers (the one-time device copy of a plan's tables is made under a
 *    lock).
 *  * No C++ exception crosses this interface.
 */
#ifndef HS_H
#define HS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hs_status {
    HS_OK = 0,
    HS_ERR_INVALID = -1,      /* bad argument, shape, alignment or pointer    */
    HS_ERR_OVERFLOW = -2,     /* more candidates than the output capacity     */
    HS_ERR_HIP = -3,          /* a HIP runtime call failed (no GPU, launch)   */
    HS_ERR_UNSUPPORTED = -4,  /* valid request the library does not implement */
    HS_ERR_NOMEM = -5         /* host or device allocation failed             */
} hs_status;

/* Which points a harmonic plane sums (Sec. III). */
typedef enum hs_mapping {
    HS_MAP_PAPER = 0,         /* Eq. 1-2: HP_k = sum_{m=1..k} FOP(floor(i/m),  */
                              /* floor(j/m)), cumulative over k (default)      */
    HS_MAP_FRACTIONAL = 1     /* HP_k = sum_{m=1..k} FOP(floor(m i/k),         */
                              /* floor(m j/k)): the FOP at the fractions m/k   */
                              /* of each point, terms added in m order; not    */
                              /* cumulative.  hs_sum and hs_detect only.       */
} hs_mapping;

typedef enum hs_dtype {
    HS_DTYPE_F32 = 0,         /* IEEE binary32 power                          */
    HS_DTYPE_F16 = 1,         /* IEEE binary16 of power * input_scale         */
    HS_DTYPE_BF16 = 2         /* bfloat16 of power * input_scale              */
} hs_dtype;

/* One candidate: CL1 (packed row, plane, bin) and CL2 (power), 8 bytes. */
typedef struct hs_cand {
    uint32_t idx;
    float power;
} hs_cand;

typedef struct hs_plan hs_plan;

typedef struct hs_plan_desc {
    int64_t n_temp;            /* N_temp >= 1 (Sec. III: 85)                    */
    int64_t n_chan;            /* N_chan >= 1 of a single-FOP plan (2^21);      */
                               /* ignored when n_fops >= 1                       */
    int32_t n_hp;              /* N_hp, 1..16 (Sec. III: 8)                      */
    int32_t dtype;             /* hs_dtype of the stored FOP                     */
    float input_scale;         /* stored = power * input_scale; a power of two;  */
                               /* 0 means 1; must be 1 for HS_DTYPE_F32          */
    int32_t n_fops;            /* 0: single FOP; >= 1: batch of n_fops FOPs      */
    const int64_t* n_chans;    /* HOST array [n_fops]: bins of each FOP          */
    int32_t tile_rows;         /* tuning: rows per tile, 0 = planner's choice    */
    int32_t persistent_blocks; /* tuning: batched grid size, 0 = planner         */
    int32_t schedule;          /* tuning: which detection kernel and order.      */
                               /* 0 = planner's choice: the strip walk for       */
                               /* 16-bit storage or more than 8 planes, the tile */
                               /* kernel otherwise; 4 = strip walk; 2 = tile     */
                               /* kernel (walk units and tiles dealt to the      */
                               /* eight XCDs so that sources are L2 hits);       */
                               /* 1 = strip walk, 3 = tile kernel, both in       */
                               /* increasing order (contiguous chunks).  The     */
                               /* walk needs N_temp >= 2 and a threshold table   */
                               /* of at most 16 KB; otherwise the tile kernel    */
                               /* runs.  Results do not depend on it.            */
    int32_t mapping;           /* hs_mapping (0 = HS_MAP_PAPER)                  */
    int32_t bins_per_lane;     /* tuning: bins per lane V of the strip walk (2,  */
                               /* 4 or 8: strips of 64 V bins); 0 = planner (8  */
                               /* for 16-bit storage up to 8 planes and for     */
                               /* batches, else 4)                              */
} hs_plan_desc;

/* Geometry chosen by the planner (host values; no GPU needed). */
typedef struct hs_plan_info {
    int32_t n_temp, n_hp, dtype, n_fops;
    int64_t n_chan_max;
    int32_t s_row, s_k, s_bin;  /* candidate-word shifts: row << s_row,          */
                                /* (k-1) << s_bin, field widths ceil(log2 .)     */
    int32_t tile_bins;          /* bins per tile                                 */
    int32_t tile_rows;          /* rows per tile                                 */
    int32_t row_blocks;         /* tiles across the rows                         */
    int32_t lds_bytes;          /* dynamic LDS of the fused kernel               */
    int64_t tiles_total;        /* tiles over all FOPs                           */
    int32_t src_rows[17];       /* src_rows[m]: distinct source rows of stretch  */
                                /* factor m over one full-height tile            */
    int64_t staged_words;       /* source words staged per full tile, m >= 2     */
    int32_t detector;           /* detection kernel: 0 tile kernel, 1 strip      */
                                /* walk, 2 fractional-mapping kernel             */
    int32_t mapping;            /* hs_mapping of the plan                        */
    int32_t bins_per_lane;      /* strip walk: bins per lane (0: no walk)        */
} hs_plan_info;

/* Create a plan.  Validates the shapes (HS_ERR_INVALID: N_temp < 1, n_hp
 * outside 1..16, unknown dtype or mapping, bins_per_lane not 0, 2, 4 or
 * 8, input_scale not a power of two, n_fops outside 0..65535, a batch with the fractional mapping,
 * a bin count < 1, or a candidate word wider than 32 bits, i.e.
 * ceil(log2 N_temp) + ceil(log2 N_hp) + ceil(log2 N_chan) > 32).  Host only:
 * touches no GPU. */
hs_status hs_plan_create(hs_plan** plan, const hs_plan_desc* desc);

/* Release a plan and the device tables it owns.  NULL is accepted. */
hs_status hs_plan_destroy(hs_plan* plan);

/* Planner geometry, for inspection and tests.  Host only. */
hs_status hs_plan_info_get(const hs_plan* plan, hs_plan_info* info);

/* The full-tile schedule of a single-FOP plan, for inspection and tests
 * (host only): words[0..8] are the offsets of eight lists in the entries that
 * follow, each entry (row_block << 24) | bin_tile; list b % 8 is walked by
 * block b.  Writes min(capacity, n) words to `words` (host memory, may be
 * NULL when capacity is 0) and returns n, the schedule's length in words
 * (0: the plan walks tiles in contiguous chunks), or -1 for a NULL plan. */
int64_t hs_plan_schedule(const hs_plan* plan, uint32_t* words, int64_t capacity);

/* Copy the plan's device tables (unit schedule and row table of the strip
 * walk, tile schedule of the tile kernels, per-FOP table of a batched plan)
 * to the current device, synchronously.  Every GPU call of a plan makes this
 * copy itself on first use on a device, except under stream capture: a call
 * being captured on a device that has no copy yet returns HS_ERR_INVALID and
 * launches nothing, so call this (or make one eager call) before capturing a
 * graph.  Calls also return HS_ERR_INVALID for a stream of another device
 * than the current one.  The copies are freed by hs_plan_destroy.
 * HS_ERR_NOMEM / HS_ERR_HIP on allocation or copy failure. */
hs_status hs_plan_upload(const hs_plan* plan);

/* All harmonic planes (Eq. 1-2), materialised: hp is [n_hp][N_temp][N_chan]
 * fp32 (plane-major, leading dimension N_chan) in unscaled units.
 * Single-FOP plans only. */
hs_status hs_sum(const hs_plan* plan, const void* fop, int64_t ld, float* hp, void* stream);

/* Harmonic planes and threshold detection fused (Sec. III detection; the
 * loop order of Algorithm 2, no plane is written to memory).
 *   ta       [n_hp][N_temp] fp32 thresholds, TA(k, row), unscaled units.
 *   out      [capacity] candidates, in no particular order.
 *   counts   [n_hp + 1] int64: candidates of each plane, then the total.
 *            Always the true counts, also when they exceed capacity; the
 *            call zeroes them first.
 * When the total exceeds capacity, `capacity` of the candidates are written
 * (which ones is unspecified); see hs_check_counts.  Single-FOP plans only. */
hs_status hs_detect(const hs_plan* plan, const void* fop, int64_t ld, const float* ta,
                    hs_cand* out, int64_t capacity, int64_t* counts, void* stream);

/* Per-plane capped candidate lists: the N_hp x N_cand list of Sec. III.
 * Input: a complete candidate list of this plan (cand[0..n), e.g. the first
 * counts[n_hp] entries of hs_detect when they fit its capacity), not
 * modified.  Output: out [n_hp][n_cand]; row k-1 holds min(n_cand,
 * candidates of plane k) entries chosen by `policy`, and out_counts [n_hp]
 * int64 (device) that number; entries past it are not written.
 *   HS_SELECT_TOP       the largest powers, ties to the smaller CL1 word,
 *                       listed in that order (powers in the IEEE total
 *                       order of their bits, -0 below +0);
 *   HS_SELECT_LAST_ALG2 the candidates met last when the loops run in
 *                       Algorithm 2 order (bin, template, plane), i.e. the
 *                       largest (bin, row) of the plane, listed oldest first
 *                       (Sec. IV-A: the last N_cand are kept);
 *   HS_SELECT_LAST_ALG1 the same for Algorithm 1 order (plane, template,
 *                       bin): the largest (row, bin), oldest first.
 * Deterministic: the same set gives the same lists in any input order.
 * n_cand <= 1024: a bounded selection (partition by plane, then per plane a
 * radix select on the policy's key and an LDS sort of the kept entries);
 * larger caps: HS_SELECT_TOP by two full radix sorts, the other policies
 * HS_ERR_UNSUPPORTED.  `work`: device memory of
 * hs_select_workspace_bytes(plan, n) bytes.  Stream-ordered.  hs_select_top
 * is hs_select with HS_SELECT_TOP. */
typedef enum hs_select_policy {
    HS_SELECT_TOP = 0,
    HS_SELECT_LAST_ALG2 = 1,
    HS_SELECT_LAST_ALG1 = 2
} hs_select_policy;
size_t hs_select_workspace_bytes(const hs_plan* plan, int64_t n);
hs_status hs_select(const hs_plan* plan, const hs_cand* cand, int64_t n, int32_t n_cand, int32_t policy,
                    hs_cand* out, int64_t* out_counts, void* work, void* stream);
hs_status hs_select_top(const hs_plan* plan, const hs_cand* cand, int64_t n, int32_t n_cand, hs_cand* out,
                        int64_t* out_counts, void* work, void* stream);

/* SingleHP baseline (Sec. IV-B; the kernel of Sec. V-A): the planes are
 * formed one after another through memory, HP_k = HP_{k-1} + SP_k, one
 * launch per plane, each plane written to `work` and read back for the next,
 * and thresholded as it is formed.  Same arguments, results and counts
 * semantics as hs_detect (the same candidate set, bitwise); it exists to
 * measure the fused kernel against the paper's baseline method on the same
 * GPU.  fp32 single-FOP plans only (HS_ERR_UNSUPPORTED otherwise).  `work`:
 * device memory of hs_singlehp_workspace_bytes(plan) bytes (two planes). */
size_t hs_singlehp_workspace_bytes(const hs_plan* plan);
hs_status hs_detect_singlehp(const hs_plan* plan, const float* fop, int64_t ld, const float* ta,
                             hs_cand* out, int64_t capacity, int64_t* counts, void* work, void* stream);

/* The single-launch SingleHP kernel (Sec. V-A evaluates both): the same
 * planes through the same two plane buffers, all N_hp of them formed in
 * order inside one launch (a point of HP_k needs only the same point of
 * HP_{k-1}, so each thread carries its own points from plane to plane).
 * Arguments, workspace and results as hs_detect_singlehp. */
hs_status hs_detect_singlehp_one(const hs_plan* plan, const float* fop, int64_t ld, const float* ta,
                                 hs_cand* out, int64_t capacity, int64_t* counts, void* work, void* stream);

/* hs_detect over a batch of FOPs of different lengths in one launch of a
 * persistent kernel.  Once the plan's tables are on the device
 * (hs_plan_upload or one eager call) the call does no host synchronisation
 * and no allocation, so it can be captured into a HIP graph; before that a
 * captured call returns HS_ERR_INVALID.  All arrays are DEVICE arrays:
 *   fops        [n_fops] pointers to the FOPs (each with the plan's dtype)
 *   lds         [n_fops] leading dimensions
 *   ta          [n_hp][N_temp], shared by every FOP
 *   out_offsets [n_fops] first entry of each FOP's candidates in `out`
 *   caps        [n_fops] capacity of each FOP's candidate range
 *   counts      [n_fops][n_hp + 1] per-FOP counts as in hs_detect
 * Alignment rules of the FOP apply to every FOP (checked on the device:
 * misaligned FOPs are skipped and their total count is set to -1).
 * `stream` must belong to the current device (HS_ERR_INVALID otherwise):
 * the plan's tables are copied per device.  Batched plans only. */
hs_status hs_detect_batched(const hs_plan* plan, const void* const* fops, const int64_t* lds,
                            const float* ta, hs_cand* out, const int64_t* out_offsets,
                            const int64_t* caps, int64_t* counts, void* stream);

/* Sort n candidates in place into the canonical order: ascending CL1 word
 * (row, then plane, then bin; CL1 words are unique within one FOP), a stable
 * radix sort on the low 32 bits of each 8-byte entry.  `work` is device
 * scratch of at least hs_sort_workspace_bytes(n) bytes (that query needs the
 * current HIP device; it returns 0 for n <= 1 or when no device answers). */
size_t hs_sort_workspace_bytes(int64_t n);
hs_status hs_sort_candidates(hs_cand* cand, int64_t n, void* work, void* stream);

/* Vector-Jacobian product of hs_sum (the transpose of Eq. 1-2): given
 * g = dL/dHP [n_hp][N_temp][N_chan] fp32 (leading dimension N_chan),
 * overwrites dfop [N_temp][N_chan] fp32 with
 *   dL/dFOP(a, b) = sum_{m=1..n_hp} sum over the m x m box of points (r, j)
 *                   with floor((r - c)/m) + c = a and floor(j/m) = b of
 *                   G_m(r, j),   G_m = sum_{k >= m} g_k,  c = N_temp / 2,
 * in unscaled units.  `work` is device scratch of
 * hs_backward_workspace_bytes(plan) bytes (per-tile partial sums).
 * Deterministic: no floating-point atomics, so the same input gives bitwise
 * the same output.  Single-FOP plans only. */
size_t hs_backward_workspace_bytes(const hs_plan* plan);
hs_status hs_sum_backward(const hs_plan* plan, const float* g, float* dfop, void* work,
                          void* stream);

/* Log-sum-exp statistic of each plane of one FOP (tau > 0):
 *   lse[k-1] = log sum_{i,j} exp(HP_k(i,j) / tau)        ([n_hp] fp64, device)
 * and, when `loss` is not NULL, the scalar
 *   *loss = sum_{k=1..n_hp} tau * lse[k-1]               (fp64, device; k order)
 * formed with running maxima and a fixed-order reduction (deterministic for
 * a given device and plan).  For fp32 plans hs_lse_forward is fused: each
 * lane keeps a (maximum, sum of exponentials) pair per plane over the points
 * it forms, the pairs are merged per block and then over the blocks in
 * order, and no plane is stored; other storage types materialise the planes
 * in `work` first.  hs_lse_backward overwrites dfop [N_temp][N_chan] fp32
 * with g times the gradient of L = sum_k tau * lse[k-1] with respect to the
 * FOP (unscaled units), g = *gscale (fp64, device; NULL means 1), so that an
 * autograd engine can pass the upstream gradient without a host copy: the
 * weights exp(HP_k / tau - lse[k-1]) taken through the transpose of
 * hs_sum_backward, formed inside its tile pass from the FOP (no weight plane
 * is stored), then the tile partials added in a fixed order
 * (deterministic).  `work` must hold hs_lse_workspace_bytes(plan) bytes.
 * Single-FOP plans only. */
size_t hs_lse_workspace_bytes(const hs_plan* plan);
hs_status hs_lse_forward(const hs_plan* plan, const void* fop, int64_t ld, float tau, double* lse,
                         double* loss, void* work, void* stream);
hs_status hs_lse_backward(const hs_plan* plan, const void* fop, int64_t ld, const double* lse,
                          float tau, const double* gscale, float* dfop, void* work, void* stream);

/* hs_lse_forward for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results (bitwise) as hs_lse_forward, with no workspace
 * argument.  Its scratch (the per-block pairs, at most 512 KB: 4096 blocks
 * x 16 planes x 2 floats) is a static device array, one per GPU, held until
 * the process ends; its address is looked up on the first call on each
 * device.  It calls no hipMalloc or hipFree and copies no plan tables (the
 * tile kernel takes the schedule if hs_plan_upload or an earlier call put it
 * on the device, else contiguous chunks, with the same results).  Every call
 * on a GPU shares that GPU's scratch: calls that overlap on one GPU (two
 * streams, two threads) race.  fp32 single-FOP plans with the paper's
 * mapping only (HS_ERR_UNSUPPORTED otherwise); HS_ERR_INVALID if the grid's
 * pairs would not fit the scratch (not reachable with the planner's grid). */
hs_status hs_lse_forward_noalloc(const hs_plan* plan, const void* fop, int64_t ld, float tau, double* lse,
                                 double* loss, void* stream);

/* Measurement: one streaming read of `bytes` bytes at `src` (device,
 * 16-byte aligned, bytes a multiple of 16) by `grid` blocks of 256 threads
 * (1..65536) with 16-byte loads.  Block b writes the fp32 sum
 * of the words it read to sink[b] (device, `grid` floats), so the sum of
 * sink is the sum of the buffer's fp32 values (up to rounding order).  Its
 * time over a resident FOP is the read-bandwidth ceiling the detection
 * kernels are compared against (they read the FOP once).  HS_ERR_INVALID
 * for a bad pointer, size, alignment or grid. */
hs_status hs_stream_read(const void* src, int64_t bytes, float* sink, int32_t grid, void* stream);

/* Host check of counts copied back from hs_detect: HS_ERR_OVERFLOW when
 * counts[n_hp] > capacity, HS_OK otherwise. */
hs_status hs_check_counts(const int64_t* counts_host, int32_t n_hp, int64_t capacity);

/* Static description of a status code. */
const char* hs_status_string(hs_status status);

/* Library version string. */
const char* hs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HS_H */
