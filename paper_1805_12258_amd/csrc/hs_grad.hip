// Transpose of the plane map (the vector-Jacobian product of Eq. 1-2) and
// the log-sum-exp statistic built on it.
//
// Backward.  With G_m = sum_{k >= m} g_k (suffix sums over the planes),
//     dFOP(a, b) = sum_m  sum_{(r, j) : src(r, m) = a, floor(j/m) = b}  G_m(r, j),
// where src(r, m) = floor((r - c)/m) + c is the source row of Eq. 1.  The
// preimage of (a, b) under m is an m x m box of plane points (clipped to the
// plane).  Two deterministic passes, no floating-point atomics:
//   1. per tile of 32 rows x 256 bins: read g_H .. g_1 once (coalesced), form
//      the suffix sums in registers, write G_1 to dFOP, and for m >= 2 stage
//      G_m in LDS and sum each target's box inside the tile (fixed order) into
//      a per-(m, tile) partial rectangle in the workspace;
//   2. per dFOP point: add, for m = 2..H in order, the (at most 4) tile
//      partials that cover it.
// The same input gives bitwise the same output.
//
// Log-sum-exp.  lse_k = log sum_{i,j} exp(HP_k(i,j) / tau) per plane, with a
// running maximum (each term exp(x - M) <= 1) and a fixed two-level
// reduction; lse is returned in fp64 so that the weights
// exp(HP_k / tau - lse_k) of the backward keep fp32 accuracy even where
// |lse| is large.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hs_internal.h"

namespace hsk {

namespace {

// Pass 1 tiles are kMaxTileRows x kTileBins like the forward's, covered by
// 8 waves of 4 rows each.
constexpr int kGWaves = 8;
constexpr int kGRows = kMaxTileRows / kGWaves;
constexpr int kGThreads = kGWaves * kLanes;

__device__ __forceinline__ int src_row(int r, int m, int c)
{
    return floordiv32(r - c, m) + c;
}

// Offset (in floats) of the partial rectangles of stretch factor m.
__host__ __device__ inline int64_t partial_offset(int m, int row_blocks, int64_t n_bt)
{
    int64_t o = 0;
    for (int k = 2; k < m; ++k)
        o += (int64_t)row_blocks * stage_rows(k) * n_bt * stage_pitch(k);
    return o;
}

// Pass 1: one block per tile (rb, bt).
__global__ __launch_bounds__(kGThreads) void k_bwd_tiles(const float* __restrict__ g, float* __restrict__ dfop,
                                                         float* __restrict__ part, int T, int N, int H,
                                                         int R, int row_blocks, int n_bt)
{
    __shared__ float tile[kMaxTileRows * kTileBins];
    const int rb = blockIdx.x / n_bt;
    const int bt = blockIdx.x - rb * n_bt;
    const int r0 = rb * R;
    const int nr = min(R, T - r0);
    const int j0 = bt * kTileBins;
    const int nb = min(kTileBins, N - j0);
    const int c = T / 2;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t plane = (int64_t)T * N;

    float s[kGRows][kV], nx[kGRows][kV];
#pragma unroll
    for (int q = 0; q < kGRows; ++q)
#pragma unroll
        for (int v = 0; v < kV; ++v) s[q][v] = 0.0f;

    // g_m at the thread's points, into nx (0 outside the tile); 16-byte
    // loads when the tile is full and the rows are 16-byte aligned
    const bool vec = nb == kTileBins && (N & 3) == 0 && (reinterpret_cast<uintptr_t>(g) & 15) == 0;
    auto load_plane = [&](int m) {
#pragma unroll
        for (int q = 0; q < kGRows; ++q) {
            const int rr = wave + kGWaves * q;
            const float* src = g + (int64_t)(m - 1) * plane + (int64_t)(r0 + (rr < nr ? rr : 0)) * N + j0;
            if (rr < nr && vec) {
                const float4 t4 = *reinterpret_cast<const float4*>(src + kV * lane);
                nx[q][0] = t4.x; nx[q][1] = t4.y; nx[q][2] = t4.z; nx[q][3] = t4.w;
            } else {
#pragma unroll
                for (int v = 0; v < kV; ++v) {
                    const int jj = kV * lane + v;
                    nx[q][v] = (rr < nr && jj < nb) ? src[jj] : 0.0f;
                }
            }
        }
    };
    load_plane(H);

    for (int m = H; m >= 1; --m) {
        // suffix sum G_m = g_m + G_{m+1} at the thread's points (outside the
        // tile both are 0)
#pragma unroll
        for (int q = 0; q < kGRows; ++q)
#pragma unroll
            for (int v = 0; v < kV; ++v) s[q][v] = nx[q][v] + s[q][v];
        // the next plane's loads fly while this factor's boxes are summed
        if (m > 1) load_plane(m - 1);
        if (m == 1) {
#pragma unroll
            for (int q = 0; q < kGRows; ++q) {
                const int rr = wave + kGWaves * q;
                if (rr >= nr) continue;
                float* dst = dfop + (int64_t)(r0 + rr) * N + j0;
#pragma unroll
                for (int v = 0; v < kV; ++v) {
                    const int jj = kV * lane + v;
                    if (jj < nb) dst[jj] = s[q][v];
                }
            }
            break;
        }
        __syncthreads();               // the previous factor's gathers are done
#pragma unroll
        for (int q = 0; q < kGRows; ++q) {
            const int rr = wave + kGWaves * q;
#pragma unroll
            for (int v = 0; v < kV; ++v) tile[rr * kTileBins + kV * lane + v] = s[q][v];
        }
        __syncthreads();
        // every target cell of the tile for factor m: rows src(r0, m) + tr,
        // bins floor(j0/m) + tc; its box inside this tile, summed row by row
        const int NR = stage_rows(m), P = stage_pitch(m);
        const int lo = src_row(r0, m, c);
        const int blo = j0 / m;
        float* out = part + partial_offset(m, row_blocks, n_bt) +
                     (((int64_t)rb * NR) * n_bt + bt) * P;
        for (int e = threadIdx.x; e < NR * P; e += kGThreads) {
            const int tr = e / P, tc = e - tr * P;
            const int a = lo + tr, b = blo + tc;
            const int ra = max(c + m * (a - c), r0), rz = min(c + m * (a - c) + m - 1, r0 + nr - 1);
            const int ja = max(m * b, j0), jz = min(m * b + m - 1, j0 + nb - 1);
            float acc = 0.0f;
            for (int r = ra; r <= rz; ++r)
                for (int j = ja; j <= jz; ++j) acc += tile[(r - r0) * kTileBins + (j - j0)];
            out[(int64_t)tr * n_bt * P + tc] = acc;
        }
    }
}

// Pass 2: dFOP(a, b) += sum over m = 2..H of the partials covering (a, b).
__global__ __launch_bounds__(256) void k_bwd_reduce(float* __restrict__ dfop, const float* __restrict__ part,
                                                    int T, int N, int H, int R, int row_blocks, int n_bt)
{
    const int c = T / 2;
    const int64_t total = (int64_t)T * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e / N), b = (int)(e - (int64_t)a * N);
        float acc = dfop[e];
        for (int m = 2; m <= H; ++m) {
            const int first = max(c + m * (a - c), 0), last = min(c + m * (a - c) + m - 1, T - 1);
            if (first > last || (int64_t)m * b > N - 1) continue;
            const int jb0 = m * b, jb1 = min(m * b + m - 1, N - 1);
            const int NR = stage_rows(m), P = stage_pitch(m);
            const float* pm = part + partial_offset(m, row_blocks, n_bt);
            float pmsum = 0.0f;
            for (int rb = first / R; rb <= last / R; ++rb) {
                const int tr = a - src_row(rb * R, m, c);
                for (int bt = jb0 / kTileBins; bt <= jb1 / kTileBins; ++bt) {
                    const int tc = b - (bt * kTileBins) / m;
                    pmsum += pm[(((int64_t)rb * NR + tr) * n_bt + bt) * P + tc];
                }
            }
            acc += pmsum;
        }
        dfop[e] = acc;
    }
}

// ---- statistic backward, weights formed in the transpose's tile pass -------
//
// dL/dFOP for L = sum_k tau lse_k is the transpose applied to the weights
// g_k = gscale exp(HP_k / tau - lse_k).  Instead of writing the H weight
// planes and reading them back, the tile pass forms them: each thread takes
// one row and four bins of a 16-row x 256-bin tile, sums HP_1..HP_H from the
// FOP in the order of Eq. 2 (the forward's sums, so the weights are those of
// the planes the statistic was taken over), turns each into its weight in
// registers, forms the suffix sums G_m, writes G_1 to dFOP, and for m >= 2
// sums each target's m x m box inside the tile into the per-(m, tile)
// partial rectangles that the second pass adds (the same deterministic
// layout and order as the plain transpose above).
template <int A, int B, typename F>
__host__ __device__ inline void static_for(F&& f)
{
    if constexpr (A <= B) {
        f(std::integral_constant<int, A>{});
        static_for<A + 1, B>(f);
    }
}

constexpr int kFR = 16;                     // rows per tile: one wave each
constexpr int kFThreads = kFR * kLanes;     // 1024

template <typename TIn> struct GIo;
template <> struct GIo<float> {
    __device__ static float ld(const void* p, int64_t e) { return static_cast<const float*>(p)[e]; }
    // four consecutive values at element e (16-byte aligned)
    __device__ static void ld4(const void* p, int64_t e, float (&x)[4])
    {
        const float4 q = *reinterpret_cast<const float4*>(static_cast<const float*>(p) + e);
        x[0] = q.x;
        x[1] = q.y;
        x[2] = q.z;
        x[3] = q.w;
    }
};
template <> struct GIo<_Float16> {
    __device__ static float ld(const void* p, int64_t e) { return (float)static_cast<const _Float16*>(p)[e]; }
    __device__ static void ld4(const void* p, int64_t e, float (&x)[4])
    {
        const uint2 q = *reinterpret_cast<const uint2*>(static_cast<const _Float16*>(p) + e);
        _Float16 h[4];
        __builtin_memcpy(h, &q, 8);
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = (float)h[v];
    }
};
struct bf16_bits {
    uint16_t b;
};
template <> struct GIo<bf16_bits> {
    __device__ static float ld(const void* p, int64_t e)
    {
        return __uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[e] << 16);
    }
    __device__ static void ld4(const void* p, int64_t e, float (&x)[4])
    {
        const uint2 q = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(p) + e);
        x[0] = __uint_as_float(q.x << 16);
        x[1] = __uint_as_float(q.x & 0xffff0000u);
        x[2] = __uint_as_float(q.y << 16);
        x[3] = __uint_as_float(q.y & 0xffff0000u);
    }
};

// Rows of partial sums a 16-row tile produces for stretch factor m: the most
// distinct floor(i/m) over kFR consecutive template indices.
__host__ __device__ constexpr int fused_rows(int m) { return (kFR + m - 2) / m + 1; }
__host__ __device__ inline int64_t fused_partial_offset(int m, int row_blocks, int64_t n_bt)
{
    int64_t o = 0;
    for (int k = 2; k < m; ++k) o += (int64_t)row_blocks * fused_rows(k) * n_bt * stage_pitch(k);
    return o;
}

// LDS of one tile.  gt: the tile's G_m values, one row per wave, with zero
// bins on both sides (the first target column starts up to m - 1 bins
// before the tile, the last one can end up to 23 bins after it for m <= 16)
// so that the m-bin sums read zeros outside the tile instead of testing
// bounds.
// hr: the rows' m-bin sums (pitch stage_pitch(2), the widest), with zero
// rows above and below for the same reason on the m-row sums: a target row
// reaches at most m - 1 rows above the tile and 2m - 2 below.
constexpr int kGPad = kMaxH;                       // zero bins before the tile
constexpr int kGPadR = 2 * kMaxH;                  // and after it
constexpr int kGPitch = kGPad + kTileBins + kGPadR;
constexpr int kHPitch = stage_pitch(2);
template <int H> constexpr int hr_top() { return H - 1; }
template <int H> constexpr int hr_rows() { return kFR + 3 * H - 3; }

// The weight g_k = gscale exp(HP_k / tau - lse_k) in base 2 and fp32, with
// no fp64 operation per point: with L_k = tau lse_k / input_scale (fp64,
// in storage units) split as L_hi + L_lo (two fp32 values, L_lo below half
// an ulp of L_hi),
//     log2 g_k = (HP - L_hi) c - L_lo c + log2|gscale|,  c = log2(e) / (tau scale),
// formed as fma(HP - L_hi, c, K_k) with K_k = -L_lo c + log2|gscale| per
// plane.  HP - L_hi is exact where HP is within a factor two of L_hi (the
// weights that matter: lse_k is at least max HP_k / tau), and the remaining
// roundings leave a few fp32 ulps of relative error in the exponent.  A
// negative gscale flips the sign of the result, zero gives zero weights.
// Up to eight planes the tile kernel keeps to 64 VGPRs so that two blocks
// (eight waves per SIMD) share a compute unit and one block's loads overlap
// the other's arithmetic.
template <int H> constexpr int bwd_min_waves() { return H <= 8 ? 8 : 4; }

template <typename TIn, int H>
__global__ __launch_bounds__(kFThreads, bwd_min_waves<H>()) void k_lse_bwd_tiles(const void* __restrict__ fop, int64_t ld, int T, int N,
                                                             double inv_scale, double tau, float c2,
                                                             const double* __restrict__ lse,
                                                             const double* __restrict__ gscale_p,
                                                             float* __restrict__ dfop, float* __restrict__ part,
                                                             int row_blocks, int n_bt)
{
    __shared__ __align__(16) float gt[kFR * kGPitch];
    __shared__ float hr[hr_rows<H>() * kHPitch];
    __shared__ float lsplit[2 * H];                  // L_hi, K of every plane
    const int rb = blockIdx.x / n_bt;
    const int bt = blockIdx.x - rb * n_bt;
    const int r0 = rb * kFR;
    const int nr = min(kFR, T - r0);
    const int j0 = bt * kTileBins;
    const int nb = min(kTileBins, N - j0);
    const int c = T / 2;
    const int lane = threadIdx.x & 63;
    const int rr = threadIdx.x >> 6;            // row of the tile (the wave)
    const int r = r0 + rr;
    const bool row_ok = rr < nr;
    const bool full = row_ok && nb == kTileBins;
    const double gsc = gscale_p ? *gscale_p : 1.0;
    if (threadIdx.x < H) {
        const double L = tau * lse[threadIdx.x] / inv_scale;
        const float hi = (float)L;
        const float lo = (float)(L - (double)hi);
        lsplit[2 * threadIdx.x] = hi;
        lsplit[2 * threadIdx.x + 1] = (float)(-(double)lo * (double)c2 + log2(fabs(gsc)));
    }
    // zero pads (never written afterwards)
    for (int e = threadIdx.x; e < kFR * (kGPad + kGPadR); e += kFThreads) {
        const int row = e / (kGPad + kGPadR), q = e - row * (kGPad + kGPadR);
        gt[row * kGPitch + (q < kGPad ? q : kTileBins + q)] = 0.0f;
    }
    for (int e = threadIdx.x; e < hr_rows<H>() * kHPitch; e += kFThreads) hr[e] = 0.0f;

    // weights of every plane at the thread's four points (0 outside the plane)
    float G[H][kV];
    {
        // every source value first (all loads in flight together), then the
        // sums.  Plane 1: the thread's four values (one 16-byte load in a
        // full tile).  m >= 2: the four bins j .. j+3 read elements
        // floor(j/m) and at most one more, so two loads and a select.
        const int jl = j0 + kV * lane;
        const int jc = min(jl, N - 1);                 // lanes past the end read a valid element
        {
            const int64_t rowe = (int64_t)(row_ok ? r : 0) * ld;
            if (nb == kTileBins) {
                GIo<TIn>::ld4(fop, rowe + jl, G[0]);
            } else {
#pragma unroll
                for (int v = 0; v < kV; ++v) G[0][v] = GIo<TIn>::ld(fop, rowe + min(jl + v, N - 1));
            }
        }
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int sr = row_ok ? floordiv32(r - c, m) + c : 0;
            const int e0 = jc / m;
            const int e1 = min(e0 + 1, (N - 1) / m);
            const float x0 = GIo<TIn>::ld(fop, (int64_t)sr * ld + e0);
            const float x1 = GIo<TIn>::ld(fop, (int64_t)sr * ld + e1);
            const int split = m * (e0 + 1) - jc;           // bins v < split read element e0
#pragma unroll
            for (int v = 0; v < kV; ++v) G[m - 1][v] = v < split ? x0 : x1;
        });
        __syncthreads();                               // split exponents and zero pads are in LDS
        float acc[kV];
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            const float lhi = lsplit[2 * (k - 1)], kk = lsplit[2 * (k - 1) + 1];
#pragma unroll
            for (int v = 0; v < kV; ++v) {
                acc[v] = k == 1 ? G[0][v] : acc[v] + G[k - 1][v];
                G[k - 1][v] = __builtin_amdgcn_exp2f(__builtin_fmaf(acc[v] - lhi, c2, kk));
            }
        }
        if (!full) {
#pragma unroll
            for (int v = 0; v < kV; ++v) {
                const bool ok = row_ok && kV * lane + v < nb;
#pragma unroll
                for (int k = 0; k < H; ++k) G[k][v] = ok ? G[k][v] : 0.0f;
            }
        }
    }
    // suffix sums G_m = g_m + G_{m+1}, from the last plane down
#pragma unroll
    for (int m = H - 1; m >= 1; --m) {
#pragma unroll
        for (int v = 0; v < kV; ++v) G[m - 1][v] = G[m - 1][v] + G[m][v];
    }
    if (gsc < 0.0) {
#pragma unroll
        for (int m = 0; m < H; ++m)
#pragma unroll
            for (int v = 0; v < kV; ++v) G[m][v] = -G[m][v];
    }
    if (row_ok) {
        float* dst = dfop + (int64_t)r * N + j0 + kV * lane;
        if (full && (N & 3) == 0 && (reinterpret_cast<uintptr_t>(dfop) & 15) == 0) {
            *reinterpret_cast<float4*>(dst) = make_float4(G[0][0], G[0][1], G[0][2], G[0][3]);
        } else {
#pragma unroll
            for (int v = 0; v < kV; ++v)
                if (kV * lane + v < nb) dst[v] = G[0][v];
        }
    }
    // box sums of G_m, m >= 2, inside the tile: each wave sums its own row
    // over the m bins of every target column (no barrier: it reads back
    // what it wrote), then each target's sum over its m rows; the zero pads
    // stand for everything outside the tile
    float* const grow = gt + rr * kGPitch + kGPad;
    static_for<2, H>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        constexpr int NR = fused_rows(m), P = stage_pitch(m);
        *reinterpret_cast<float4*>(grow + kV * lane) = make_float4(G[m - 1][0], G[m - 1][1], G[m - 1][2], G[m - 1][3]);
        // the wave reads back bins its other lanes wrote: keep the order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int jfirst = m * (j0 / m) - j0;          // first target's first bin, in (-m, 0]
        if (m > 2) __syncthreads();                    // the previous factor's row sums are read
#pragma unroll
        for (int tc = lane; tc < P + 63 - (P + 63) % 64; tc += 64) {
            if (tc < P) {
                const float* src = grow + jfirst + m * tc;
                float acc = src[0];
#pragma unroll
                for (int dc = 1; dc < m; ++dc) acc += src[dc];
                hr[(hr_top<H>() + rr) * kHPitch + tc] = acc;
            }
        }
        __syncthreads();
        const int rfirst = c + m * (src_row(r0, m, c) - c) - r0;   // first target's first row, in (-m, 0]
        float* out = part + fused_partial_offset(m, row_blocks, n_bt) + (((int64_t)rb * NR) * n_bt + bt) * P;
        for (int e = threadIdx.x; e < NR * P; e += kFThreads) {
            const int tr = e / P, tc = e - tr * P;
            const float* src = hr + (hr_top<H>() + rfirst + m * tr) * kHPitch + tc;
            float acc = src[0];
#pragma unroll
            for (int dr = 1; dr < m; ++dr) acc += src[dr * kHPitch];
            out[(int64_t)tr * n_bt * P + tc] = acc;
        }
    });
}

// Second pass of the statistic's backward: dFOP(a, b) += the tile partials
// covering (a, b) for m = 2..H (m and the tile height are compile-time
// constants).  Only points that some m >= 2 box maps to are touched: bins
// b <= (N - 1) / 2 of rows whose boxes meet the plane; each thread takes
// four consecutive bins of one row.
template <int H, int R>
__global__ __launch_bounds__(256) void k_bwd_reduce_t(float* __restrict__ dfop, const float* __restrict__ part, int T,
                                                      int N, int row_blocks, int n_bt)
{
    const int c = T / 2;
    const int half = (N - 1) / 2 + 1;             // bins with an m = 2 box
    const int nq = (half + 3) / 4;
    const int64_t total = (int64_t)T * nq;
    const bool narrow = total < ((int64_t)1 << 31);   // 32-bit index arithmetic (the usual case)
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int a = narrow ? (int)((uint32_t)e / (uint32_t)nq) : (int)(e / nq);
        const int b0 = (int)(e - (int64_t)a * nq) * 4;
        float add[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        bool any = false;
        static_for<2, H>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr int NR = fused_rows(m), P = stage_pitch(m);
            const int first = max(c + m * (a - c), 0), last = min(c + m * (a - c) + m - 1, T - 1);
            if (first > last) return;
            const float* pm = part + fused_partial_offset(m, row_blocks, n_bt);
            for (int rb = first / R; rb <= last / R; ++rb) {
                const int tr = a - src_row(rb * R, m, c);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int b = b0 + v;
                    if ((int64_t)m * b > N - 1) continue;
                    const int jb0 = m * b, jb1 = min(m * b + m - 1, N - 1);
                    for (int bt = jb0 / kTileBins; bt <= jb1 / kTileBins; ++bt) {
                        const int tc = b - (bt * kTileBins) / m;
                        add[v] += pm[(((int64_t)rb * NR + tr) * n_bt + bt) * P + tc];
                        any = true;
                    }
                }
            }
        });
        if (any) {
            float* d = dfop + (int64_t)a * N + b0;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (b0 + v < half) d[v] = d[v] + add[v];
        }
    }
}

// Log-sum-exp, level 1: block (k, i) reduces a contiguous chunk of plane k
// to a (max, sum of exp(x - max)) pair, x = HP / tau evaluated in fp64.
constexpr int kLseBlocks = 256;

__device__ __forceinline__ void lse_merge(double& M, float& S, double M2, float S2)
{
    if (S2 == 0.0f) return;
    if (S == 0.0f) { M = M2; S = S2; return; }
    if (M2 > M) { S = S * expf((float)(M - M2)) + S2; M = M2; }
    else S = S + S2 * expf((float)(M2 - M));
}

__global__ __launch_bounds__(256) void k_lse_part(const float* __restrict__ hp, int64_t plane, double inv_tau,
                                                  double* __restrict__ pm, float* __restrict__ ps)
{
    const int k = blockIdx.y;
    const int64_t chunk = (plane + gridDim.x - 1) / gridDim.x;
    const int64_t beg = blockIdx.x * chunk, end = min(plane, beg + chunk);
    const float* x = hp + (int64_t)k * plane;
    double M = 0.0;
    float S = 0.0f;
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const double xd = (double)x[e] * inv_tau;
        if (S == 0.0f) { M = xd; S = 1.0f; }
        else if (xd > M) { S = S * expf((float)(M - xd)) + 1.0f; M = xd; }
        else S += expf((float)(xd - M));
    }
    __shared__ double sm[256];
    __shared__ float ss[256];
    sm[threadIdx.x] = M;
    ss[threadIdx.x] = S;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double m1 = sm[threadIdx.x];
            float s1 = ss[threadIdx.x];
            lse_merge(m1, s1, sm[threadIdx.x + w], ss[threadIdx.x + w]);
            sm[threadIdx.x] = m1;
            ss[threadIdx.x] = s1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pm[(int64_t)k * gridDim.x + blockIdx.x] = sm[0];
        ps[(int64_t)k * gridDim.x + blockIdx.x] = ss[0];
    }
}

// Level 2: one thread per plane merges the block pairs in block order.
__global__ void k_lse_final(const double* __restrict__ pm, const float* __restrict__ ps, int H, int nblk,
                            double* __restrict__ lse)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= H) return;
    double M = 0.0;
    float S = 0.0f;
    for (int i = 0; i < nblk; ++i) lse_merge(M, S, pm[(int64_t)k * nblk + i], ps[(int64_t)k * nblk + i]);
    lse[k] = M + log((double)S);
}

// L = sum_k tau * lse[k-1], in k order (fp64).
__global__ void k_lse_loss(const double* __restrict__ lse, int H, double tau, double* __restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0;
    for (int k = 0; k < H; ++k) L += tau * lse[k];
    *loss = L;
}

// Fused statistic, level 2: one block per plane.  The blocks' pairs (max
// m_b in storage units, sum s_b of exp((x - m_b) * cd)) are merged in fp64,
// cd = inv_scale / tau: first the largest m_b, then the sum of
// s_b * exp((m_b - M) * cd); each thread takes a fixed stride of blocks and
// the threads are combined by a fixed tree (deterministic).
// lse = M * cd + log(S).
constexpr int kLseFinalThreads = 256;

__global__ __launch_bounds__(kLseFinalThreads) void k_lse_fused_final(const float* __restrict__ part, int nblk, int H,
                                                                    double cd, double* __restrict__ lse)
{
    const int k = blockIdx.x;
    __shared__ double red[kLseFinalThreads];
    double m = -__builtin_inf();
    for (int b = threadIdx.x; b < nblk; b += kLseFinalThreads) {
        const double s2 = part[((int64_t)b * H + k) * 2 + 1];
        if (s2 != 0.0) m = fmax(m, (double)part[((int64_t)b * H + k) * 2]);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kLseFinalThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double M = red[0];
    __syncthreads();
    double acc = 0.0;
    if (M != -__builtin_inf()) {
        for (int b = threadIdx.x; b < nblk; b += kLseFinalThreads) {
            const double s2 = part[((int64_t)b * H + k) * 2 + 1];
            if (s2 != 0.0) acc += s2 * exp(((double)part[((int64_t)b * H + k) * 2] - M) * cd);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kLseFinalThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lse[k] = M * cd + log(red[0]);
}

int grid_for(int64_t n, int threads, int cap)
{
    const int64_t b = (n + threads - 1) / threads;
    return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

}  // namespace

int64_t backward_partial_floats(int T, int H, int R, int64_t N)
{
    const int row_blocks = (T + R - 1) / R;
    const int64_t n_bt = (N + kTileBins - 1) / kTileBins;
    return partial_offset(H + 1, row_blocks, n_bt);
}

hipError_t launch_backward(const float* g, float* dfop, float* part, int T, int64_t N, int H, int R,
                           hipStream_t s)
{
    const int row_blocks = (T + R - 1) / R;
    const int n_bt = (int)((N + kTileBins - 1) / kTileBins);
    const int64_t tiles = (int64_t)row_blocks * n_bt;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bwd_tiles, dim3((unsigned)tiles), dim3(kGThreads), 0, s, g, dfop, part, T,
                       (int)N, H, R, row_blocks, n_bt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bwd_reduce, dim3(grid_for((int64_t)T * N, 256, 65536)), dim3(256), 0, s, dfop,
                       part, T, (int)N, H, R, row_blocks, n_bt);
    return hipGetLastError();
}

hipError_t launch_lse_backward_fused(int dtype, const void* fop, int64_t ld, int T, int64_t N, int H, float inv_scale,
                                    double tau, const double* lse, const double* gscale, float* dfop, float* part,
                                    hipStream_t s)
{
    const int row_blocks = (T + kFR - 1) / kFR;
    const int n_bt = (int)((N + kTileBins - 1) / kTileBins);
    const int64_t tiles = (int64_t)row_blocks * n_bt;
    if (tiles > 0x7fffffff || H < 1 || H > kMaxH) return hipErrorInvalidValue;
    const dim3 g((unsigned)tiles), b(kFThreads);
    const float c2 = (float)(1.4426950408889634 * (double)inv_scale / tau);   // log2(e) / (tau scale)
    bool ok = false;
    static_for<1, kMaxH>([&](auto hc) {
        constexpr int HH = decltype(hc)::value;
        if (HH != H) return;
        ok = true;
        switch (dtype) {
        case HS_DTYPE_F32:
            hipLaunchKernelGGL((k_lse_bwd_tiles<float, HH>), g, b, 0, s, fop, ld, T, (int)N, (double)inv_scale, tau, c2, lse,
                               gscale, dfop, part, row_blocks, n_bt);
            break;
        case HS_DTYPE_F16:
            hipLaunchKernelGGL((k_lse_bwd_tiles<_Float16, HH>), g, b, 0, s, fop, ld, T, (int)N, (double)inv_scale, tau, c2, lse,
                               gscale, dfop, part, row_blocks, n_bt);
            break;
        case HS_DTYPE_BF16:
            hipLaunchKernelGGL((k_lse_bwd_tiles<bf16_bits, HH>), g, b, 0, s, fop, ld, T, (int)N, (double)inv_scale, tau,
                               c2, lse, gscale, dfop, part, row_blocks, n_bt);
            break;
        default:
            ok = false;
        }
    });
    if (!ok) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t quads = (int64_t)T * (((N - 1) / 2 + 1 + 3) / 4);
    static_for<2, kMaxH>([&](auto hc) {
        constexpr int HH = decltype(hc)::value;
        if (HH == H)
            hipLaunchKernelGGL((k_bwd_reduce_t<HH, kFR>), dim3(grid_for(quads, 256, 65536)), dim3(256), 0, s, dfop,
                               part, T, (int)N, row_blocks, n_bt);
    });
    return hipGetLastError();
}

int lse_backward_tile_rows() { return kFR; }

int64_t lse_part_bytes(int H) { return (int64_t)H * kLseBlocks * (8 + 4); }

hipError_t launch_lse_reduce(const float* hp, int64_t plane, int H, double tau, void* work, double* lse,
                             hipStream_t s)
{
    double* pm = static_cast<double*>(work);
    float* ps = reinterpret_cast<float*>(pm + (int64_t)H * kLseBlocks);
    hipLaunchKernelGGL(k_lse_part, dim3(kLseBlocks, H), dim3(256), 0, s, hp, plane, 1.0 / tau, pm, ps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lse_final, dim3(1), dim3(64), 0, s, pm, ps, H, kLseBlocks, lse);
    return hipGetLastError();
}

hipError_t launch_lse_fused_final(const float* part, int nblk, int H, double inv_scale, double tau,
                                  double* lse, hipStream_t s)
{
    hipLaunchKernelGGL(k_lse_fused_final, dim3(H), dim3(kLseFinalThreads), 0, s, part, nblk, H, inv_scale / tau, lse);
    return hipGetLastError();
}

hipError_t launch_lse_loss(const double* lse, int H, double tau, double* loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_lse_loss, dim3(1), dim3(64), 0, s, lse, H, tau, loss);
    return hipGetLastError();
}


}  // namespace hsk
