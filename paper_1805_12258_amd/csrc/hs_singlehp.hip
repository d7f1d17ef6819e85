// SingleHP baseline (Sec. IV-B, kernel of Sec. V-A): harmonic planes formed
// one after another through memory, HP_k = HP_{k-1} + SP_k (Eq. 2), each
// plane written out and read back for the next, and thresholded as it is
// formed.  It is the method the paper's MultipleHP improves on; here it
// serves as the measured reference point for the fused kernels on the same
// GPU.  The sums are the fused kernels' (same order, fp32), so planes and
// candidate sets are bitwise the same.  Two forms, as evaluated in Sec. V-A:
// multiple launches (one per plane) and a single launch that walks the
// planes in order inside the kernel.  HP_k at a point needs only HP_{k-1}
// at the same point, and every thread keeps the same points for every
// plane, so the single launch needs no grid-wide barrier between planes: a
// thread reads back the plane values it wrote itself.
#include <hip/hip_runtime.h>

#include "hs_internal.h"

namespace hsk {

namespace {

constexpr int kSThreads = 256;

// Plane k: each thread forms 4 consecutive bins of one row.  The loop bound
// is uniform per block so every wave votes on every step.
__device__ __forceinline__ void single_plane_pass(const float* __restrict__ fop, int64_t ld, int T, int N, int c,
                                                  int k, const float* prev, float* cur,
                                                  const float* __restrict__ ta, hs_cand* __restrict__ out,
                                                  int64_t cap, unsigned long long* __restrict__ counts, int s_row,
                                                  int s_bin, int H)
{
    const int64_t nq = (N + 3) / 4;
    const int64_t total = (int64_t)T * nq;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * kSThreads; base < total; base += (int64_t)gridDim.x * kSThreads) {
        const int64_t e = base + threadIdx.x;
        const bool live = e < total;
        int r = 0, j0 = 0;
        float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        bool in[4] = {false, false, false, false};
        if (live) {
            r = (int)(e / nq);
            j0 = (int)(e - (int64_t)r * nq) * 4;
            const int sr = floordiv32(r - c, k) + c;      // source row of Eq. 1
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u;
                in[u] = j < N;
                if (in[u]) {
                    v[u] = k == 1 ? fop[(int64_t)r * ld + j]
                                  : prev[(int64_t)r * N + j] + fop[(int64_t)sr * ld + j / k];
                    cur[(int64_t)r * N + j] = v[u];
                }
            }
        }
        const float t = live ? ta[(int64_t)(k - 1) * T + r] : 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool hit = live && in[u] && v[u] > t;
            const uint64_t mk = __builtin_amdgcn_ballot_w64(hit);
            if (mk == 0) continue;
            const unsigned long long n = __builtin_popcountll(mk);
            unsigned long long first = 0;
            if (lane == 0) {
                first = atomicAdd(&counts[H], n);
                atomicAdd(&counts[k - 1], n);
            }
            first = __shfl(first, 0, 64);
            if (hit) {
                const uint64_t pos = first + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
                if ((int64_t)pos < cap) {
                    hs_cand h;
                    h.idx = ((uint32_t)r << s_row) | ((uint32_t)(k - 1) << s_bin) | (uint32_t)(j0 + u);
                    h.power = v[u];
                    out[pos] = h;
                }
            }
        }
    }
}

__global__ __launch_bounds__(kSThreads) void k_single_plane(const float* __restrict__ fop, int64_t ld, int T,
                                                           int N, int c, int k, const float* prev, float* cur,
                                                           const float* __restrict__ ta,
                                                           hs_cand* __restrict__ out, int64_t cap,
                                                           unsigned long long* __restrict__ counts, int s_row,
                                                           int s_bin, int H)
{
    single_plane_pass(fop, ld, T, N, c, k, prev, cur, ta, out, cap, counts, s_row, s_bin, H);
}

// The single launch: planes 1..H in order, ping-ponging between the two
// plane buffers as the multiple launches do.
__global__ __launch_bounds__(kSThreads) void k_single_all(const float* __restrict__ fop, int64_t ld, int T, int N,
                                                         int c, float* buf0, float* buf1,
                                                         const float* __restrict__ ta, hs_cand* __restrict__ out,
                                                         int64_t cap, unsigned long long* __restrict__ counts,
                                                         int s_row, int s_bin, int H)
{
    for (int k = 1; k <= H; ++k) {
        float* prev = (k & 1) ? buf1 : buf0;
        float* cur = (k & 1) ? buf0 : buf1;
        single_plane_pass(fop, ld, T, N, c, k, prev, cur, ta, out, cap, counts, s_row, s_bin, H);
    }
}

int single_grid(int T, int N)
{
    const int64_t quads = (int64_t)T * ((N + 3) / 4);
    const int64_t want = (quads + kSThreads - 1) / kSThreads;
    return (int)(want < 8192 ? (want < 1 ? 1 : want) : 8192);
}

}  // namespace

// H launches, one per plane, through two plane buffers (`work`: 2 x T x N
// fp32), or one launch (single_launch) through the same buffers.  counts
// must be cleared by the caller.
hipError_t launch_singlehp(const float* fop, int64_t ld, int T, int N, int H, const float* ta, hs_cand* out,
                           int64_t cap, unsigned long long* counts, int s_row, int s_bin, float* work,
                           bool single_launch, hipStream_t s)
{
    const int64_t plane = (int64_t)T * N;
    const int grid = single_grid(T, N);
    float* buf[2] = {work, work + ((plane + 63) & ~(int64_t)63)};
    if (single_launch) {
        hipLaunchKernelGGL(k_single_all, dim3(grid), dim3(kSThreads), 0, s, fop, ld, T, N, T / 2, buf[0], buf[1], ta,
                           out, cap, counts, s_row, s_bin, H);
        return hipGetLastError();
    }
    for (int k = 1; k <= H; ++k) {
        // plane k reads buf[k & 1] and writes buf[(k + 1) & 1], as in the single launch
        hipLaunchKernelGGL(k_single_plane, dim3(grid), dim3(kSThreads), 0, s, fop, ld, T, N, T / 2, k,
                           buf[k & 1], buf[(k + 1) & 1], ta, out, cap, counts, s_row, s_bin, H);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hsk
