/*
 * Harmonic-summing ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU implementation of the harmonic-summing
 * module of Wang, Thiagaraj & Sinnen, "Harmonic-summing Module of SKA on FPGA
 * -- Optimising the Irregular Memory Accesses" (arXiv:1805.12258).  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this file.  It shares no code with the GPU library and includes none of
 * its headers.
 *
 * Conventions (the paper's notation):
 *   FOP  : N_temp rows (templates) x N_chan bins of single-precision power,
 *          row-major with leading dimension ld >= N_chan (Sec. III).
 *   rows : storage row r in [0, T) holds template index i = r - T/2 (integer
 *          division).  For odd T this is the paper's range
 *          i in [-(T-1)/2, (T-1)/2] (Sec. III, Eq. 1); for even T it is
 *          [-T/2, T/2-1], the convention under which the touch statistics of
 *          the 64 x 2^12 example in Sec. IV-A come out as printed.
 *   SP_m(i,j) = FOP(floor(i/m), floor(j/m))           (Sec. III, Eq. 1)
 *   HP_1 = FOP,  HP_k = HP_{k-1} + SP_k, k = 2..H    (Sec. III, Eq. 2)
 *   candidate: HP_k(i,j) > TA(k, i)                  (Sec. III, detection)
 *   fractional variant (the incoherent-sum reading of "the k-th harmonic
 *   plane sums the FOP at the fractions m/k of each point"; not Eq. 1-2):
 *   HPF_k(i,j) = sum_{m=1..k} FOP(floor(m*i/k), floor(m*j/k)), m in order
 *   packed word CL1 = F * 2^(sk+sj) + (k-1) * 2^sj + B, where F is the
 *   storage row, B the bin, sj = ceil(log2 N), sk = ceil(log2 H); for the
 *   specification (85, 8, 2^21) this is the paper's F*2^24 + H*2^21 + B
 *   (Sec. III, candidate list format).  CL2 is the fp32 power.
 *
 * Every sum is formed in the order of Eq. 2 (m = 1, 2, ..., k), each partial
 * sum rounded to the working precision.  Build without -ffast-math and with
 * -ffp-contract=off.
 *
 * Parity pins live in tests/test_oracle_*.py: brute force per point, integer
 * planes, loop-order freedom (Sec. III, Algorithms 1 and 2), the k = 1
 * identity, monotonicity, injected harmonic sums, the touch statistics and
 * staging counts printed in Sec. IV, the packing formula, finite differences
 * for the transpose.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* floor(a / b) for b > 0 and any sign of a (Eq. 1 uses the floor, also for
 * the negative template indices). */
static int64_t fdiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if (q * b > a) q -= 1;
    return q;
}

/* Smallest s with 2^s >= x (x >= 1): the "ceil(log2(*))" field width of the
 * candidate word (Sec. III). */
static int ceil_log2(int64_t x)
{
    int s = 0;
    while (((int64_t)1 << s) < x) s++;
    return s;
}

int hso_field_bits(int64_t T, int64_t N, int H, int* s_row, int* s_k, int* s_bin)
{
    if (T < 1 || N < 1 || H < 1) return -1;
    *s_bin = ceil_log2(N);
    *s_k = ceil_log2(H);
    *s_row = ceil_log2(T);
    return (*s_bin + *s_k + *s_row) <= 32 ? 0 : -2;
}

uint32_t hso_pack(int64_t r, int k, int64_t j, int64_t N, int H)
{
    int sj = ceil_log2(N), sk = ceil_log2(H);
    return (uint32_t)(((uint64_t)r << (sk + sj)) | ((uint64_t)(k - 1) << sj) | (uint64_t)j);
}

/* Source storage row of stretch factor m for storage row r (Eq. 1). */
static int64_t src_row(int64_t r, int64_t m, int64_t T)
{
    int64_t c = T / 2;
    return fdiv(r - c, m) + c;
}

/* ---------------------------------------------------------------------- */
/* All H harmonic planes in fp32, Algorithm 1 loop order (k, i, j).        */
/* hp is [H][T][N] (leading dimension N).                                  */
/* ---------------------------------------------------------------------- */
int hso_sum_f32(const float* fop, int64_t T, int64_t N, int64_t ld, int H, float* hp)
{
    if (T < 1 || N < 1 || H < 1 || ld < N) return -1;
    for (int k = 1; k <= H; k++) {
        float* cur = hp + (int64_t)(k - 1) * T * N;
        const float* prev = hp + (int64_t)(k - 2) * T * N;
        for (int64_t r = 0; r < T; r++) {
            int64_t rs = src_row(r, k, T);
            for (int64_t j = 0; j < N; j++) {
                float sp = fop[rs * ld + fdiv(j, k)];          /* SP_k(i,j) */
                cur[r * N + j] = (k == 1) ? sp : prev[r * N + j] + sp;
            }
        }
    }
    return 0;
}

/* Same planes in fp64 from fp64 input (accuracy truth).  Rows are
 * independent within a plane: nthreads OpenMP threads share them. */
int hso_sum_f64(const double* fop, int64_t T, int64_t N, int64_t ld, int H, double* hp, int nthreads)
{
    if (T < 1 || N < 1 || H < 1 || ld < N) return -1;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#else
    (void)nthreads;
#endif
    for (int k = 1; k <= H; k++) {
        double* cur = hp + (int64_t)(k - 1) * T * N;
        const double* prev = hp + (int64_t)(k - 2) * T * N;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
        for (int64_t r = 0; r < T; r++) {
            int64_t rs = src_row(r, k, T);
            for (int64_t j = 0; j < N; j++) {
                double sp = fop[rs * ld + fdiv(j, k)];
                cur[r * N + j] = (k == 1) ? sp : prev[r * N + j] + sp;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Harmonic planes plus threshold detection, Algorithm 1 loop order.        */
/* One working plane holds HP_{k-1} and is overwritten in place by HP_k    */
/* (each point of HP_k depends only on the same point of HP_{k-1}).         */
/*                                                                          */
/* ta     : [H][T] thresholds (one per row per plane, Sec. III).            */
/* scale  : the FOP holds x*scale; the test is HP_k > ta*scale and the      */
/*          reported power is HP_k/scale (scale must be a power of two, so  */
/*          both are exact).  Use 1 for plain fp32 input.                   */
/* idx,pw : candidate words (CL1) and powers (CL2), in Algorithm 1 order    */
/*          (k, then row, then bin); at most cap are written.               */
/* counts : [H+1] true number of candidates per plane, then the total.      */
/* nthreads: OpenMP threads over rows (1 = the single-core baseline).       */
/* Returns 0, or -3 if the total exceeds cap (counts are still exact).      */
/* ---------------------------------------------------------------------- */
int hso_detect_f32(const float* fop, int64_t T, int64_t N, int64_t ld, int H,
                   const float* ta, float scale, uint32_t* idx, float* pw,
                   int64_t cap, int64_t* counts, int nthreads)
{
    if (T < 1 || N < 1 || H < 1 || ld < N || !(scale > 0.0f)) return -1;
    int s_row, s_k, s_bin;
    if (hso_field_bits(T, N, H, &s_row, &s_k, &s_bin) != 0) return -2;
    float* cur = (float*)malloc(sizeof(float) * (size_t)(T * N));
    int64_t* rowcnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T + 1));
    if (!cur || !rowcnt) { free(cur); free(rowcnt); return -4; }
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#else
    (void)nthreads;
#endif
    int64_t total = 0;
    for (int k = 1; k <= H; k++) {
        /* Pass 1: HP_k = HP_{k-1} + SP_k for every row; count candidates. */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
        for (int64_t r = 0; r < T; r++) {
            int64_t rs = src_row(r, k, T);
            float thr = ta[(int64_t)(k - 1) * T + r] * scale;
            int64_t n = 0;
            float* row = cur + r * N;
            for (int64_t j = 0; j < N; j++) {
                float sp = fop[rs * ld + fdiv(j, k)];
                float v = (k == 1) ? sp : row[j] + sp;
                row[j] = v;
                n += (v > thr);
            }
            rowcnt[r] = n;
        }
        /* Row offsets in Algorithm 1 order. */
        int64_t run = total;
        for (int64_t r = 0; r < T; r++) { int64_t n = rowcnt[r]; rowcnt[r] = run; run += n; }
        rowcnt[T] = run;
        counts[k - 1] = run - total;
        /* Pass 2: write this plane's candidates at their offsets. */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
        for (int64_t r = 0; r < T; r++) {
            float thr = ta[(int64_t)(k - 1) * T + r] * scale;
            int64_t o = rowcnt[r];
            const float* row = cur + r * N;
            uint32_t hi = (uint32_t)(((uint64_t)r << (s_k + s_bin)) | ((uint64_t)(k - 1) << s_bin));
            for (int64_t j = 0; j < N; j++) {
                float v = row[j];
                if (v > thr) {
                    if (o < cap) { idx[o] = hi | (uint32_t)j; pw[o] = v / scale; }
                    o++;
                }
            }
        }
        total = run;
    }
    counts[H] = total;
    free(cur);
    free(rowcnt);
    return total > cap ? -3 : 0;
}

/* ---------------------------------------------------------------------- */
/* Transpose of the plane map (vector-Jacobian product), fp64.              */
/* Given cotangents g_k = dL/dHP_k ([H][T][N]), the derivative of L with    */
/* respect to each FOP point, written out from Eq. 1-2: HP_k(i,j) holds     */
/* FOP(floor(i/m), floor(j/m)) once for every m <= k, so each g_k(i,j) is   */
/* added to those k source points.  Explicit loop over (k, i, j, m).        */
/* dfop is [T][N] and is overwritten.                                       */
/* ---------------------------------------------------------------------- */
int hso_vjp_f64(const double* g, int64_t T, int64_t N, int H, double* dfop)
{
    if (T < 1 || N < 1 || H < 1) return -1;
    memset(dfop, 0, sizeof(double) * (size_t)(T * N));
    for (int k = 1; k <= H; k++) {
        const double* gk = g + (int64_t)(k - 1) * T * N;
        for (int64_t r = 0; r < T; r++)
            for (int64_t j = 0; j < N; j++) {
                double v = gk[r * N + j];
                if (v == 0.0) continue;
                for (int m = 1; m <= k; m++)
                    dfop[src_row(r, m, T) * N + fdiv(j, m)] += v;
            }
    }
    return 0;
}

/* Number of times each FOP point is read when every point of HP_k is formed
 * for the planes k listed in kmask (bit k-1): the per-point "touching
 * frequency" of Sec. IV-A.  Equal to the transpose above applied to
 * g_k = 1 for the selected planes, counted in integers.  touch is [T][N]. */
int hso_touch_counts(int64_t T, int64_t N, int H, uint32_t kmask, int64_t* touch)
{
    if (T < 1 || N < 1 || H < 1) return -1;
    memset(touch, 0, sizeof(int64_t) * (size_t)(T * N));
    for (int k = 1; k <= H; k++) {
        if (!(kmask >> (k - 1) & 1u)) continue;
        for (int64_t r = 0; r < T; r++)
            for (int64_t j = 0; j < N; j++)
                for (int m = 1; m <= k; m++)
                    touch[src_row(r, m, T) * N + fdiv(j, m)] += 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Fractional variant: HPF_k(i,j) = sum_{m=1..k} FOP(floor(m i/k),          */
/* floor(m j/k)), each plane on its own (no recursion over k: the source    */
/* points of plane k are the fractions m/k of (i, j), m = 1..k), terms      */
/* added in the order m = 1, 2, ..., k with each partial sum rounded.       */
/* Template indices are signed (i = r - T/2) and divided with the floor.    */
/* ---------------------------------------------------------------------- */
static int64_t frac_row(int64_t r, int64_t m, int64_t k, int64_t T)
{
    int64_t c = T / 2;
    return fdiv(m * (r - c), k) + c;
}

static float frac_point_f32(const float* fop, int64_t ld, int64_t T, int64_t r, int64_t j, int k)
{
    float v = 0.0f;
    for (int m = 1; m <= k; m++) {
        float x = fop[frac_row(r, m, k, T) * ld + fdiv((int64_t)m * j, k)];
        v = (m == 1) ? x : v + x;
    }
    return v;
}

int hso_sum_frac_f32(const float* fop, int64_t T, int64_t N, int64_t ld, int H, float* hp)
{
    if (T < 1 || N < 1 || H < 1 || ld < N) return -1;
    for (int k = 1; k <= H; k++)
        for (int64_t r = 0; r < T; r++)
            for (int64_t j = 0; j < N; j++)
                hp[((int64_t)(k - 1) * T + r) * N + j] = frac_point_f32(fop, ld, T, r, j, k);
    return 0;
}

int hso_sum_frac_f64(const double* fop, int64_t T, int64_t N, int64_t ld, int H, double* hp)
{
    if (T < 1 || N < 1 || H < 1 || ld < N) return -1;
    for (int k = 1; k <= H; k++)
        for (int64_t r = 0; r < T; r++)
            for (int64_t j = 0; j < N; j++) {
                double v = 0.0;
                for (int m = 1; m <= k; m++) {
                    double x = fop[frac_row(r, m, k, T) * ld + fdiv((int64_t)m * j, k)];
                    v = (m == 1) ? x : v + x;
                }
                hp[((int64_t)(k - 1) * T + r) * N + j] = v;
            }
    return 0;
}

/* Detection on the fractional planes: the same test, word and order as
 * hso_detect_f32 (plane k, then row, then bin).  Rows are independent: a
 * first pass counts each row's candidates (OpenMP over rows), the second
 * forms the values again and writes them at the rows' offsets. */
int hso_detect_frac_f32(const float* fop, int64_t T, int64_t N, int64_t ld, int H,
                        const float* ta, float scale, uint32_t* idx, float* pw,
                        int64_t cap, int64_t* counts, int nthreads)
{
    if (T < 1 || N < 1 || H < 1 || ld < N || !(scale > 0.0f)) return -1;
    int s_row, s_k, s_bin;
    if (hso_field_bits(T, N, H, &s_row, &s_k, &s_bin) != 0) return -2;
    int64_t* rowoff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T * H + 1));
    if (!rowoff) return -4;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#else
    (void)nthreads;
#endif
    for (int64_t e = 0; e < T * H; e++) {
        int k = (int)(e / T) + 1;
        int64_t r = e % T;
        float thr = ta[(int64_t)(k - 1) * T + r] * scale;
        int64_t n = 0;
        for (int64_t j = 0; j < N; j++) n += (frac_point_f32(fop, ld, T, r, j, k) > thr);
        rowoff[e] = n;
    }
    int64_t run = 0;
    for (int k = 1; k <= H; k++) {
        int64_t start = run;
        for (int64_t r = 0; r < T; r++) {
            int64_t n = rowoff[(int64_t)(k - 1) * T + r];
            rowoff[(int64_t)(k - 1) * T + r] = run;
            run += n;
        }
        counts[k - 1] = run - start;
    }
    counts[H] = run;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t e = 0; e < T * H; e++) {
        int k = (int)(e / T) + 1;
        int64_t r = e % T;
        float thr = ta[(int64_t)(k - 1) * T + r] * scale;
        uint32_t hi = (uint32_t)(((uint64_t)r << (s_k + s_bin)) | ((uint64_t)(k - 1) << s_bin));
        int64_t o = rowoff[e];
        for (int64_t j = 0; j < N; j++) {
            float v = frac_point_f32(fop, ld, T, r, j, k);
            if (v > thr) {
                if (o < cap) { idx[o] = hi | (uint32_t)j; pw[o] = v / scale; }
                o++;
            }
        }
    }
    free(rowoff);
    return run > cap ? -3 : 0;
}
