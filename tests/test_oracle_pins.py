"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle with
a retyped copy of its own loop: they use brute force per point, exact integer
planes, closed forms, values printed in the paper, or library routines.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """A fixture of values printed in the paper (each file cites its passage)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def rand_exp(T, N, seed):
    rng = np.random.default_rng(seed)
    return rng.exponential(1.0, size=(T, N)).astype(np.float32)


# --- P1: brute force per point ------------------------------------------------

@pytest.mark.parametrize("T,N", [(5, 64), (9, 257), (21, 1024), (64, 300)])
def test_integer_planes_exact(T, N):
    """Integer-valued FOP: every partial sum is exact in fp32, so the fp32
    oracle equals the fp64 per-point definition bit for bit (Eq. 1-2)."""
    rng = np.random.default_rng(T * 1000 + N)
    fop = rng.integers(0, 16, size=(T, N)).astype(np.float32)
    hp = oracle.sum_f32(fop, 8)
    ref = brute.planes_f64(fop, 8)
    assert np.array_equal(hp.astype(np.float64), ref)


@pytest.mark.parametrize("T,N,H", [(5, 64, 8), (21, 1024, 8), (9, 333, 16), (1, 50, 3)])
def test_random_planes_within_summation_bound(T, N, H):
    """Exp(1) FOP: the fp32 sum of k non-negative terms lies within
    (k-1) * 2^-24 * S (first order) of the fp64 definition."""
    fop = rand_exp(T, N, 11)
    hp = oracle.sum_f32(fop, H).astype(np.float64)
    ref = brute.planes_f64(fop, H)
    for k in range(1, H + 1):
        bound = (k - 1) * 2.0 ** -24 * ref[k - 1] * (1 + 1e-6)
        assert np.all(np.abs(hp[k - 1] - ref[k - 1]) <= bound)


def test_point_definition():
    """A handful of single points evaluated by a plain loop over m."""
    fop = rand_exp(21, 512, 3)
    hp64 = oracle.sum_f64(fop, 8)
    for (k, r, j) in [(1, 0, 0), (8, 0, 511), (8, 20, 511), (5, 3, 17), (3, 10, 2), (8, 15, 300)]:
        assert hp64[k - 1, r, j] == pytest.approx(brute.point_f64(fop, k, r, j), rel=1e-15)


def test_example_point_sources():
    """HP_8 at template 60, bin 1000 reads the 8 points (60,1000), (30,500),
    (20,333), (15,250), (12,200), (10,166), (8,142), (7,125) (Sec. IV-A)."""
    i, j = 60, 1000
    got = [(i // m, j // m) for m in range(1, 9)]
    assert got == [(60, 1000), (30, 500), (20, 333), (15, 250), (12, 200), (10, 166),
                   (8, 142), (7, 125)]
    # the oracle reads exactly these: put a one-hot at each and check HP_8
    T = 2 * 60 + 1
    c = T // 2
    for (a, b) in got:
        fop = np.zeros((T, 1001), dtype=np.float32)
        fop[a + c, b] = 1.0
        assert oracle.sum_f32(fop, 8)[7, i + c, j] == 1.0
    fop = np.zeros((T, 1001), dtype=np.float32)
    for (a, b) in got:
        fop[a + c, b] = 1.0
    assert oracle.sum_f32(fop, 8)[7, i + c, j] == 8.0


# --- P2: loop-order freedom (Algorithms 1 and 2) -------------------------------

@pytest.mark.parametrize("T,N,H", [(5, 64, 8), (7, 50, 5), (4, 40, 6)])
def test_algorithm2_order_bitwise(T, N, H):
    fop = rand_exp(T, N, T + N)
    assert np.array_equal(oracle.sum_f32(fop, H), brute.planes_alg2_f32(fop, H))


# --- P3 / P4: k = 1 identity and monotonicity -----------------------------------

def test_k1_identity_and_detection():
    fop = rand_exp(21, 4096, 5)
    ta = synth.thresholds(8, 21)
    hp = oracle.sum_f32(fop, 8)
    assert np.array_equal(hp[0], fop)
    idx, pw, counts = oracle.detect_f32(fop, 8, ta)
    r, k, j = oracle.unpack(idx, 4096, 8)
    sel = k == 1
    want = np.argwhere(fop > ta[0][:, None])
    got = np.stack([r[sel], j[sel]], axis=1)
    assert np.array_equal(got, want)            # Algorithm 1 order: row, then bin
    assert np.array_equal(pw[sel], fop[fop > ta[0][:, None]])


def test_monotone_in_k():
    fop = rand_exp(21, 2048, 6)
    hp = oracle.sum_f32(fop, 16)
    assert np.all(np.diff(hp, axis=0) >= 0)


# --- P5: injected harmonics, hand sums -----------------------------------------

def sigma(n):
    return sum(d for d in range(1, n + 1) if n % d == 0)


@pytest.mark.parametrize("z0", [-1, 0, 1])
def test_injected_harmonic_sums(z0):
    """Noise-free plane with 20/n at (n*z0, n*f0): HP_K(K*z0, K*f0) equals
    20*sigma(K)/K, because only the stretch factors m dividing K land on a
    harmonic cell (f0 > H keeps the others off every cell)."""
    T, N, H, f0 = 21, 4096, 8, 97
    fop = np.zeros((T, N), dtype=np.float32)
    synth.inject(fop, [(z0, f0, 20.0, 8)])
    hp = oracle.sum_f32(fop, H).astype(np.float64)
    c = T // 2
    expect = [20.0, 30.0, 80.0 / 3, 35.0, 24.0, 40.0, 160.0 / 7, 37.5]
    for K in range(1, 9):
        assert 20.0 * sigma(K) / K == pytest.approx(expect[K - 1])
        assert hp[K - 1, K * z0 + c, K * f0] == pytest.approx(expect[K - 1], rel=1e-6)


def test_injected_on_noise_matches_hand_sum():
    """Tiny workload: at each signal's K-th harmonic cell, the fp64 plane equals
    the noise already at the K source cells plus the injected 20/n terms."""
    fop = synth.make_tiny().numpy()
    hp = oracle.sum_f64(fop, 8)
    c = fop.shape[0] // 2
    for (z0, f0, p0, nh) in synth.tiny_signals():
        for K in range(1, 9):
            i, j = K * z0, K * f0
            hand = sum(float(fop[(i // m) + c, j // m]) for m in range(1, K + 1))
            assert hp[K - 1, i + c, j] == pytest.approx(hand, rel=1e-12)
            assert hand >= 20.0 * sigma(K) / K * (1 - 1e-6)


# --- P6: touch statistics printed in Sec. IV-A ---------------------------------

TOUCH = golden("touch_map_64x4096.json")


@pytest.fixture(scope="module")
def touch64():
    g = TOUCH
    return oracle.touch_counts(g["n_temp"], g["n_chan"], g["n_hp"], [g["n_hp"]])


def test_touch_max_204(touch64):
    """Each point of the deep red area is touched 204 times (= sum m^2)."""
    H = TOUCH["n_hp"]
    assert touch64.max() == TOUCH["max_touches"] == sum(m * m for m in range(1, H + 1))
    assert touch64.sum() == H * TOUCH["n_temp"] * TOUCH["n_chan"]


def test_touch_zoom_share(touch64):
    """The 16 x 2^10 high-touch area holds 73.4 % of all touches."""
    c, h = TOUCH["n_temp"] // 2, TOUCH["zoom_rows"] // 2
    share = touch64[c - h:c + h, :TOUCH["zoom_bins"]].sum() / touch64.sum()
    assert round(share * 100, 1) == TOUCH["zoom_share_percent"]


def test_touch_deep_red_share(touch64):
    """Points touched 204 times: 1.56 % of the plane (printed as 1.7 %, read
    off a colour map)."""
    share = (touch64 == TOUCH["max_touches"]).mean() * 100
    assert TOUCH["deep_red_share_percent"] - 0.2 <= share <= TOUCH["deep_red_share_percent"]


def test_touch_cumulative_shares(touch64):
    """2.2 % of the points carry about 50 % of the touches, 25 % carry 90 %."""
    g = golden("preload_shares.json")
    s = np.sort(touch64.ravel())[::-1]
    cs = np.cumsum(s) / s.sum()
    f50 = (np.searchsorted(cs, g["touch_share_of_first_half_percent"] / 100) + 1) / s.size
    f90 = (np.searchsorted(cs, 0.9) + 1) / s.size
    assert round(f50 * 100, 1) == g["points_percent_for_half_of_touches"]
    assert abs(f90 * 100 - g["points_percent_for_90_percent"]) <= 2


def test_touch_equals_transpose_with_unit_cotangent(touch64):
    """The touch map is the transpose applied to g_8 = 1, g_k<8 = 0."""
    T, N = 64, 1 << 12
    g = np.zeros((8, T, N))
    g[7] = 1.0
    assert np.array_equal(oracle.vjp_f64(g), touch64.astype(np.float64))


# --- P7: staging counts (source rows / columns per work group, Sec. IV-C) ------

def needed_rows(rows_i, m):
    return len(np.unique(np.asarray(rows_i) // m))


def test_one_column_bound_240():
    """Needed points for one column of all 8 planes: the bound
    2*sum ceil((T-1)/(2i)) + H = 240, and the exact count 237 under Eq. 1."""
    T, H = 85, 8
    bound = 2 * sum(math.ceil((T - 1) / (2 * i)) for i in range(1, H + 1)) + H
    assert bound == 240
    i = brute.template_index(T)
    exact = sum(needed_rows(i, m) for m in range(1, H + 1))
    assert exact == 237 <= bound


def max_cols(ncol, m, aligned):
    starts = range(0, 840 * ncol, ncol) if aligned else range(0, 840)
    return max(len(set((j0 + t) // m for t in range(ncol))) for j0 in starts)


def test_loaded_points_table_unoptimised():
    """N_lpoints/cc of the unoptimised reordered kernel for the half FOP
    (template rows 1..42), column-aligned work groups: the printed table rows
    (3,6,12,23), (2,4,8,15), (2,4,7,13), (2,4,7,13) for 1, 4, 16, 64 columns."""
    rows_i = np.arange(1, 43)
    printed = {int(k): tuple(v) for k, v in golden("staging_counts.json")["loaded_points_unoptimised"].items()}
    for ncol, row in printed.items():
        total = sum(needed_rows(rows_i, m) * max_cols(ncol, m, True) for m in range(1, 9))
        got = tuple(math.ceil(total * p / (ncol * 42)) for p in (1, 2, 4, 8))
        assert got == row, (ncol, got)


def test_average_points_per_column_16():
    """Sixteen columns per work group need 141.4 points per column on average
    (printed 141.5, i.e. 1.66x the 85-row FOP), counting 2*ceil(42/m)+1 rows
    and the worst-case column span of each stretch factor."""
    g = golden("staging_counts.json")
    ncol = g["rfop_columns"]
    tot = sum((2 * math.ceil(42 / m) + 1) * max_cols(ncol, m, False) for m in range(1, 9))
    avg = tot / ncol
    assert abs(avg - g["rfop_avg_points_per_column"]) < 0.1
    assert round(avg / g["n_temp"], 2) == g["rfop_size_ratio"]


# --- P8: detection statistics on pure noise -------------------------------------

def test_noise_candidate_counts():
    """Pure Exp(1) noise: HP_k is a sum of k independent Exp(1) values away
    from the first rows/bins, so count_k ~ T*N*P(Gamma(k,1) > T_k)."""
    from scipy.stats import gamma
    T, N, H = 21, 1 << 16, 8
    fop = synth.noise(T, N, 1).numpy()
    ta = synth.thresholds(H, T)
    _, _, counts = oracle.detect_f32(fop, H, ta, nthreads=4)
    for k in range(1, H + 1):
        lam = T * N * gamma.sf(float(ta[k - 1, 0]), k)
        assert abs(counts[k - 1] - lam) <= 5 * math.sqrt(lam) + 5, (k, counts[k - 1], lam)
    assert counts[H] == counts[:H].sum()


def test_detect_matches_thresholded_planes():
    """Candidates = {HP_k > TA(k,row)} over the fp32 planes, strict '>'."""
    fop = rand_exp(21, 3000, 9)
    ta = synth.thresholds(8, 21).copy()
    ta[3, 5] = 1e30          # one row switched off
    ta[0, 7] = -1.0          # one row fully on
    hp = oracle.sum_f32(fop, 8)
    k, r, j, p = brute.candidates_from_planes(hp, ta)
    idx, pw, counts = oracle.detect_f32(fop, 8, ta, nthreads=3)
    rr, kk, jj = oracle.unpack(idx, 3000, 8)
    got = np.lexsort((jj, rr, kk))
    want = np.lexsort((j, r, k))
    assert np.array_equal(kk[got], k[want]) and np.array_equal(rr[got], r[want])
    assert np.array_equal(jj[got], j[want]) and np.array_equal(pw[got], p[want])
    assert counts[7 - 1 + 1] == (hp[7] > ta[7][:, None]).sum()
    # strict comparison: a value equal to its threshold is not a candidate
    fop2 = np.full((3, 8), 7.0, dtype=np.float32)
    ta2 = np.full((1, 3), 7.0, dtype=np.float32)
    assert oracle.detect_f32(fop2, 1, ta2)[2][1] == 0


def test_detect_scale_and_capacity():
    """Scaled storage (x*s, s a power of two): same candidate set, powers /s.
    Capacity: only the first cap entries are written, counts stay exact."""
    fop = rand_exp(9, 2000, 10)
    ta = synth.thresholds(4, 9)
    idx, pw, counts = oracle.detect_f32(fop, 4, ta)
    idx2, pw2, counts2 = oracle.detect_f32(fop * np.float32(0.125), 4, ta, scale=0.125)
    assert np.array_equal(idx, idx2) and np.array_equal(pw, pw2)
    assert np.array_equal(counts, counts2)
    idx3, pw3, counts3 = oracle.detect_f32(fop, 4, ta, cap=10)
    assert np.array_equal(counts3, counts) and len(idx3) == 10
    assert np.array_equal(idx3, idx[:10])


def test_tiny_workload_detects_all_injected_fundamentals():
    """Each tiny-workload signal crosses every plane's threshold at its K-th
    harmonic cell (20*sigma(K)/K > T_K for K = 1..8, plus non-negative noise)."""
    fop = synth.make_tiny().numpy()
    ta = synth.thresholds(8, fop.shape[0])
    idx, pw, counts = oracle.detect_f32(fop, 8, ta, nthreads=4)
    keys = set(int(x) for x in idx)
    c = fop.shape[0] // 2
    for (z0, f0, _, _) in synth.tiny_signals():
        for K in range(1, 9):
            assert oracle.pack(K * z0 + c, K, K * f0, fop.shape[1], 8) in keys


# --- P9: packing ------------------------------------------------------------------

def test_packing_paper_formula():
    """CL1 = F*2^24 + H*2^21 + B for 85 templates, 8 planes, 2^21 bins, with the
    plane field holding k-1 (3 bits for 8 planes)."""
    g = golden("candidate_word.json")
    N, H = g["n_chan"], g["n_hp"]
    assert oracle.field_bits(g["n_temp"], N, H) == (7, 3, 21)
    for (F, k, B) in [(0, 1, 0), (84, 8, 2 ** 21 - 1), (42, 3, 12345), (1, 2, 1)]:
        w = oracle.pack(F, k, B, N, H)
        assert w == F * 2 ** g["shift_template"] + (k - 1) * 2 ** g["shift_plane"] + B
        r, kk, j = oracle.unpack(np.array([w], dtype=np.uint32), N, H)
        assert (r[0], kk[0], j[0]) == (F, k, B)
    assert oracle.pack(84, 8, 2 ** 21 - 1, N, H) == 0x54FFFFFF
    # 16 planes: 4 plane bits, row field at bit 25, still 32 bits for 85 rows
    assert oracle.field_bits(85, N, 16) == (7, 4, 21)
    assert oracle.pack(84, 16, 2 ** 21 - 1, N, 16) == (84 << 25) | (15 << 21) | (2 ** 21 - 1)
    with pytest.raises(ValueError):
        oracle.field_bits(255, 1 << 22, 16)


# --- transpose and log-sum-exp -------------------------------------------------------

def test_vjp_scatter_equals_boxsum():
    rng = np.random.default_rng(4)
    for (H, T, N) in [(8, 21, 300), (16, 9, 100), (3, 64, 50), (1, 5, 7)]:
        g = rng.standard_normal((H, T, N))
        np.testing.assert_allclose(oracle.vjp_f64(g), brute.vjp_boxsum_f64(g),
                                   rtol=1e-12, atol=1e-12)


def test_vjp_adjoint_identity():
    """<VJP(g), x> = <g, HP(x)> for random x, g (fp64)."""
    rng = np.random.default_rng(8)
    H, T, N = 8, 21, 500
    x = rng.standard_normal((T, N))
    g = rng.standard_normal((H, T, N))
    lhs = (oracle.vjp_f64(g) * x).sum()
    rhs = (g * oracle.sum_f64(x, H)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_lse_against_scipy():
    from scipy.special import logsumexp
    from oracle import lse
    rng = np.random.default_rng(12)
    S = rng.exponential(3.0, size=(4, 9, 300)).astype(np.float32)
    got = lse.lse_f64(S, 0.5)
    for k in range(4):
        assert got[k] == pytest.approx(logsumexp(S[k].astype(np.float64) / 0.5), rel=1e-13)
    w = lse.weights_f64(S, 0.5)
    np.testing.assert_allclose(w.sum(axis=(1, 2)), 1.0, rtol=1e-12)


def test_lse_gradient_finite_differences():
    """Central differences (eps = 1e-3, fp64 forward) of L = sum_k tau*LSE_k
    against the oracle gradient, on points drawn where the gradient is large
    and uniformly."""
    from oracle import lse
    rng = np.random.default_rng(13)
    T, N, H, tau = 9, 200, 8, 0.5
    x = rng.exponential(1.0, size=(T, N))

    def L(v):
        return lse.loss_f64(oracle.sum_f64(v, H), tau)

    g = lse.grad_fop_f64(oracle.sum_f64(x, H), tau)
    flat = np.abs(g).ravel()
    top = np.argsort(flat)[::-1][:16]
    uni = rng.choice(T * N, size=16, replace=False)
    eps = 1e-3
    gmax = flat.max()
    for p in np.concatenate([top, uni]):
        a, b = divmod(int(p), N)
        xp = x.copy(); xp[a, b] += eps
        xm = x.copy(); xm[a, b] -= eps
        fd = (L(xp) - L(xm)) / (2 * eps)
        assert abs(fd - g[a, b]) <= 1e-4 * gmax + 1e-3 * abs(g[a, b]), (a, b, fd, g[a, b])


def test_lse_point_gradient_equals_plane_gradient():
    """The per-point transpose (box sums of the weights) equals the scatter
    form of the whole-plane gradient at every point of a small plane."""
    from oracle import lse
    rng = np.random.default_rng(14)
    T, N, H, tau = 11, 97, 6, 0.5
    x = rng.exponential(1.0, size=(T, N)).astype(np.float32)
    S = oracle.sum_f32(x, H)
    g = lse.grad_fop_f64(S, tau, gscale=1.5)
    L = lse.lse_f64(S, tau)
    for a in range(T):
        for b in range(0, N, 7):
            assert lse.grad_point_f64(S, L, tau, a, b, gscale=1.5) == pytest.approx(g[a, b], rel=1e-12)


# --- per-plane capped lists (Sec. III: N_cand per plane) --------------------------

def test_select_top_against_sorted_brute_force():
    """The oracle's capped lists against Python's sorted() with an explicit
    (plane, -power, word) key on a small list with many tied powers and
    signed zeros."""
    rng = np.random.default_rng(3)
    N, H = 1 << 10, 5
    n = 400
    r = rng.integers(0, 7, n)
    k = rng.integers(1, H + 1, n)
    j = rng.integers(0, N, n)
    words = np.array(sorted(set(oracle.pack(a, b, c, N, H) for a, b, c in zip(r, k, j))), dtype=np.uint32)
    pw = rng.choice(np.array([0.0, -0.0, 1.5, 2.0, 2.0, 7.25, -3.0, 1e30], dtype=np.float32), len(words))
    perm = rng.permutation(len(words))
    words, pw = words[perm], pw[perm]

    def total(p):
        b = int(np.float32(p).view(np.uint32))
        return (0xFFFFFFFF - b) if b & 0x80000000 else (b | 0x80000000)

    for n_cand in (1, 3, 50, 1000):
        oi, op, oc = oracle.select_top(words, pw, N, H, n_cand)
        for kk in range(1, H + 1):
            mine = [(int(w), p) for w, p in zip(words, pw) if oracle.unpack([w], N, H)[1][0] == kk]
            want = sorted(mine, key=lambda t: (-total(t[1]), t[0]))[:n_cand]
            assert oc[kk - 1] == len(want)
            assert [int(x) for x in oi[kk - 1, :len(want)]] == [w for w, _ in want]
            got_bits = op[kk - 1, :len(want)].view(np.uint32).tolist()
            assert got_bits == [int(np.float32(p).view(np.uint32)) for _, p in want]


def test_select_last_against_streaming_process():
    """The "last N_cand" lists against the process they describe: run the
    loops of Algorithm 2 (j, then i, then k) or Algorithm 1 (k, i, j) over
    thresholded planes of a tiny FOP, appending each hit to its plane's
    ring of N_cand slots (Sec. IV-A: the last N_cand are kept), and read the
    rings out oldest first."""
    from collections import deque
    T, N, H = 9, 300, 6
    fop = rand_exp(T, N, 23)
    ta = np.stack([np.full(T, k + 1.5 * math.sqrt(k), np.float32) for k in range(1, H + 1)])
    hp = brute.planes_alg2_f32(fop, H)
    idx, pw, cnt = oracle.detect_f32(fop, H, ta)
    assert cnt[H] > 200
    for order in ("alg2", "alg1"):
        for n_cand in (1, 7, 40, 10 ** 6):
            rings = [deque(maxlen=n_cand) for _ in range(H)]
            if order == "alg2":
                loops = ((k, r, j) for j in range(N) for r in range(T) for k in range(1, H + 1))
            else:
                loops = ((k, r, j) for k in range(1, H + 1) for r in range(T) for j in range(N))
            for k, r, j in loops:
                v = hp[k - 1, r, j]
                if v > ta[k - 1, r]:
                    rings[k - 1].append((oracle.pack(r, k, j, N, H), v))
            perm = np.random.default_rng(n_cand).permutation(len(idx))   # input order must not matter
            oi, op, oc = oracle.select_last(idx[perm], pw[perm], N, H, n_cand, order=order)
            for k in range(1, H + 1):
                want = list(rings[k - 1])
                assert oc[k - 1] == len(want)
                assert [int(w) for w in oi[k - 1, :len(want)]] == [w for w, _ in want], (order, n_cand, k)
                assert np.array_equal(op[k - 1, :len(want)], np.array([v for _, v in want], np.float32))


# --- fractional variant: HPF_k(i,j) = sum_{m=1..k} FOP(floor(m i/k), floor(m j/k)) ---
# (the incoherent-sum reading of "the FOP at the fractions m/k of each point";
# not Eq. 1-2 of the paper, which it matches only for k <= 2)

@pytest.mark.parametrize("T,N,H", [(5, 64, 8), (9, 257, 16), (21, 1000, 8), (64, 300, 8)])
def test_frac_integer_planes_exact(T, N, H):
    """Integer-valued FOP: the fp32 and fp64 oracles equal whole-plane integer
    gather-sums (numpy, no rounding) bit for bit."""
    rng = np.random.default_rng(T * 7 + N)
    x = rng.integers(0, 16, size=(T, N))
    ref = brute.frac_planes_int(x, H)
    assert np.array_equal(oracle.sum_frac_f32(x.astype(np.float32), H).astype(np.int64), ref)
    assert np.array_equal(oracle.sum_frac_f64(x.astype(np.float64), H).astype(np.int64), ref)


def test_frac_k1_identity_and_k2_equals_paper():
    """HPF_1 is the FOP; HPF_2 adds the same two points as Eq. 2's HP_2 (two
    fp32 terms commute, so bitwise); from k = 3 on the mappings differ."""
    fop = rand_exp(21, 700, 5)
    hf = oracle.sum_frac_f32(fop, 8)
    hp = oracle.sum_f32(fop, 8)
    assert np.array_equal(hf[0], fop)
    assert np.array_equal(hf[1].view(np.uint32), hp[1].view(np.uint32))
    assert not np.array_equal(hf[2], hp[2])


# Spike plane for the hand-derived values: T = 9 (row centre c = 4, storage
# row r holds i = r - 4), value 1 at (r = 3, i.e. i = -1; bin 5) and 2 at
# (r = 4, i = 0; bin 6).  Each entry: (k, r, j, value), value = the sum of the
# spikes hit by the points (floor(m i/k), floor(m j/k)), m = 1..k.
FRAC_HAND = [
    (2, 3, 10, 1.0),   # m=1: (floor(-1/2), floor(10/2)) = (-1, 5)
    (2, 3, 11, 1.0),   # m=1: (-1, 5); m=2: (-1, 11)
    (2, 2, 10, 1.0),   # i=-2, m=1: (-1, 5)
    (2, 4, 10, 0.0),   # i=0: (0, 5), (0, 10)
    (2, 4, 12, 2.0),   # m=1: (0, 6)
    (3, 3, 15, 1.0),   # m=1: (floor(-1/3), floor(15/3)) = (-1, 5)
    (3, 3, 8, 1.0),    # m=2: (floor(-2/3), floor(16/3)) = (-1, 5)
    (3, 2, 8, 0.0),    # i=-2: (-1, 2), (-2, 5), (-2, 8)
    (4, 3, 20, 1.0),   # m=1: (-1, 5)
    (4, 3, 7, 1.0),    # m=3: (floor(-3/4), floor(21/4)) = (-1, 5)
    (4, 3, 10, 1.0),   # m=2: (floor(-2/4), floor(20/4)) = (-1, 5)
    (5, 3, 10, 0.0),   # i=-1: (-1, 2), (-1, 4), (-1, 6), (-1, 8), (-1, 10)
    (3, 4, 9, 2.0),    # i=0, m=2: (0, 6)
]


def test_frac_hand_points():
    """Values derived by hand at single points of a two-spike plane, with
    negative template indices (floor, not truncation)."""
    fop = np.zeros((9, 32), dtype=np.float32)
    fop[3, 5] = 1.0
    fop[4, 6] = 2.0
    hf = oracle.sum_frac_f32(fop, 6)
    for k, r, j, v in FRAC_HAND:
        assert hf[k - 1, r, j] == v, (k, r, j)
    # (k=6, r=3, j=12): the six points are (-1, 2), (-1, 4), (-1, 6), (-1, 8),
    # (-1, 10), (-1, 12): none is a spike (bin 6 holds its spike at i = 0)
    assert hf[5, 3, 12] == 0.0


@pytest.mark.parametrize("z0", [-1, 0, 1])
def test_frac_harmonic_sum_closed_form(z0):
    """Noise-free plane with 20/n at (n z0, n f0): at (k z0, k f0) the k
    fractions m/k land exactly on the harmonics m = 1..k, so HPF_k there is
    20 (1 + 1/2 + ... + 1/k); Eq. 2's HP_k there is 20 sigma(k)/k instead."""
    T, N, H, f0 = 21, 4096, 8, 97
    fop = np.zeros((T, N), dtype=np.float32)
    synth.inject(fop, [(z0, f0, 20.0, 8)])
    hf = oracle.sum_frac_f32(fop, H).astype(np.float64)
    hd = oracle.sum_frac_f64(fop, H)
    c = T // 2
    expect = [20.0, 30.0, 110.0 / 3, 125.0 / 3, 137.0 / 3, 49.0, 363.0 / 7, 761.0 / 14]
    for k in range(1, H + 1):
        # the injected 20/n are fp32 values (relative error <= 2^-24 each)
        assert hd[k - 1, k * z0 + c, k * f0] == pytest.approx(expect[k - 1], rel=1e-7)
        assert hf[k - 1, k * z0 + c, k * f0] == pytest.approx(expect[k - 1], rel=1e-6)


def test_frac_point_definition():
    """Single points of an Exp(1) plane against a plain loop in Python floats."""
    fop = rand_exp(21, 512, 13)
    hd = oracle.sum_frac_f64(fop, 8)
    rows = fop.astype(np.float64).tolist()
    for (k, r, j) in [(1, 0, 0), (3, 0, 511), (8, 20, 500), (5, 7, 333), (7, 10, 1), (8, 3, 77)]:
        assert hd[k - 1, r, j] == pytest.approx(brute.frac_point_py(rows, k, r, j), rel=1e-13)


@pytest.mark.parametrize("T,N,H", [(5, 64, 8), (21, 1024, 8), (9, 333, 16)])
def test_frac_f32_within_summation_bound(T, N, H):
    """fp32 sums of k non-negative terms lie within (k-1) 2^-24 S of fp64."""
    fop = rand_exp(T, N, 17)
    hf = oracle.sum_frac_f32(fop, H).astype(np.float64)
    hd = oracle.sum_frac_f64(fop, H)
    for k in range(1, H + 1):
        assert np.all(np.abs(hf[k - 1] - hd[k - 1]) <= (k - 1) * 2.0 ** -24 * hd[k - 1] * (1 + 1e-6))


def test_frac_detect_matches_thresholded_planes():
    """Detection on the fractional planes: the candidates of thresholding the
    fp32 planes, with the Sec. III word, in (k, row, bin) order; exact counts
    also past a small capacity, and a power-of-two input scale."""
    T, N, H = 21, 3000, 8
    fop = rand_exp(T, N, 19)
    ta = np.stack([np.full(T, k + 2.5 * math.sqrt(k), np.float32) for k in range(1, H + 1)])
    ta[2, 5] = -np.inf
    hf = oracle.sum_frac_f32(fop, H)
    k, r, j, p = brute.candidates_from_planes(hf, ta)
    idx, pw, cnt = oracle.detect_frac_f32(fop, H, ta)
    want = np.array([oracle.pack(rr, kk, jj, N, H) for kk, rr, jj in zip(k, r, j)], dtype=np.uint32)
    assert np.array_equal(idx, want)
    assert np.array_equal(pw.view(np.uint32), p.astype(np.float32).view(np.uint32))
    assert list(cnt[:H]) == [int((k == kk).sum()) for kk in range(1, H + 1)] and cnt[H] == len(want)
    i2, p2, c2 = oracle.detect_frac_f32(fop, H, ta, cap=10)
    assert np.array_equal(c2, cnt) and np.array_equal(i2, want[:10])
    s = 0.125
    i3, p3, c3 = oracle.detect_frac_f32(fop * s, H, ta, scale=s)
    assert np.array_equal(c3, cnt) and np.array_equal(i3, want)
    assert np.array_equal(p3.view(np.uint32), pw.view(np.uint32))
    i4, p4, c4 = oracle.detect_frac_f32(fop, H, ta, nthreads=4)
    assert np.array_equal(c4, cnt) and np.array_equal(i4, want) and np.array_equal(p4, pw)
