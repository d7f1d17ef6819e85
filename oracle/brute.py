"""Brute-force definitions (numpy) -- test infrastructure, pins the C oracle.

Each function is the definition written out with no blocking or reordering:

* :func:`planes_f64` evaluates every point of every harmonic plane on its own,
  HP_k(i,j) = sum_{m=1..k} FOP(floor(i/m), floor(j/m))   (Sec. III, Eq. 1-2),
  in fp64 with numpy's floor division (``//`` floors negative numbers).
* :func:`planes_alg2_f32` follows Algorithm 2's loop order (j outer, i, then
  k inner) in plain Python loops on fp32 scalars, for tiny planes only.  The
  paper states the loops of Algorithm 1 may be interchanged (Sec. III); the
  two orders give bitwise equal planes because every point is summed over
  m = 1..k in the same order either way.
* :func:`vjp_boxsum_f64` is the transpose written as "gather pooling": with
  suffix sums G_m = sum_{k>=m} g_k, each FOP point (a,b) receives, for every
  m, the sum of G_m over the m x m block of points (i,j) with floor(i/m) = a
  and floor(j/m) = b, clipped to the plane.  It is a different formula from
  the scatter loop in ``hs_oracle.c`` and must agree with it.

* :func:`frac_planes_int` and :func:`frac_point_py` are the fractional
  variant HPF_k(i,j) = sum_{m=1..k} FOP(floor(m i/k), floor(m j/k)): the
  first as whole-plane integer gathers (exact for integer-valued FOPs), the
  second as a plain loop for one point.

Rows: storage row r holds template index i = r - T//2.
"""
import numpy as np


def template_index(T):
    """Template index i of each storage row r (i = r - T//2)."""
    return np.arange(T, dtype=np.int64) - T // 2


def source_rows(T, m):
    """Storage row read by SP_m for each storage row (Eq. 1, floor)."""
    i = template_index(T)
    return (i // m) + T // 2


def source_bins(N, m):
    """Bin read by SP_m for each bin j (Eq. 1, floor)."""
    return np.arange(N, dtype=np.int64) // m


def planes_f64(fop, H, n_chan=None):
    """HP_1..HP_H as [H][T][N] float64, every point from the definition."""
    fop = np.asarray(fop)
    T = fop.shape[0]
    N = fop.shape[1] if n_chan is None else n_chan
    x = fop.astype(np.float64)
    out = np.empty((H, T, N), dtype=np.float64)
    for k in range(1, H + 1):
        acc = np.zeros((T, N), dtype=np.float64)
        for m in range(1, k + 1):
            acc += x[np.ix_(source_rows(T, m), source_bins(N, m))]
        out[k - 1] = acc
    return out


def point_f64(fop, k, r, j):
    """HP_k at storage row r, bin j, in fp64 (one point, plain loop)."""
    T = fop.shape[0]
    i = r - T // 2
    s = 0.0
    for m in range(1, k + 1):
        s += float(fop[i // m + T // 2, j // m])
    return s


def planes_alg2_f32(fop, H):
    """Algorithm 2 order (j, i, k) in fp32 scalar arithmetic; tiny planes only."""
    fop = np.asarray(fop, dtype=np.float32)
    T, N = fop.shape
    if T * N * H > 200000:
        raise ValueError("plain-loop Algorithm 2 is for tiny planes")
    out = np.empty((H, T, N), dtype=np.float32)
    c = T // 2
    for j in range(N):
        for r in range(T):
            i = r - c
            acc = np.float32(0.0)
            for k in range(1, H + 1):
                sp = fop[i // k + c, j // k]
                acc = sp if k == 1 else np.float32(acc + sp)
                out[k - 1, r, j] = acc
    return out


def candidates_from_planes(hp, ta, scale=1.0):
    """Set of candidate (k, r, j) and powers from given planes: HP_k > TA*scale."""
    H, T, N = hp.shape
    res = []
    for k in range(1, H + 1):
        thr = (ta[k - 1].astype(np.float32) * np.float32(scale))[:, None]
        rr, jj = np.nonzero(hp[k - 1] > thr)
        res.append((np.full(rr.shape, k), rr, jj, hp[k - 1][rr, jj]))
    k = np.concatenate([x[0] for x in res])
    r = np.concatenate([x[1] for x in res])
    j = np.concatenate([x[2] for x in res])
    p = np.concatenate([x[3] for x in res])
    return k, r, j, p


def vjp_boxsum_f64(g):
    """dL/dFOP from g = dL/dHP by block sums of suffix sums (gather form)."""
    g = np.asarray(g, dtype=np.float64)
    H, T, N = g.shape
    G = np.cumsum(g[::-1], axis=0)[::-1]          # G_m = sum_{k >= m} g_k
    d = np.zeros((T, N), dtype=np.float64)
    c = T // 2
    for m in range(1, H + 1):
        # index (a, b) of the block that each plane point falls into
        a = (template_index(T) // m) + c
        b = np.arange(N) // m
        # sum over rows within each block, then over bins within each block
        rows = np.zeros((T, N), dtype=np.float64)
        np.add.at(rows, a, G[m - 1])
        blk = np.zeros((T, N), dtype=np.float64)
        np.add.at(blk.T, b, rows.T)
        d += blk
    return d


def frac_planes_int(fop_int, H):
    """HPF_1..HPF_H as [H][T][N] int64 from an integer-valued FOP, each plane
    one integer gather-sum over its k fractions m/k (no rounding)."""
    x = np.asarray(fop_int, dtype=np.int64)
    T, N = x.shape
    i = template_index(T)
    j = np.arange(N, dtype=np.int64)
    out = np.empty((H, T, N), dtype=np.int64)
    for k in range(1, H + 1):
        acc = np.zeros((T, N), dtype=np.int64)
        for m in range(1, k + 1):
            acc += x[np.ix_((m * i) // k + T // 2, (m * j) // k)]
        out[k - 1] = acc
    return out


def frac_point_py(fop, k, r, j):
    """HPF_k at storage row r, bin j in Python floats (fp64), plain loop."""
    T = len(fop)
    i = r - T // 2
    s = 0.0
    for m in range(1, k + 1):
        s += float(fop[(m * i) // k + T // 2][(m * j) // k])
    return s
