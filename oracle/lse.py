"""Log-sum-exp detection statistic -- oracle (test infrastructure).

The statistic is not in the paper; it is the differentiable summary used for
the backward pass of the plane map (the transpose of Eq. 1-2):

    LSE_k = log sum_{i,j} exp(S_k(i,j) / tau),    L = sum_k tau * LSE_k,
    dL/dS_k(i,j) = w_k(i,j) = exp(S_k(i,j)/tau - LSE_k)   (softmax weights),

summed over every point of plane k of one FOP.  Everything here is fp64 and
uses the max shift (LSE = M/tau + log sum exp((S - M)/tau)).  S_k are the
fp32 planes (the same values the GPU forms) promoted to fp64.

Pins: scipy.special.logsumexp (independent library routine), sum_k w_k = 1
per plane, and central finite differences of L through the fp64 planes.
"""
import numpy as np

from . import vjp_f64


def lse_f64(S, tau):
    """LSE_k per plane for planes S [H][T][N] (any float dtype)."""
    S = np.asarray(S, dtype=np.float64)
    H = S.shape[0]
    out = np.empty(H, dtype=np.float64)
    for k in range(H):
        x = S[k].ravel() / tau
        M = x.max()
        out[k] = M + np.log(np.exp(x - M).sum())
    return out


def weights_f64(S, tau, lse=None):
    """Softmax weights w_k = exp(S_k/tau - LSE_k), [H][T][N] fp64."""
    S = np.asarray(S, dtype=np.float64)
    if lse is None:
        lse = lse_f64(S, tau)
    return np.exp(S / tau - lse[:, None, None])


def loss_f64(S, tau):
    """L = sum_k tau * LSE_k."""
    return float(tau * lse_f64(S, tau).sum())


def grad_fop_f64(S, tau, gscale=1.0):
    """dL/dFOP (times gscale) from fp32-or-fp64 planes S of that FOP."""
    w = weights_f64(S, tau)
    return vjp_f64(w * gscale)


def grad_point_f64(S, lse, tau, a, b, gscale=1.0):
    """dL/dFOP at one FOP point (storage row a, bin b), gscale times the
    gradient of L = sum_k tau * LSE_k, from the planes S [H][T][N] and their
    LSE (both promoted to fp64).  Transpose of Eq. 1 written out: the point
    feeds every (r, j) with floor((r - c)/m) + c = a and floor(j/m) = b, for
    m = 1..H, in planes k >= m; c = T // 2.  Only that m x m box of weights
    is evaluated, so this serves sampled checks on full-size planes."""
    H, T, N = S.shape
    c = T // 2
    total = 0.0
    for m in range(1, H + 1):
        r_lo, r_hi = max(c + m * (a - c), 0), min(c + m * (a - c) + m - 1, T - 1)
        j_lo, j_hi = m * b, min(m * b + m - 1, N - 1)
        if r_lo > r_hi or j_lo > j_hi:
            continue
        for k in range(m, H + 1):
            box = np.asarray(S[k - 1, r_lo:r_hi + 1, j_lo:j_hi + 1], dtype=np.float64)
            total += np.exp(box / tau - lse[k - 1]).sum()
    return gscale * total
