"""Harmonic-summing ORACLE -- test infrastructure, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1805_12258_amd``) and never imports it.

Two independent layers:

* ``hs_oracle.c`` (loaded here through ctypes): the harmonic planes of
  Eq. 1-2 summed in the order of Algorithm 1 (k, i, j), in fp32 (the parity
  truth) and fp64 (the accuracy truth), threshold detection with the packed
  candidate word of Sec. III, the transpose (explicit scatter over
  (k, i, j, m)) and the touch counts of Sec. IV-A; and the fractional
  variant HPF_k(i,j) = sum_{m=1..k} FOP(floor(m i/k), floor(m j/k)) (planes
  in fp32 and fp64, detection).
* ``brute`` (numpy): each point of each plane evaluated on its own from the
  definition, and Algorithm 2's loop order (j, i, k) in plain Python loops for
  tiny planes.  These pin the C layer.

The log-sum-exp statistic lives in :mod:`oracle.lse` (numpy, fp64).

Functions whose result has no pin other than the definition itself are listed
in the module docstrings as "parity unpinned".
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhs_oracle.so")
_lib = None


def build(force=False):
    """Compile hs_oracle.c with gcc (-O2, OpenMP, no fast-math, no FP contraction)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load_library(path):
    """Open a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    lib.hso_sum_f32.argtypes = [P, I64, I64, I64, I, P]
    lib.hso_sum_f64.argtypes = [P, I64, I64, I64, I, P, I]
    lib.hso_detect_f32.argtypes = [P, I64, I64, I64, I, P, ctypes.c_float, P, P, I64, P, I]
    lib.hso_vjp_f64.argtypes = [P, I64, I64, I, P]
    lib.hso_touch_counts.argtypes = [I64, I64, I, ctypes.c_uint32, P]
    lib.hso_sum_frac_f32.argtypes = [P, I64, I64, I64, I, P]
    lib.hso_sum_frac_f64.argtypes = [P, I64, I64, I64, I, P]
    lib.hso_detect_frac_f32.argtypes = [P, I64, I64, I64, I, P, ctypes.c_float, P, P, I64, P, I]
    lib.hso_pack.argtypes = [I64, I, I64, I64, I]
    lib.hso_pack.restype = ctypes.c_uint32
    lib.hso_field_bits.argtypes = [I64, I64, I, P, P, P]
    for f in (lib.hso_sum_f32, lib.hso_sum_f64, lib.hso_detect_f32, lib.hso_vjp_f64,
              lib.hso_touch_counts, lib.hso_field_bits, lib.hso_sum_frac_f32, lib.hso_sum_frac_f64,
              lib.hso_detect_frac_f32):
        f.restype = I
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = load_library(_LIB_PATH)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _plane_args(fop, n_chan):
    if fop.ndim != 2:
        raise ValueError("FOP must be 2-D [templates][ld]")
    T, ld = fop.shape
    N = ld if n_chan is None else int(n_chan)
    if N > ld or N < 1:
        raise ValueError("n_chan out of range")
    return T, N, ld


def sum_f32(fop, H, n_chan=None):
    """All H planes [H][T][N] in fp32 (Eq. 2 order, Algorithm 1 loops)."""
    fop = np.ascontiguousarray(fop, dtype=np.float32)
    T, N, ld = _plane_args(fop, n_chan)
    hp = np.empty((H, T, N), dtype=np.float32)
    rc = _load().hso_sum_f32(_ptr(fop), T, N, ld, H, _ptr(hp))
    if rc != 0:
        raise ValueError("hso_sum_f32 rc=%d" % rc)
    return hp


def sum_f64(fop, H, n_chan=None, nthreads=1):
    """All H planes [H][T][N] in fp64 from an fp64 copy of the input
    (nthreads: OpenMP threads over rows; the result does not depend on it)."""
    fop = np.ascontiguousarray(fop, dtype=np.float64)
    T, N, ld = _plane_args(fop, n_chan)
    hp = np.empty((H, T, N), dtype=np.float64)
    rc = _load().hso_sum_f64(_ptr(fop), T, N, ld, H, _ptr(hp), int(nthreads))
    if rc != 0:
        raise ValueError("hso_sum_f64 rc=%d" % rc)
    return hp


def detect_f32(fop, H, ta, scale=1.0, cap=None, n_chan=None, nthreads=1):
    """Candidates of all H planes, Algorithm 1 order.

    Returns (idx uint32[n], power float32[n], counts int64[H+1]); the lists
    hold min(total, cap) entries, counts are always the true totals.
    """
    fop = np.ascontiguousarray(fop, dtype=np.float32)
    T, N, ld = _plane_args(fop, n_chan)
    ta = np.ascontiguousarray(ta, dtype=np.float32)
    if ta.shape != (H, T):
        raise ValueError("thresholds must be [H][T]")
    if cap is None:
        cap = H * T * N
    cap = int(cap)
    idx = np.empty(max(cap, 1), dtype=np.uint32)
    pw = np.empty(max(cap, 1), dtype=np.float32)
    counts = np.zeros(H + 1, dtype=np.int64)
    rc = _load().hso_detect_f32(_ptr(fop), T, N, ld, H, _ptr(ta), float(scale),
                                _ptr(idx), _ptr(pw), cap, _ptr(counts), int(nthreads))
    if rc not in (0, -3):
        raise ValueError("hso_detect_f32 rc=%d" % rc)
    n = min(int(counts[H]), cap)
    return idx[:n].copy(), pw[:n].copy(), counts


def sum_frac_f32(fop, H, n_chan=None):
    """Fractional-variant planes [H][T][N] in fp32: HPF_k(i,j) = sum over
    m = 1..k of FOP(floor(m i/k), floor(m j/k)), added in m order."""
    fop = np.ascontiguousarray(fop, dtype=np.float32)
    T, N, ld = _plane_args(fop, n_chan)
    hp = np.empty((H, T, N), dtype=np.float32)
    rc = _load().hso_sum_frac_f32(_ptr(fop), T, N, ld, H, _ptr(hp))
    if rc != 0:
        raise ValueError("hso_sum_frac_f32 rc=%d" % rc)
    return hp


def sum_frac_f64(fop, H, n_chan=None):
    """Fractional-variant planes in fp64 from an fp64 copy of the input."""
    fop = np.ascontiguousarray(fop, dtype=np.float64)
    T, N, ld = _plane_args(fop, n_chan)
    hp = np.empty((H, T, N), dtype=np.float64)
    rc = _load().hso_sum_frac_f64(_ptr(fop), T, N, ld, H, _ptr(hp))
    if rc != 0:
        raise ValueError("hso_sum_frac_f64 rc=%d" % rc)
    return hp


def detect_frac_f32(fop, H, ta, scale=1.0, cap=None, n_chan=None, nthreads=1):
    """Candidates of the fractional-variant planes, in (k, row, bin) order,
    with the word and counts of detect_f32 (nthreads: OpenMP threads over
    rows; the result does not depend on it)."""
    fop = np.ascontiguousarray(fop, dtype=np.float32)
    T, N, ld = _plane_args(fop, n_chan)
    ta = np.ascontiguousarray(ta, dtype=np.float32)
    if ta.shape != (H, T):
        raise ValueError("thresholds must be [H][T]")
    if cap is None:
        cap = H * T * N
    cap = int(cap)
    idx = np.empty(max(cap, 1), dtype=np.uint32)
    pw = np.empty(max(cap, 1), dtype=np.float32)
    counts = np.zeros(H + 1, dtype=np.int64)
    rc = _load().hso_detect_frac_f32(_ptr(fop), T, N, ld, H, _ptr(ta), float(scale),
                                     _ptr(idx), _ptr(pw), cap, _ptr(counts), int(nthreads))
    if rc not in (0, -3):
        raise ValueError("hso_detect_frac_f32 rc=%d" % rc)
    n = min(int(counts[H]), cap)
    return idx[:n].copy(), pw[:n].copy(), counts


def vjp_f64(g):
    """Transpose of the plane map: dL/dFOP from g = dL/dHP ([H][T][N]), fp64."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    H, T, N = g.shape
    d = np.empty((T, N), dtype=np.float64)
    rc = _load().hso_vjp_f64(_ptr(g), T, N, H, _ptr(d))
    if rc != 0:
        raise ValueError("hso_vjp_f64 rc=%d" % rc)
    return d


def touch_counts(T, N, H, planes=None):
    """Read count of every FOP point when the listed planes are formed (Sec. IV-A)."""
    planes = [H] if planes is None else list(planes)
    mask = 0
    for k in planes:
        mask |= 1 << (k - 1)
    t = np.empty((T, N), dtype=np.int64)
    rc = _load().hso_touch_counts(T, N, H, mask, _ptr(t))
    if rc != 0:
        raise ValueError("hso_touch_counts rc=%d" % rc)
    return t


def pack(r, k, j, N, H):
    """Candidate word CL1 for storage row r, plane k (1-based), bin j."""
    return int(_load().hso_pack(int(r), int(k), int(j), int(N), int(H)))


def field_bits(T, N, H):
    """(s_row, s_k, s_bin) widths of the candidate word; raises if > 32 bits."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = _load().hso_field_bits(T, N, H, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if rc != 0:
        raise ValueError("candidate word does not fit 32 bits")
    return a.value, b.value, c.value


def unpack(idx, N, H):
    """Split candidate words into (row, k, bin) arrays (inverse of pack)."""
    _, sk, sj = field_bits(1, N, H)
    idx = np.asarray(idx, dtype=np.uint64)
    j = idx & np.uint64((1 << sj) - 1)
    k = ((idx >> np.uint64(sj)) & np.uint64((1 << sk) - 1)) + np.uint64(1)
    r = idx >> np.uint64(sj + sk)
    return r.astype(np.int64), k.astype(np.int64), j.astype(np.int64)


def _power_total_order(pw):
    """fp32 powers as unsigned keys in the IEEE total order of their bits."""
    b = np.asarray(pw, dtype=np.float32).view(np.uint32).astype(np.uint64)
    neg = (b & np.uint64(0x80000000)) != 0
    return np.where(neg, np.uint64(0xFFFFFFFF) - b, b | np.uint64(0x80000000))


def select_top(idx, pw, N, H, n_cand):
    """Per-plane capped lists (Sec. III: at most N_cand candidates for each
    of the N_hp planes).  Policy: the n_cand largest powers of plane k
    (IEEE total order of the fp32 bits), ties to the smaller word, in that
    order.  Returns (idx [H][n_cand] uint32, pw [H][n_cand] float32,
    counts [H]); unused slots hold 0."""
    idx = np.asarray(idx, dtype=np.uint32)
    pw = np.asarray(pw, dtype=np.float32)
    _, k, _ = unpack(idx, N, H)
    key = _power_total_order(pw)
    out_i = np.zeros((H, n_cand), dtype=np.uint32)
    out_p = np.zeros((H, n_cand), dtype=np.float32)
    cnt = np.zeros(H, dtype=np.int64)
    for kk in range(1, H + 1):
        sel = np.nonzero(k == kk)[0]
        # descending power key, then ascending word (lexsort: last key first)
        order = sel[np.lexsort((idx[sel], -key[sel].astype(np.float64)))][:n_cand]
        cnt[kk - 1] = len(order)
        out_i[kk - 1, :len(order)] = idx[order]
        out_p[kk - 1, :len(order)] = pw[order]
    return out_i, out_p, cnt


def select_last(idx, pw, N, H, n_cand, order="alg2", T=None):
    """Per-plane capped lists under the "last N_cand" policy (Sec. IV-A: when
    a plane has more than N_cand candidates, the ones met last in processing
    order are kept).  order "alg2": the loop order of Algorithm 2 (bin j
    outer, then template i, plane k inner), so within a plane the candidates
    arrive by ascending (j, row); "alg1": Algorithm 1 (plane, template, bin),
    ascending (row, j), i.e. ascending word within a plane.  Returns
    (idx [H][n_cand], pw [H][n_cand], counts [H]); each plane's kept entries
    in processing order (the earliest kept first), unused slots 0."""
    idx = np.asarray(idx, dtype=np.uint32)
    pw = np.asarray(pw, dtype=np.float32)
    r, k, j = unpack(idx, N, H)
    out_i = np.zeros((H, n_cand), dtype=np.uint32)
    out_p = np.zeros((H, n_cand), dtype=np.float32)
    cnt = np.zeros(H, dtype=np.int64)
    for kk in range(1, H + 1):
        sel = np.nonzero(k == kk)[0]
        if order == "alg2":
            seq = sel[np.lexsort((r[sel], j[sel]))]          # ascending (j, row)
        elif order == "alg1":
            seq = sel[np.lexsort((j[sel], r[sel]))]          # ascending (row, j)
        else:
            raise ValueError("order must be alg1 or alg2")
        keep = seq[max(0, len(seq) - n_cand):]
        cnt[kk - 1] = len(keep)
        out_i[kk - 1, :len(keep)] = idx[keep]
        out_p[kk - 1, :len(keep)] = pw[keep]
    return out_i, out_p, cnt
