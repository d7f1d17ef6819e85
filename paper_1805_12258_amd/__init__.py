"""MI355X harmonic summing: Python binding of libhs.so (argument marshalling only).

Every computation runs in the HIP kernels of ``libhs.so``; this module only
turns torch tensors into device pointers, sizes and the current HIP stream
and calls the C ABI declared in ``include/hs.h``.  The functions keep the C
names (``hs_plan_create``, ``hs_sum``, ``hs_detect``, ...).  :class:`Plan`
and the helpers at the bottom are conveniences over the same calls.

The library must be built in-tree first::

    python paper_1805_12258_amd/build.py

Importing this package raises ``ImportError`` when it is not.  torch is
imported before the library is opened so that both use the same HIP runtime.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhs.so is not built; run `python paper_1805_12258_amd/build.py` "
                      "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

HS_OK = 0
HS_ERR_INVALID = -1
HS_ERR_OVERFLOW = -2
HS_ERR_HIP = -3
HS_ERR_UNSUPPORTED = -4
HS_ERR_NOMEM = -5

HS_DTYPE_F32, HS_DTYPE_F16, HS_DTYPE_BF16 = 0, 1, 2
_DTYPES = {torch.float32: HS_DTYPE_F32, torch.float16: HS_DTYPE_F16, torch.bfloat16: HS_DTYPE_BF16}
_DTYPE_NAMES = {"f32": HS_DTYPE_F32, "f16": HS_DTYPE_F16, "bf16": HS_DTYPE_BF16}


class hs_cand(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_uint32), ("power", ctypes.c_float)]


class hs_plan_desc(ctypes.Structure):
    _fields_ = [("n_temp", ctypes.c_int64), ("n_chan", ctypes.c_int64), ("n_hp", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("input_scale", ctypes.c_float),
                ("n_fops", ctypes.c_int32), ("n_chans", ctypes.POINTER(ctypes.c_int64)),
                ("tile_rows", ctypes.c_int32), ("persistent_blocks", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("mapping", ctypes.c_int32),
                ("bins_per_lane", ctypes.c_int32)]


class hs_plan_info(ctypes.Structure):
    _fields_ = [("n_temp", ctypes.c_int32), ("n_hp", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n_fops", ctypes.c_int32), ("n_chan_max", ctypes.c_int64),
                ("s_row", ctypes.c_int32), ("s_k", ctypes.c_int32), ("s_bin", ctypes.c_int32),
                ("tile_bins", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("row_blocks", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("tiles_total", ctypes.c_int64), ("src_rows", ctypes.c_int32 * 17),
                ("staged_words", ctypes.c_int64), ("detector", ctypes.c_int32),
                ("mapping", ctypes.c_int32), ("bins_per_lane", ctypes.c_int32)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SIG = {
    "hs_plan_create": ([ctypes.POINTER(_P), ctypes.POINTER(hs_plan_desc)], ctypes.c_int),
    "hs_plan_destroy": ([_P], ctypes.c_int),
    "hs_plan_info_get": ([_P, ctypes.POINTER(hs_plan_info)], ctypes.c_int),
    "hs_plan_schedule": ([_P, ctypes.POINTER(ctypes.c_uint32), _I64], _I64),
    "hs_plan_upload": ([_P], ctypes.c_int),
    "hs_sum": ([_P, _P, _I64, _P, _P], ctypes.c_int),
    "hs_detect": ([_P, _P, _I64, _P, _P, _I64, _P, _P], ctypes.c_int),
    "hs_detect_batched": ([_P, _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "hs_select_workspace_bytes": ([_P, _I64], ctypes.c_size_t),
    "hs_select_top": ([_P, _P, _I64, ctypes.c_int32, _P, _P, _P, _P], ctypes.c_int),
    "hs_select": ([_P, _P, _I64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P], ctypes.c_int),
    "hs_singlehp_workspace_bytes": ([_P], ctypes.c_size_t),
    "hs_detect_singlehp": ([_P, _P, _I64, _P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_detect_singlehp_one": ([_P, _P, _I64, _P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_workspace_bytes": ([_I64], ctypes.c_size_t),
    "hs_sort_candidates": ([_P, _I64, _P, _P], ctypes.c_int),
    "hs_backward_workspace_bytes": ([_P], ctypes.c_size_t),
    "hs_sum_backward": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "hs_lse_workspace_bytes": ([_P], ctypes.c_size_t),
    "hs_lse_forward": ([_P, _P, _I64, ctypes.c_float, _P, _P, _P, _P], ctypes.c_int),
    "hs_lse_forward_noalloc": ([_P, _P, _I64, ctypes.c_float, _P, _P, _P], ctypes.c_int),
    "hs_lse_backward": ([_P, _P, _I64, _P, ctypes.c_float, _P, _P, _P, _P],
                        ctypes.c_int),
    "hs_stream_read": ([_P, _I64, _P, ctypes.c_int32, _P], ctypes.c_int),
    "hs_check_counts": ([ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, _I64], ctypes.c_int),
    "hs_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "hs_version": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()["_c_" + _name] = _f


class HsError(RuntimeError):
    """A libhs call returned an error status."""

    def __init__(self, status, what):
        self.status = status
        msg = _c_hs_status_string(status).decode()
        super().__init__("%s failed: %s (%d)" % (what, msg, status))


def _check(status, what):
    if status != HS_OK:
        raise HsError(status, what)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libhs takes device tensors only")


# --- C names --------------------------------------------------------------------

HS_MAP_PAPER, HS_MAP_FRACTIONAL = 0, 1
_MAPPINGS = {"paper": HS_MAP_PAPER, "fractional": HS_MAP_FRACTIONAL}


def hs_plan_create(n_temp, n_chan=0, n_hp=8, dtype="f32", input_scale=1.0, n_chans=None,
                   tile_rows=0, persistent_blocks=0, schedule=0, mapping="paper", bins_per_lane=0):
    """Create a plan (host only).  Returns an opaque handle (ctypes.c_void_p)."""
    d = hs_plan_desc()
    d.n_temp = int(n_temp)
    d.n_chan = int(n_chan or 0)
    d.n_hp = int(n_hp)
    d.dtype = _DTYPE_NAMES[dtype] if isinstance(dtype, str) else _DTYPES.get(dtype, dtype)
    d.input_scale = float(input_scale)
    keep = None
    if n_chans is not None:
        keep = (ctypes.c_int64 * len(n_chans))(*[int(x) for x in n_chans])
        d.n_fops = len(n_chans)
        d.n_chans = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int64))
    d.tile_rows = int(tile_rows)
    d.persistent_blocks = int(persistent_blocks)
    d.schedule = int(schedule)
    d.mapping = _MAPPINGS[mapping] if isinstance(mapping, str) else int(mapping)
    d.bins_per_lane = int(bins_per_lane)
    h = ctypes.c_void_p()
    _check(_c_hs_plan_create(ctypes.byref(h), ctypes.byref(d)), "hs_plan_create")
    return h


def hs_plan_destroy(handle):
    _check(_c_hs_plan_destroy(handle), "hs_plan_destroy")


def hs_plan_upload(handle):
    """Copy the plan's device tables to the current device (synchronous)."""
    _check(_c_hs_plan_upload(handle), "hs_plan_upload")


def hs_plan_info_get(handle):
    info = hs_plan_info()
    _check(_c_hs_plan_info_get(handle, ctypes.byref(info)), "hs_plan_info_get")
    out = {k: getattr(info, k) for k, _ in hs_plan_info._fields_}
    out["src_rows"] = list(info.src_rows)
    return out


def hs_select_workspace_bytes(handle, n):
    return int(_c_hs_select_workspace_bytes(handle, int(n)))


HS_SELECT_TOP, HS_SELECT_LAST_ALG2, HS_SELECT_LAST_ALG1 = 0, 1, 2
_POLICIES = {"top": HS_SELECT_TOP, "last_alg2": HS_SELECT_LAST_ALG2, "last_alg1": HS_SELECT_LAST_ALG1}


def hs_select(handle, cand, n, n_cand, policy, out, out_counts, work, stream=None):
    _need_cuda(cand, out, out_counts, work)
    _check(_c_hs_select(handle, _ptr(cand), int(n), int(n_cand), int(policy), _ptr(out), _ptr(out_counts),
                        _ptr(work), _stream(stream)), "hs_select")


def hs_select_top(handle, cand, n, n_cand, out, out_counts, work, stream=None):
    _need_cuda(cand, out, out_counts, work)
    _check(_c_hs_select_top(handle, _ptr(cand), int(n), int(n_cand), _ptr(out), _ptr(out_counts),
                            _ptr(work), _stream(stream)), "hs_select_top")


def hs_singlehp_workspace_bytes(handle):
    return int(_c_hs_singlehp_workspace_bytes(handle))


def hs_detect_singlehp(handle, fop, ld, ta, out, capacity, counts, work, stream=None):
    _need_cuda(fop, ta, counts, work)
    _check(_c_hs_detect_singlehp(handle, _ptr(fop), int(ld), _ptr(ta), _ptr(out), int(capacity),
                                 _ptr(counts), _ptr(work), _stream(stream)), "hs_detect_singlehp")


def hs_detect_singlehp_one(handle, fop, ld, ta, out, capacity, counts, work, stream=None):
    _need_cuda(fop, ta, counts, work)
    _check(_c_hs_detect_singlehp_one(handle, _ptr(fop), int(ld), _ptr(ta), _ptr(out), int(capacity),
                                     _ptr(counts), _ptr(work), _stream(stream)), "hs_detect_singlehp_one")


def hs_plan_schedule(handle):
    """The plan's full-tile schedule as a list of uint32 words (host only):
    nine list offsets, then entries (row_block << 24) | bin_tile."""
    n = _c_hs_plan_schedule(handle, None, 0)
    if n < 0:
        raise HsError(HS_ERR_INVALID, "hs_plan_schedule")
    buf = (ctypes.c_uint32 * max(n, 1))()
    _c_hs_plan_schedule(handle, buf, n)
    return list(buf[:n])


def hs_sum(handle, fop, ld, hp, stream=None):
    _need_cuda(fop, hp)
    _check(_c_hs_sum(handle, _ptr(fop), int(ld), _ptr(hp), _stream(stream)), "hs_sum")


def hs_detect(handle, fop, ld, ta, out, capacity, counts, stream=None):
    _need_cuda(fop, ta, out, counts)
    _check(_c_hs_detect(handle, _ptr(fop), int(ld), _ptr(ta), _ptr(out), int(capacity),
                        _ptr(counts), _stream(stream)), "hs_detect")


def hs_detect_batched(handle, fops, lds, ta, out, out_offsets, caps, counts, stream=None):
    _need_cuda(fops, lds, ta, out, out_offsets, caps, counts)
    _check(_c_hs_detect_batched(handle, _ptr(fops), _ptr(lds), _ptr(ta), _ptr(out),
                                _ptr(out_offsets), _ptr(caps), _ptr(counts), _stream(stream)),
           "hs_detect_batched")


def hs_sort_workspace_bytes(n):
    return int(_c_hs_sort_workspace_bytes(int(n)))


def hs_sort_candidates(cand, n, work, stream=None):
    _need_cuda(cand, work)
    _check(_c_hs_sort_candidates(_ptr(cand), int(n), _ptr(work), _stream(stream)),
           "hs_sort_candidates")


def hs_stream_read(src, nbytes, sink, grid, stream=None):
    """One streaming read of `nbytes` bytes of `src` by `grid` blocks; block b
    writes the sum of its fp32 words to sink[b]."""
    _need_cuda(src, sink)
    if sink.dtype != torch.float32 or sink.numel() < int(grid):
        raise ValueError("sink must hold at least grid fp32 values")
    if src.numel() * src.element_size() < int(nbytes):
        raise ValueError("src holds fewer than nbytes bytes")
    _check(_c_hs_stream_read(_ptr(src), int(nbytes), _ptr(sink), int(grid), _stream(stream)), "hs_stream_read")


def hs_backward_workspace_bytes(handle):
    return int(_c_hs_backward_workspace_bytes(handle))


def hs_sum_backward(handle, g, dfop, work, stream=None):
    _need_cuda(g, dfop, work)
    _check(_c_hs_sum_backward(handle, _ptr(g), _ptr(dfop), _ptr(work), _stream(stream)),
           "hs_sum_backward")


def hs_lse_workspace_bytes(handle):
    return int(_c_hs_lse_workspace_bytes(handle))


def hs_lse_forward(handle, fop, ld, tau, lse, loss, work, stream=None):
    _need_cuda(fop, lse, loss, work)
    _check(_c_hs_lse_forward(handle, _ptr(fop), int(ld), float(tau), _ptr(lse), _ptr(loss), _ptr(work),
                             _stream(stream)), "hs_lse_forward")


def hs_lse_forward_noalloc(handle, fop, ld, tau, lse, loss, stream=None):
    _need_cuda(fop, lse, loss)
    _check(_c_hs_lse_forward_noalloc(handle, _ptr(fop), int(ld), float(tau), _ptr(lse), _ptr(loss),
                                     _stream(stream)), "hs_lse_forward_noalloc")


def hs_lse_backward(handle, fop, ld, lse, tau, gscale, dfop, work, stream=None):
    """gscale: a one-element fp64 device tensor (the upstream gradient) or None (1)."""
    _need_cuda(fop, lse, gscale, dfop, work)
    _check(_c_hs_lse_backward(handle, _ptr(fop), int(ld), _ptr(lse), float(tau), _ptr(gscale),
                              _ptr(dfop), _ptr(work), _stream(stream)), "hs_lse_backward")


def hs_check_counts(counts_host, n_hp, capacity):
    arr = (ctypes.c_int64 * (n_hp + 1))(*[int(x) for x in counts_host[:n_hp + 1]])
    return _c_hs_check_counts(arr, int(n_hp), int(capacity))


def hs_status_string(status):
    return _c_hs_status_string(int(status)).decode()


def hs_version():
    return _c_hs_version().decode()


# --- conveniences ------------------------------------------------------------------

def check_tensor(t, what, dtype, shape, device):
    """ValueError unless t is a contiguous `dtype` tensor of `shape` on
    `device` (device None: any).  The C ABI takes bare pointers, so shapes of
    device buffers are checked here, before any launch."""
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a tensor" % what)
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor of shape %s (got %s %s)"
                         % (what, dtype, tuple(shape), t.dtype, tuple(t.shape)))
    if device is not None and (not t.is_cuda or t.device != device):
        raise ValueError("%s must be on %s" % (what, device))


def check_cand_out(out, capacity, device):
    """ValueError unless `out` is a contiguous [rows][2] int32 tensor (on
    `device`, None: any) with at least `capacity` rows."""
    if not isinstance(out, torch.Tensor) or out.dtype != torch.int32 or out.dim() != 2 \
            or out.shape[1] != 2 or not out.is_contiguous():
        raise ValueError("candidate output must be a contiguous [capacity][2] int32 tensor")
    if capacity < 0 or capacity > out.shape[0]:
        raise ValueError("capacity %d outside 0..%d (rows of the output)" % (capacity, out.shape[0]))
    if device is not None and (not out.is_cuda or out.device != device):
        raise ValueError("candidate output must be on %s" % device)


class Plan:
    """Owning wrapper of an hs_plan handle."""

    def __init__(self, n_temp, n_chan=0, n_hp=8, dtype="f32", input_scale=1.0, n_chans=None,
                 tile_rows=0, persistent_blocks=0, schedule=0, mapping="paper", bins_per_lane=0):
        self.n_temp, self.n_hp = int(n_temp), int(n_hp)
        self.n_chan = int(n_chan or 0)
        self.n_chans = None if n_chans is None else [int(x) for x in n_chans]
        if isinstance(dtype, str):
            self.dtype = _DTYPE_NAMES[dtype]
        else:
            self.dtype = _DTYPES.get(dtype, dtype)
        self.torch_dtype = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}.get(self.dtype)
        self.input_scale = float(input_scale)
        self.handle = hs_plan_create(n_temp, n_chan, n_hp, self.dtype, input_scale, n_chans,
                                     tile_rows, persistent_blocks, schedule, mapping, bins_per_lane)
        self.info = hs_plan_info_get(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _c_hs_plan_destroy(h)
            except TypeError:          # interpreter shutdown: module globals are gone
                pass
            self.handle = None

    # -- argument checks: what the C ABI cannot see (device buffer shapes) ------

    def _fop(self, fop):
        if not isinstance(fop, torch.Tensor) or not fop.is_cuda:
            raise ValueError("FOP must be a device tensor")
        if fop.dtype != self.torch_dtype or fop.dim() != 2 or fop.shape[0] != self.n_temp:
            raise ValueError("FOP must be [n_temp][ld] of the plan's dtype")
        if fop.stride(1) != 1:
            raise ValueError("FOP rows must be contiguous")
        if fop.shape[1] < self.n_chan:
            raise ValueError("FOP has %d bins, the plan %d" % (fop.shape[1], self.n_chan))
        return fop.stride(0)

    @staticmethod
    def _dev_tensor(t, what, dtype, shape, device):
        check_tensor(t, what, dtype, shape, device)

    def _ta(self, ta, device):
        self._dev_tensor(ta, "thresholds", torch.float32, (self.n_hp, self.n_temp), device)

    def _cand_out(self, out, capacity, device):
        check_cand_out(out, capacity, device)

    def _counts(self, counts, device):
        self._dev_tensor(counts, "counts", torch.int64, (self.n_hp + 1,), device)

    def _plane(self, t, what, device):
        self._dev_tensor(t, what, torch.float32, (self.n_temp, self.n_chan), device)

    @staticmethod
    def _alloc(stream):
        """Allocate on the stream the call runs on, so that a temporary freed
        on return is not handed to other work before the kernels are done."""
        import contextlib
        return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()

    def _work(self, nbytes, device):
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)

    # -- calls -----------------------------------------------------------------------

    def sum(self, fop, out=None, stream=None):
        """All planes [H][T][N] fp32 (unscaled)."""
        ld = self._fop(fop)
        if out is None:
            with self._alloc(stream):
                out = torch.empty((self.n_hp, self.n_temp, self.n_chan), dtype=torch.float32,
                                  device=fop.device)
        self._dev_tensor(out, "planes", torch.float32, (self.n_hp, self.n_temp, self.n_chan), fop.device)
        hs_sum(self.handle, fop, ld, out, stream)
        return out

    def detect(self, fop, ta, capacity=None, out=None, counts=None, stream=None):
        """Fused planes + detection.  Returns (out, counts) device tensors:
        out is [capacity][2] int32 (word, power bits), counts [H+1] int64."""
        ld = self._fop(fop)
        dev = fop.device
        self._ta(ta, dev)
        if capacity is None:
            capacity = out.shape[0] if out is not None else 1 << 20
        capacity = int(capacity)
        with self._alloc(stream):
            if out is None:
                out = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=dev)
            if counts is None:
                counts = torch.empty(self.n_hp + 1, dtype=torch.int64, device=dev)
        self._cand_out(out, capacity, dev)
        self._counts(counts, dev)
        hs_detect(self.handle, fop, ld, ta, out, capacity, counts, stream)
        return out, counts

    def select(self, cand, n, n_cand, policy="top", stream=None):
        """Per-plane capped lists from the first n rows of a detect output
        ([cap][2] int32) under a policy ("top", "last_alg2", "last_alg1"):
        returns ([H][n_cand][2] int32, [H] int64)."""
        dev = cand.device
        self._cand_out(cand, int(n), dev)
        pol = _POLICIES[policy] if isinstance(policy, str) else int(policy)
        with self._alloc(stream):
            out = torch.zeros((self.n_hp, int(n_cand), 2), dtype=torch.int32, device=dev)
            cnt = torch.empty(self.n_hp, dtype=torch.int64, device=dev)
            work = self._work(hs_select_workspace_bytes(self.handle, n), dev)
        hs_select(self.handle, cand, n, n_cand, pol, out, cnt, work, stream)
        return out, cnt

    def select_top(self, cand, n, n_cand, stream=None):
        """select() with the "top" policy."""
        return self.select(cand, n, n_cand, "top", stream)

    def detect_singlehp(self, fop, ta, capacity=None, out=None, counts=None, stream=None, single_launch=False):
        """The SingleHP baseline (plane by plane through memory, one launch
        per plane or, with single_launch, one launch); same outputs as
        detect()."""
        ld = self._fop(fop)
        dev = fop.device
        self._ta(ta, dev)
        if capacity is None:
            capacity = out.shape[0] if out is not None else 1 << 20
        capacity = int(capacity)
        with self._alloc(stream):
            if out is None:
                out = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=dev)
            if counts is None:
                counts = torch.empty(self.n_hp + 1, dtype=torch.int64, device=dev)
            work = self._work(hs_singlehp_workspace_bytes(self.handle), dev)
        self._cand_out(out, capacity, dev)
        self._counts(counts, dev)
        (hs_detect_singlehp_one if single_launch else hs_detect_singlehp)(
            self.handle, fop, ld, ta, out, capacity, counts, work, stream)
        return out, counts

    def backward(self, g, dfop=None, stream=None):
        """dL/dFOP [T][N] fp32 from g = dL/dHP [H][T][N] fp32 (hs_sum_backward)."""
        if not isinstance(g, torch.Tensor) or not g.is_cuda:
            raise ValueError("g must be a device tensor")
        self._dev_tensor(g, "g", torch.float32, (self.n_hp, self.n_temp, self.n_chan), g.device)
        with self._alloc(stream):
            if dfop is None:
                dfop = torch.empty((self.n_temp, self.n_chan), dtype=torch.float32, device=g.device)
            work = self._work(hs_backward_workspace_bytes(self.handle), g.device)
        self._plane(dfop, "dfop", g.device)
        hs_sum_backward(self.handle, g, dfop, work, stream)
        return dfop

    def lse(self, fop, tau, stream=None, with_loss=False):
        """[H] fp64 tensor: log sum exp(HP_k / tau) over each plane; with
        with_loss, also the fp64 scalar L = sum_k tau * lse_k (both formed on
        the device)."""
        ld = self._fop(fop)
        with self._alloc(stream):
            out = torch.empty(self.n_hp, dtype=torch.float64, device=fop.device)
            loss = torch.empty((), dtype=torch.float64, device=fop.device) if with_loss else None
            work = self._work(hs_lse_workspace_bytes(self.handle), fop.device)
        hs_lse_forward(self.handle, fop, ld, tau, out, loss, work, stream)
        return (out, loss) if with_loss else out

    def lse_backward(self, fop, lse, tau, gscale=None, dfop=None, stream=None):
        """g * dL/dFOP for L = sum_k tau * lse_k, [T][N] fp32.  gscale: None
        (g = 1), a one-element fp64 device tensor (read by the kernel, no host
        copy) or a Python number (copied to the device)."""
        ld = self._fop(fop)
        dev = fop.device
        self._dev_tensor(lse, "lse", torch.float64, (self.n_hp,), dev)
        with self._alloc(stream):
            if isinstance(gscale, (int, float)):
                gscale = torch.full((), float(gscale), dtype=torch.float64, device=dev)
            if dfop is None:
                dfop = torch.empty((self.n_temp, self.n_chan), dtype=torch.float32, device=dev)
            work = self._work(hs_lse_workspace_bytes(self.handle), dev)
        if gscale is not None:
            if not isinstance(gscale, torch.Tensor) or gscale.device != dev or gscale.dtype != torch.float64 \
                    or gscale.numel() != 1 or not gscale.is_contiguous():
                raise ValueError("gscale must be a one-element fp64 tensor on %s" % dev)
        self._plane(dfop, "dfop", dev)
        hs_lse_backward(self.handle, fop, ld, lse, tau, gscale, dfop, work, stream)
        return dfop


def sort_candidates(out, n, stream=None):
    """Sort the first n rows of a detect output ([cap][2] int32) in place into
    ascending CL1 order."""
    n = int(n)
    if n > 1:
        work = torch.empty(max(hs_sort_workspace_bytes(n), 1), dtype=torch.uint8, device=out.device)
        hs_sort_candidates(out, n, work, stream)
    return out


class HarmonicSum(torch.autograd.Function):
    """planes = HarmonicSum.apply(fop, plan): all H planes of an fp32 FOP
    (hs_sum); the backward is the hand-written transpose (hs_sum_backward)."""

    @staticmethod
    def forward(ctx, fop, plan):
        if plan.dtype != 0:
            raise ValueError("autograd needs an fp32 plan")
        ctx.plan = plan
        return plan.sum(fop)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.backward(g.contiguous().float()), None


class HarmonicLSE(torch.autograd.Function):
    """loss = HarmonicLSE.apply(fop, plan, tau): L = sum_k tau * log sum
    exp(HP_k / tau) over the planes of one fp32 FOP (fp64 scalar, formed by
    the library).  The backward recomputes the planes and takes the weights
    through the transpose (hs_lse_backward), reading the upstream gradient
    from device memory: no arithmetic here and no host synchronisation."""

    @staticmethod
    def forward(ctx, fop, plan, tau):
        if plan.dtype != 0:
            raise ValueError("autograd needs an fp32 plan")
        lse, loss = plan.lse(fop, tau, with_loss=True)
        ctx.save_for_backward(fop, lse)
        ctx.plan, ctx.tau = plan, float(tau)
        return loss

    @staticmethod
    def backward(ctx, gL):
        fop, lse = ctx.saved_tensors
        g = gL.detach()
        if g.device != fop.device or g.dtype != torch.float64 or not g.is_contiguous():
            g = g.to(device=fop.device, dtype=torch.float64).contiguous()
        return ctx.plan.lse_backward(fop, lse, ctx.tau, gscale=g), None, None


def split_candidates(out, n):
    """(word uint32 numpy, power float32 numpy) of the first n entries of `out`."""
    import numpy as np
    a = out[:n].cpu().numpy()
    return a[:, 0].view(np.uint32).copy(), a[:, 1].view(np.float32).copy()
