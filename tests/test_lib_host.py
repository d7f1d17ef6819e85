"""Host-side checks of libhs.so: no GPU needed, no compute launched.

The library loads, exports every entry point include/hs.h declares, its
planner reproduces the staging counts of Sec. IV-C, and its argument
validation rejects bad shapes before anything reaches a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1805_12258_amd as hs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "hs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(hs.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_single_hip_runtime_in_process():
    maps = open("/proc/self/maps").read()
    libs = set(re.findall(r"\S*libamdhip64\S*", maps))
    assert len(libs) == 1, libs


def test_version_and_status_strings():
    assert "gfx950" in hs.hs_version()
    assert hs.hs_status_string(hs.HS_ERR_OVERFLOW) == "candidate list exceeds capacity"
    assert hs.hs_status_string(0) == "ok"


def test_plan_ska_geometry():
    """85 templates, 8 planes: distinct source rows per stretch factor are
    85, 43, 29, 22, 18, 15, 13, 12 (237 in all, under the bound 240 of Sec. IV-C)."""
    p = hs.Plan(85, 1 << 21, 8)
    info = p.info
    assert info["src_rows"][1:9] == [85, 43, 29, 22, 18, 15, 13, 12]
    assert sum(info["src_rows"][1:9]) == 237
    assert (info["s_row"], info["s_k"], info["s_bin"]) == (24, 3, 21)
    # the rows are split into equal row blocks that fit the LDS budget
    R, nb = info["tile_rows"], info["row_blocks"]
    assert R * nb >= 85 and (nb - 1) * R < 85 and R <= 48
    assert info["lds_bytes"] <= 80 * 1024
    assert info["tiles_total"] == nb * (1 << 21) // info["tile_bins"]
    # staged words per full tile ~ sum_m rows_m * B/m: 0.54x of the tile's own points
    ratio = info["staged_words"] / (85 * info["tile_bins"])
    assert 0.53 < ratio < 0.56


def test_plan_h16_packing():
    p = hs.Plan(85, 1 << 21, 16)
    assert (p.info["s_row"], p.info["s_k"], p.info["s_bin"]) == (25, 4, 21)


def test_plan_row_blocks_for_tall_planes():
    p = hs.Plan(2001, 1 << 12, 16)
    info = p.info
    assert info["row_blocks"] > 1
    assert info["lds_bytes"] <= 80 * 1024
    assert info["tile_rows"] * info["row_blocks"] >= 2001


def test_plan_batched_tiles():
    lens = [1 << 19, 1 << 20, 1 << 21, 1000, 1]
    p = hs.Plan(85, 0, 16, n_chans=lens)
    tb = p.info["tile_bins"]
    rb = p.info["row_blocks"]
    assert p.info["tiles_total"] == rb * sum((n + tb - 1) // tb for n in lens)
    assert p.info["n_chan_max"] == 1 << 21


@pytest.mark.parametrize("kw", [
    dict(n_temp=0, n_chan=10, n_hp=8),
    dict(n_temp=85, n_chan=0, n_hp=8),
    dict(n_temp=85, n_chan=10, n_hp=0),
    dict(n_temp=85, n_chan=10, n_hp=17),
    dict(n_temp=85, n_chan=10, n_hp=8, input_scale=0.1),
    dict(n_temp=85, n_chan=10, n_hp=8, input_scale=-0.5),
    dict(n_temp=255, n_chan=1 << 22, n_hp=16),        # 8 + 4 + 22 bits > 32
    dict(n_temp=85, n_chan=0, n_hp=8, n_chans=[10, 0]),
    dict(n_temp=85, n_chan=10, n_hp=8, dtype=7),
])
def test_plan_rejects_bad_shapes(kw):
    with pytest.raises(hs.HsError) as e:
        hs.Plan(**kw)
    assert e.value.status == hs.HS_ERR_INVALID


def test_plan_rejects_scaled_fp32():
    with pytest.raises(hs.HsError):
        hs.Plan(85, 1000, 8, dtype="f32", input_scale=0.5)


def test_plan_accepts_limits():
    hs.Plan(1, 1, 1)
    hs.Plan(128, 1 << 21, 16)                   # 7 + 4 + 21 = 32 bits
    hs.Plan(85, 1 << 21, 8, dtype="bf16", input_scale=0.125)


def test_check_counts():
    assert hs.hs_check_counts([1, 2, 3], 2, 3) == hs.HS_OK
    assert hs.hs_check_counts([1, 2, 4], 2, 3) == hs.HS_ERR_OVERFLOW
    assert hs.hs_check_counts([0, 0, -1], 2, 3) == hs.HS_ERR_INVALID


def test_null_arguments_rejected_without_gpu():
    p = hs.Plan(21, 1000, 8)
    null = ctypes.c_void_p(0)
    assert hs._c_hs_detect(p.handle, null, 1000, null, null, 0, null, null) == hs.HS_ERR_INVALID
    assert hs._c_hs_sum(p.handle, null, 1000, null, null) == hs.HS_ERR_INVALID
    # misaligned FOP pointer and bad leading dimension are rejected on the host
    fake = ctypes.c_void_p(0x1000 + 4)
    out = ctypes.c_void_p(0x2000)
    assert hs._c_hs_sum(p.handle, fake, 1000, out, null) == hs.HS_ERR_INVALID
    assert hs._c_hs_sum(p.handle, ctypes.c_void_p(0x1000), 1002, out, null) == hs.HS_ERR_INVALID
    assert hs._c_hs_sum(p.handle, ctypes.c_void_p(0x1000), 996, out, null) == hs.HS_ERR_INVALID
    pb = hs.Plan(21, 0, 8, n_chans=[100, 200])
    assert hs._c_hs_detect(pb.handle, ctypes.c_void_p(0x1000), 1000, out, out, 1, out,
                           null) == hs.HS_ERR_INVALID
    # the read-ceiling kernel: size, alignment and grid checked on the host
    src = ctypes.c_void_p(0x1000)
    for a, nb, gr in ((null, 16, 1), (src, 0, 1), (src, 24, 1), (fake, 16, 1), (src, 16, 0),
                      (src, 16, 65537)):
        assert hs._c_hs_stream_read(a, nb, out, gr, null) == hs.HS_ERR_INVALID


@pytest.mark.parametrize("T,N", [(85, 1 << 21), (21, 1 << 16), (64, 4097), (85, 3000), (5, 256 * 9),
                                 (9, 100)])
def test_tile_schedule(T, N):
    """The full-tile schedule lists every full tile exactly once; a bin tile
    and its half (x >> 1, the source tile of m = 2) sit on the same one of
    the eight lists, the half first; the lists are balanced."""
    p = hs.Plan(T, N, 8)
    w = np.array(hs.hs_plan_schedule(p.handle), dtype=np.int64)
    n_full, nb = N // 256, p.info["row_blocks"]
    if n_full == 0:
        assert len(w) == 0
        return
    off, ent = w[:9], w[9:]
    assert off[0] == 0 and off[8] == len(ent) and np.all(np.diff(off) >= 0)
    rb, bt = ent >> 24, ent & 0xFFFFFF
    assert np.array_equal(np.sort(rb * n_full + bt), np.arange(nb * n_full))
    lst = np.searchsorted(off[1:], np.arange(len(ent)), side="right")
    first = {}
    for i, (x, r) in enumerate(zip(bt.tolist(), rb.tolist())):
        if r == 0:
            first[x] = (lst[i], i)
    for x in range(16, n_full):
        assert first[x][0] == first[x >> 1][0], x
        assert first[x >> 1][1] < first[x][1], x
    sizes = np.diff(off) // nb
    assert sizes.max() - sizes.min() <= max(2, n_full // 16)
    if n_full & (n_full - 1) == 0 and n_full >= 8:
        assert sizes.min() == sizes.max() == n_full // 8
    # contiguous chunks on request, and for batched plans
    assert hs.hs_plan_schedule(hs.Plan(T, N, 8, schedule=1).handle) == []
    assert hs.hs_plan_schedule(hs.Plan(T, 0, 8, n_chans=[N, N]).handle) == []


def test_detector_choice():
    """Schedule 0 picks the strip walk for 16-bit storage or more than eight
    planes and the tile kernel otherwise; 1 and 4 ask for the walk, 2 and 3
    for the tile kernel; a plane too short for the walk's pipeline (or with
    a threshold table over 16 KB) gets the tile kernel whatever is asked."""
    N = 1 << 16
    def det(T, H, dtype="f32", sched=0):
        sc = 1.0 if dtype == "f32" else 0.125
        return hs.Plan(T, N, H, dtype=dtype, input_scale=sc, schedule=sched).info["detector"]
    assert det(85, 8) == 0 and det(85, 1) == 0
    assert det(85, 8, "f16") == 1 and det(85, 8, "bf16") == 1 and det(85, 9) == 1 and det(85, 16) == 1
    assert [det(85, 8, "f32", s) for s in range(5)] == [0, 1, 0, 0, 1]
    assert [det(85, 16, "f16", s) for s in range(5)] == [1, 1, 0, 0, 1]
    assert det(1, 16) == 0 and det(1, 8, "f16", 4) == 0          # T < 2
    for V in (2, 4, 8):
        p = hs.Plan(85, N, 8, schedule=4, bins_per_lane=V)
        assert p.info["bins_per_lane"] == V and p.info["detector"] == 1
    assert hs.Plan(85, N, 8, bins_per_lane=8).info["bins_per_lane"] == 0   # tile kernel: no walk
    # planner's V: eight for 16-bit storage up to eight planes, else four
    assert hs.Plan(85, N, 8, dtype="f16", input_scale=0.125).info["bins_per_lane"] == 8
    assert hs.Plan(85, N, 9, dtype="bf16", input_scale=0.125).info["bins_per_lane"] == 4
    assert hs.Plan(85, N, 16).info["bins_per_lane"] == 4
    assert hs.Plan(85, 0, 16, n_chans=[1 << 19, 1 << 20]).info["bins_per_lane"] == 8
    for bad in (1, 3, 16, -2):
        with pytest.raises(hs.HsError):
            hs.Plan(85, N, 8, bins_per_lane=bad)
    assert det(257, 16, "f32", 4) == 0                            # 257 x 16 x 4 B > 16 KB
    assert det(256, 16, "f32", 4) == 1
    with pytest.raises(hs.HsError):
        hs.Plan(85, N, 8, schedule=5)


def test_autotune_search_and_cache(tmp_path):
    """The tuner keeps the fastest valid configuration (ties: the earlier),
    skips invalid ones, and the cache round-trips."""
    from paper_1805_12258_amd import autotune as at
    cfgs = at.candidates(True, cus=256)
    per_grid = 2 * (len(at.BINS_PER_LANE) + len(at.TILE_ROWS))
    assert len(cfgs) == 1 + len(at.GRID_FACTORS) * per_grid
    assert cfgs[0] == {"schedule": 0}                                            # planner defaults first
    assert {c.get("bins_per_lane") for c in cfgs} >= {2, 4, 8}                  # B = 128, 256, 512
    batched = at.candidates(False, cus=256)
    assert all(c["schedule"] in (0, 2, 4) for c in batched)                     # XCD orders only
    assert len(batched) == 1 + len(at.GRID_FACTORS) * (len(at.BINS_PER_LANE) + len(at.TILE_ROWS))
    times = {i: 5.0 - (i % 4) for i in range(len(cfgs))}
    times[3] = None
    best, ms, tried = at.search(cfgs, lambda c: times[cfgs.index(c)], margin=0.0)
    assert ms == min(v for v in times.values() if v is not None)
    assert cfgs.index(best) == min(i for i, v in times.items() if v == ms)
    sm = at.summary(best, ms, tried)
    assert sm["default_ms"] == times[0] and sm["config"] == best
    assert sm["runner_up_ms"] >= ms and sm["margin_vs_runner_up"] >= 0.0
    assert len(tried) == len(cfgs)
    # within the margin the incumbent stays
    near = {i: 5.0 - 0.05 * i / len(cfgs) for i in range(len(cfgs))}   # under 1 % faster
    best, ms, _ = at.search(cfgs, lambda c: near[cfgs.index(c)], margin=0.02)
    assert best == cfgs[0] and ms == 5.0
    with pytest.raises(RuntimeError):
        at.search(cfgs[:2], lambda c: None)
    path = str(tmp_path / "tune.json")
    key = at.cache_key(85, 1 << 21, 8, "f32", None, "gfx950")
    assert key != at.cache_key(85, 0, 8, "f32", [1 << 19, 1 << 20], "gfx950")
    at.store_cache(path, key, {"config": best, "ms": ms})
    assert at.load_cache(path)[key]["config"] == best
    assert at.load_cache(str(tmp_path / "missing.json")) == {}


def test_mapping_field():
    """The mapping field: the paper's Eq. 1-2 by default, the fractional
    variant on request (single FOP, N <= 2^24), anything else rejected."""
    p = hs.Plan(85, 1 << 21, 8)
    assert p.info["mapping"] == hs.HS_MAP_PAPER
    f = hs.Plan(85, 1 << 21, 8, mapping="fractional")
    assert f.info["mapping"] == hs.HS_MAP_FRACTIONAL and f.info["detector"] == 2
    assert hs.hs_plan_schedule(f.handle) == []            # no tile schedule of its own
    for bad in (dict(mapping=2), dict(mapping=-1),
                dict(mapping="fractional", n_chan=0, n_chans=[100, 200]),
                dict(mapping="fractional", n_chan=(1 << 24) + 1)):
        kw = dict(n_temp=9, n_chan=1000, n_hp=8)
        kw.update(bad)
        with pytest.raises(hs.HsError) as e:
            hs.Plan(**kw)
        assert e.value.status == hs.HS_ERR_INVALID


def test_wrapper_argument_checks():
    """Shapes, dtypes and contiguity of device buffers are checked in Python
    before any call (the C ABI sees bare pointers); device None skips the
    device check so that the rules run here without a GPU."""
    import torch
    ok = torch.zeros((8, 85), dtype=torch.float32)
    hs.check_tensor(ok, "ta", torch.float32, (8, 85), None)
    for bad in (torch.zeros((8, 85), dtype=torch.float64), torch.zeros((85,), dtype=torch.float32),
                torch.zeros((85, 8), dtype=torch.float32).t(), torch.zeros((8, 84), dtype=torch.float32),
                [[0.0] * 85] * 8):
        with pytest.raises(ValueError):
            hs.check_tensor(bad, "ta", torch.float32, (8, 85), None)
    with pytest.raises(ValueError):
        hs.check_tensor(ok, "ta", torch.float32, (8, 85), torch.device("cuda", 0))   # not on the device
    out = torch.zeros((100, 2), dtype=torch.int32)
    hs.check_cand_out(out, 100, None)
    hs.check_cand_out(out, 0, None)
    for bad, cap in ((out, 101), (out, -1), (torch.zeros((100, 2), dtype=torch.int64), 10),
                     (torch.zeros((100, 3), dtype=torch.int32), 10), (torch.zeros((2, 100), dtype=torch.int32).t(), 10),
                     (torch.zeros(200, dtype=torch.int32), 10)):
        with pytest.raises(ValueError):
            hs.check_cand_out(bad, cap, None)
    # Plan methods refuse host tensors and short FOP views before any call
    plan = hs.Plan(9, 1000, 4)
    with pytest.raises(ValueError):
        plan.detect(torch.zeros((9, 1000)), torch.zeros((4, 9)), capacity=8)
    with pytest.raises(ValueError):
        plan.sum(torch.zeros((9, 1000)))
