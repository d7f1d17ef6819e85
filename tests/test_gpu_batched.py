"""Batched persistent launch: equal to per-FOP launches and to the oracle,
also when replayed from a captured HIP graph."""
import numpy as np
import pytest
import torch

import oracle
import paper_1805_12258_amd as hs
import synth
from tests.helpers import (batched_call, gpu_detect, make_batch, oracle_detect_sorted,
                           unpack_batched)

pytestmark = pytest.mark.gpu


def triples(idx, pw, s_row, s_bin):
    """(row, plane, bin, power bits) rows of a candidate list, sorted."""
    idx = idx.astype(np.uint64)
    kmask = (1 << (s_row - s_bin)) - 1
    r = (idx >> np.uint64(s_row)).astype(np.int64)
    k = ((idx >> np.uint64(s_bin)) & np.uint64(kmask)).astype(np.int64) + 1
    j = (idx & np.uint64((1 << s_bin) - 1)).astype(np.int64)
    t = np.stack([r, k, j, pw.view(np.uint32).astype(np.int64)], axis=1)
    return t[np.lexsort(t.T[::-1])]


def oracle_triples(store, H, ta, scale=1.0):
    i, p, c = oracle_detect_sorted(store, H, ta, scale=scale)
    sr, sk, sb = oracle.field_bits(store.shape[0], store.shape[1], H)
    return triples(i, p, sb + sk, sb), c


LENS = [1000, 4096, 300, 65536, 1, 257, 20000, 256, 3 * 256 + 5]


@pytest.mark.parametrize("H,T", [(16, 85), (8, 21), (3, 9)])
def test_batched_matches_oracle_and_single(H, T):
    print("case", H, T, flush=True)
    devs, stores = make_batch(LENS, T, H, 7000 + H)
    ta = synth.thresholds(H, T)
    ta[0, T // 2] = -np.inf          # one all-on row
    plan = hs.Plan(T, 0, H, n_chans=LENS)
    caps = [H * T * n + 8 for n in LENS]
    (fops, lds, tat, out, offs_d, caps_d, counts), offs = batched_call(plan, devs, ta, caps)
    res = unpack_batched(out, counts, offs, caps)
    s_row, s_bin = plan.info["s_row"], plan.info["s_bin"]
    for f, n in enumerate(LENS):
        gi, gp, gc = res[f]
        want, wc = oracle_triples(stores[f], H, ta)
        assert np.array_equal(gc, wc), (f, gc, wc)
        assert np.array_equal(triples(gi, gp, s_row, s_bin), want), f
        single = hs.Plan(T, n, H)
        si, sp, sc = gpu_detect(single, devs[f], ta, capacity=caps[f])
        assert np.array_equal(sc, gc)
        assert np.array_equal(triples(si, sp, single.info["s_row"], single.info["s_bin"]), want)


def test_batched_small_capacity_counts_exact():
    H, T = 8, 21
    devs, stores = make_batch(LENS, T, H, 8100)
    ta = synth.thresholds(H, T)
    plan = hs.Plan(T, 0, H, n_chans=LENS)
    caps = [5] * len(LENS)
    (_, _, _, out, _, _, counts), offs = batched_call(plan, devs, ta, caps)
    res = unpack_batched(out, counts, offs, caps)
    for f in range(len(LENS)):
        want, wc = oracle_triples(stores[f], H, ta)
        gi, gp, gc = res[f]
        assert np.array_equal(gc, wc)
        assert len(gi) == min(5, int(wc[-1]))
        got = triples(gi, gp, plan.info["s_row"], plan.info["s_bin"])
        wset = set(map(tuple, want))
        assert all(tuple(t) in wset for t in got)


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_batched_reduced_precision(dtype):
    H, T = 8, 85
    lens = [5000, 777, 65536]
    devs, stores = make_batch(lens, T, H, 8200, dtype=dtype, scale=0.125)
    ta = synth.thresholds(H, T)
    name = "f16" if dtype == torch.float16 else "bf16"
    plan = hs.Plan(T, 0, H, dtype=name, input_scale=0.125, n_chans=lens)
    caps = [20000] * len(lens)
    (_, _, _, out, _, _, counts), offs = batched_call(plan, devs, ta, caps)
    res = unpack_batched(out, counts, offs, caps)
    for f in range(len(lens)):
        want, wc = oracle_triples(stores[f], H, ta, scale=0.125)
        gi, gp, gc = res[f]
        assert np.array_equal(gc, wc)
        assert np.array_equal(triples(gi, gp, plan.info["s_row"], plan.info["s_bin"]), want)


def test_batched_graph_replay():
    """Capture counter clear + persistent kernel in a HIP graph; every replay
    (with eager work and synchronisation in between) equals the eager call."""
    H, T = 16, 85
    lens = [65536, 4096, 30000, 1000]
    devs, _ = make_batch(lens, T, H, 8300)
    ta = synth.thresholds(H, T)
    plan = hs.Plan(T, 0, H, n_chans=lens)
    caps = [200000] * len(lens)
    args, offs = batched_call(plan, devs, ta, caps)      # eager (uploads the plan tables)
    fops, lds, tat, out, offs_d, caps_d, counts = args
    ref = [(triples(i, p, plan.info["s_row"], plan.info["s_bin"]), c)
           for i, p, c in unpack_batched(out, counts, offs, caps)]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        hs.hs_detect_batched(plan.handle, fops, lds, tat, out, offs_d, caps_d, counts, stream=s)
    for rep in range(4):
        out.fill_(-1)
        counts.fill_(12345)
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = unpack_batched(out, counts, offs, caps)
        for f in range(len(lens)):
            gi, gp, gc = got[f]
            assert np.array_equal(gc, ref[f][1]), (rep, f)
            assert np.array_equal(triples(gi, gp, plan.info["s_row"], plan.info["s_bin"]),
                                  ref[f][0]), (rep, f)
        del junk


def _capture_status(fn):
    """Run fn under stream capture; the library's status (0 when it returned)."""
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    status = 0
    with torch.cuda.graph(g, stream=s):
        try:
            fn(s)
        except hs.HsError as e:
            status = e.status
    torch.cuda.synchronize()
    return status, g


def test_capture_on_fresh_plan_is_rejected():
    """A captured call on a plan whose tables are not on the device yet gets
    HS_ERR_INVALID and launches nothing (a copy cannot be made inside a
    graph), for the batched, walk and tile paths; after hs_plan_upload the
    same calls capture, and every replay equals the eager result."""
    H, T = 8, 21
    lens = [5000, 777, 65536]
    devs, _ = make_batch(lens, T, H, 8400)
    ta = synth.thresholds(H, T)
    caps = [20000] * len(lens)
    # batched
    plan = hs.Plan(T, 0, H, n_chans=lens)
    fops = torch.tensor([d.data_ptr() for d in devs], dtype=torch.int64, device="cuda")
    lds = torch.tensor([d.stride(0) for d in devs], dtype=torch.int64, device="cuda")
    offs = torch.tensor(np.concatenate([[0], np.cumsum(caps)[:-1]]), dtype=torch.int64, device="cuda")
    capd = torch.tensor(caps, dtype=torch.int64, device="cuda")
    tat = torch.from_numpy(ta).cuda()
    out = torch.zeros((sum(caps), 2), dtype=torch.int32, device="cuda")
    counts = torch.zeros((len(lens), H + 1), dtype=torch.int64, device="cuda")
    call = lambda s: hs.hs_detect_batched(plan.handle, fops, lds, tat, out, offs, capd, counts, stream=s)  # noqa
    st, _ = _capture_status(call)
    assert st == hs.HS_ERR_INVALID
    assert int(counts.abs().sum()) == 0                       # nothing ran
    hs.hs_plan_upload(plan.handle)
    st, g = _capture_status(call)
    assert st == 0
    g.replay()
    torch.cuda.synchronize()
    got = counts.clone()
    (_, _, _, _, _, _, ref), _ = batched_call(plan, devs, ta, caps)
    assert torch.equal(got, ref)
    # single FOP: the tile kernel (fp32, 8 planes) and the strip walk (16 planes)
    x = devs[2]
    for Hs in (8, 16):
        p1 = hs.Plan(T, lens[2], Hs)
        t1 = torch.from_numpy(synth.thresholds(Hs, T)).cuda()
        o1 = torch.zeros((1 << 16, 2), dtype=torch.int32, device="cuda")
        c1 = torch.zeros(Hs + 1, dtype=torch.int64, device="cuda")
        call1 = lambda s: hs.hs_detect(p1.handle, x, x.stride(0), t1, o1, 1 << 16, c1, stream=s)  # noqa
        st, _ = _capture_status(call1)
        assert st == hs.HS_ERR_INVALID, Hs
        hs.hs_plan_upload(p1.handle)
        st, g1 = _capture_status(call1)
        assert st == 0
        eo, ec = p1.detect(x, t1, capacity=1 << 16)
        for _ in range(3):
            c1.fill_(-1)
            g1.replay()
            torch.cuda.synchronize()
            assert torch.equal(c1, ec)


def test_batched_real_lengths_h16():
    """One FOP each of 2^19, 2^20 and 2^21 bins (the batched workload's
    lengths; the candidate word takes its bin field from the longest) in one
    batched call with 16 planes: every candidate word and power bitwise equal
    to the oracle's, FOP by FOP."""
    H, T = 16, 85
    lens = [1 << 19, 1 << 21, 1 << 20]
    print("case batched real lengths", flush=True)
    devs, stores = make_batch(lens, T, H, 9100)
    ta = synth.thresholds(H, T)
    plan = hs.Plan(T, 0, H, n_chans=lens)
    caps = [1 << 21] * len(lens)
    (_, _, _, out, _, _, counts), offs = batched_call(plan, devs, ta, caps)
    res = unpack_batched(out, counts, offs, caps)
    s_row, s_bin = plan.info["s_row"], plan.info["s_bin"]
    for f, n in enumerate(lens):
        gi, gp, gc = res[f]
        want, wc = oracle_triples(stores[f], H, ta)
        assert np.array_equal(gc, wc), (f, gc, wc)
        assert gc[-1] > 10000
        assert np.array_equal(triples(gi, gp, s_row, s_bin), want), f


@pytest.mark.parametrize("V", [2, 8])
def test_batched_walk_bins_per_lane(V):
    """The batched strip walk with 2 and 8 bins per lane equals the oracle."""
    H, T = 8, 21
    devs, stores = make_batch(LENS, T, H, 9300 + V)
    ta = synth.thresholds(H, T)
    plan = hs.Plan(T, 0, H, n_chans=LENS, schedule=4, bins_per_lane=V)
    assert plan.info["bins_per_lane"] == V
    caps = [H * T * n + 8 for n in LENS]
    (_, _, _, out, _, _, counts), offs = batched_call(plan, devs, ta, caps)
    res = unpack_batched(out, counts, offs, caps)
    for f in range(len(LENS)):
        gi, gp, gc = res[f]
        want, wc = oracle_triples(stores[f], H, ta)
        assert np.array_equal(gc, wc), f
        assert np.array_equal(triples(gi, gp, plan.info["s_row"], plan.info["s_bin"]), want), f
