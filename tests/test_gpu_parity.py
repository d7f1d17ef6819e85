"""GPU parity: libhs (through the C ABI) against the CPU oracle.

Planes must be bitwise equal to the fp32 oracle (same sum order, Eq. 2) and
candidate lists equal as sets of (word, power bits) after sorting by word,
with exact per-plane counts.  Inputs are seeded; padding columns beyond the
last bin hold NaN so a read outside the plane cannot go unnoticed.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1805_12258_amd as hs
import synth
from tests.helpers import (assert_same_candidates, gpu_detect, oracle_detect_sorted,
                           padded_device, random_thresholds)

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, 1, 1), (1, 300, 16), (5, 64, 8), (9, 257, 3), (21, 1000, 13), (64, 4097, 16),
    (85, 5000, 8), (127, 777, 5), (2, 513, 2), (85, 256 * 7 + 3, 16),
]


def exp_plane(T, N, seed):
    return synth.noise(T, N, seed)


@pytest.mark.parametrize("T,N,H", SHAPES)
def test_sum_bitwise(T, N, H):
    print("case", T, N, H, flush=True)
    x = exp_plane(T, N, 100 + T + N + H)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    hp = plan.sum(dev).cpu().numpy()
    ref = oracle.sum_f32(store.numpy(), H)
    assert np.array_equal(hp.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("T,N,H", SHAPES)
def test_detect_bitwise(T, N, H):
    print("case", T, N, H, flush=True)
    x = exp_plane(T, N, 200 + T + N + H)
    ta = random_thresholds(H, T, T * N + H)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    got = gpu_detect(plan, dev, ta, capacity=H * T * N + 16)
    want = oracle_detect_sorted(store, H, ta)
    assert_same_candidates(got, want)


@pytest.mark.parametrize("T,N,H,rows", [(21, 3000, 8, 4), (64, 1000, 16, 7), (85, 2000, 8, 30)])
def test_row_blocked_tiles(T, N, H, rows):
    print("case", T, N, H, rows, flush=True)
    x = exp_plane(T, N, 300 + rows)
    ta = random_thresholds(H, T, rows)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H, tile_rows=rows)
    assert plan.info["row_blocks"] == (T + rows - 1) // rows
    got = gpu_detect(plan, dev, ta, capacity=H * T * N)
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta))
    hp = plan.sum(dev).cpu().numpy()
    assert np.array_equal(hp.view(np.uint32), oracle.sum_f32(store.numpy(), H).view(np.uint32))


@pytest.mark.parametrize("T,N,H,blocks", [(85, 256 * 300 + 17, 8, 0), (33, 1 << 16, 16, 13),
                                           (21, 256 * 40, 8, 100), (85, 256 * 64, 8, 9)])
def test_schedule_orders(T, N, H, blocks):
    """Both detection kernels (strip walk, tile kernel), in XCD order and in
    increasing order, give the oracle's planes and candidates, also with
    grids that leave the eight lists different numbers of blocks."""
    print("case", T, N, H, blocks, flush=True)
    x = exp_plane(T, N, 900 + blocks)
    ta = random_thresholds(H, T, N + blocks)
    dev, store = padded_device(x)
    want = oracle_detect_sorted(store, H, ta)
    ref = oracle.sum_f32(store.numpy(), H)
    for sched in (0, 1, 2, 3, 4):
        plan = hs.Plan(T, N, H, persistent_blocks=blocks, schedule=sched)
        assert (len(hs.hs_plan_schedule(plan.handle)) > 0) == (sched in (0, 2, 4))
        assert plan.info["detector"] == (1 if sched in (1, 4) or (sched == 0 and H > 8) else 0)
        assert_same_candidates(gpu_detect(plan, dev, ta, capacity=H * T * N), want)
        hp = plan.sum(dev).cpu().numpy()
        assert np.array_equal(hp.view(np.uint32), ref.view(np.uint32)), sched


def test_every_point_a_candidate():
    """Thresholds of -inf: every point of every plane is a candidate, which
    overflows each block's LDS buffer and exercises the spill path."""
    T, N, H = 21, 3000, 8
    x = exp_plane(T, N, 7)
    ta = np.full((H, T), -np.inf, dtype=np.float32)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    got = gpu_detect(plan, dev, ta, capacity=H * T * N)
    assert got[2][-1] == H * T * N
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta))


def test_capacity_overflow_counts_exact():
    T, N, H = 21, 5000, 8
    x = exp_plane(T, N, 8)
    ta = synth.thresholds(H, T)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    wi, wp, wc = oracle_detect_sorted(store, H, ta)
    cap = 10
    gi, gp, gc = gpu_detect(plan, dev, ta, capacity=cap)
    assert np.array_equal(gc, wc)
    assert len(gi) == cap
    pos = np.searchsorted(wi, gi)
    assert np.all(wi[pos] == gi) and np.array_equal(wp[pos].view(np.uint32), gp.view(np.uint32))
    assert hs.hs_check_counts(gc, H, cap) == hs.HS_ERR_OVERFLOW
    assert hs.hs_check_counts(gc, H, int(gc[-1])) == hs.HS_OK


def test_tiny_workload():
    """The tiny configuration: 21 x 2^16, 8 planes, T_k = k + 6 sqrt(k)."""
    x = synth.make_tiny()
    H, T = 8, x.shape[0]
    ta = synth.thresholds(H, T)
    dev, store = padded_device(x, pad=0)
    plan = hs.Plan(T, x.shape[1], H)
    got = gpu_detect(plan, dev, ta)
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta))
    hp = plan.sum(dev).cpu().numpy()
    assert np.array_equal(hp.view(np.uint32), oracle.sum_f32(store.numpy(), H).view(np.uint32))


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("T,N,H", [(21, 1 << 16, 8), (9, 1001, 16), (85, 3000, 8)])
def test_reduced_precision_bitwise(dtype, T, N, H):
    """fp16/bf16 storage of x/8: the kernel converts exactly and sums in fp32,
    so its planes and candidates equal the fp32 oracle run on the stored
    values (converted to fp32) with the same scale."""
    print("case", dtype, T, N, H, flush=True)
    x = synth.make_tiny() if (T, N) == (21, 1 << 16) else exp_plane(T, N, 400 + N)
    ta = synth.thresholds(H, T)
    scale = 0.125
    dev, store = padded_device(x, dtype=dtype, scale=scale)
    name = "f16" if dtype == torch.float16 else "bf16"
    plan = hs.Plan(T, N, H, dtype=name, input_scale=scale)
    got = gpu_detect(plan, dev, ta)
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta, scale=scale))
    hp = plan.sum(dev).cpu().numpy()
    ref = oracle.sum_f32(store.to(torch.float32).numpy(), H) / np.float32(scale)
    assert np.array_equal(hp.view(np.uint32), ref.view(np.uint32))


def test_repeat_calls_deterministic_sets():
    T, N, H = 85, 20000, 8
    x = exp_plane(T, N, 9)
    ta = synth.thresholds(H, T)
    dev, _ = padded_device(x)
    plan = hs.Plan(T, N, H)
    a = gpu_detect(plan, dev, ta)
    b = gpu_detect(plan, dev, ta)
    assert_same_candidates(a, (np.sort(b[0]), b[1][np.argsort(b[0])], b[2]))


def test_ska_full_size():
    """The bench workload at full size (85 x 2^21, 8 planes, 50 signals, the
    launch configuration the benchmark times): every candidate, bitwise."""
    x = synth.make_ska()
    H, T = 8, x.shape[0]
    ta = synth.thresholds(H, T)
    dev = x.to("cuda")
    plan = hs.Plan(T, x.shape[1], H)
    got = gpu_detect(plan, dev, ta, capacity=1 << 22)
    want = oracle_detect_sorted(x, H, ta, nthreads=16)
    assert_same_candidates(got, want)
    assert 250000 < got[2][-1] < 350000


def test_large_ragged_h16():
    T, N, H = 85, (1 << 20) + 77, 16
    x = exp_plane(T, N, 31)
    ta = synth.thresholds(H, T)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    got = gpu_detect(plan, dev, ta, capacity=1 << 22)
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta, nthreads=16))


@pytest.mark.parametrize("name,dtype,u_in,sub", [("f16", torch.float16, 2.0 ** -11, 8 * 2.0 ** -25),
                                                 ("bf16", torch.bfloat16, 2.0 ** -8, 0.0)])
def test_reduced_precision_error_bound(name, dtype, u_in, sub):
    """fp16/bf16 storage of power/8 against the fp64 oracle of the original
    fp32 plane, at every point of every plane: all terms are >= 0, so
    |S_gpu - S_64| <= (u_in + (k-1) 2^-24) S_64 + k delta_sub, with u_in the
    unit roundoff of the storage format and delta_sub the absolute error of
    an fp16 subnormal (in power units)."""
    T, N, H = 85, 1 << 16, 8
    x = synth.noise(T, N, 4000)
    synth.inject(x, synth.draw_signals(T, N, H, 20, 4000))
    scale = 0.125
    store = synth.quantize(x, dtype, scale).cuda()
    plan = hs.Plan(T, N, H, dtype=name, input_scale=scale)
    got = plan.sum(store).cpu().numpy().astype(np.float64)
    ref = oracle.sum_f64(x.numpy(), H)
    k = np.arange(1, H + 1, dtype=np.float64)[:, None, None]
    bound = (u_in + (k - 1) * 2.0 ** -24) * ref + k * sub
    err = np.abs(got - ref)
    assert np.all(err <= bound * (1 + 1e-12)), float((err / np.maximum(bound, 1e-300)).max())
    rel = err[ref >= 1.0] / ref[ref >= 1.0]
    print("%s: max rel error (S >= 1) %.3g, max abs error %.3g" % (name, rel.max(), err.max()))


@pytest.mark.parametrize("T,N,H", [(21, 1000, 8), (64, 4097, 16), (85, 256 * 7 + 3, 8), (1, 300, 3),
                                   (85, 300000, 8)])
def test_singlehp_baseline(T, N, H):
    """The SingleHP baseline (planes through memory), with one launch per
    plane and with a single launch, gives the oracle's candidates and
    counts, bitwise, like the fused kernel."""
    print("case", T, N, H, flush=True)
    x = exp_plane(T, N, 500 + T + N)
    ta = random_thresholds(H, T, N + 3)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    cap = H * T * N
    t = torch.from_numpy(np.ascontiguousarray(ta, dtype=np.float32)).cuda()
    want = oracle_detect_sorted(store, H, ta)
    for single in (False, True):
        out, counts = plan.detect_singlehp(dev, t, capacity=cap, single_launch=single)
        counts = counts.cpu().numpy()
        n = int(counts[-1])
        a = out[:n].cpu().numpy()
        got = (a[:, 0].view(np.uint32).copy(), a[:, 1].view(np.float32).copy(), counts)
        assert_same_candidates(got, want)


@pytest.mark.parametrize("T,N,H,n_cands", [(21, 1 << 14, 8, (1, 7, 100, 100000)), (33, 3000, 5, (2, 64)),
                                           (9, 1000, 1, (3,))])
def test_select_top_capped(T, N, H, n_cands):
    """Per-plane capped lists from the GPU candidate list equal the oracle's
    selection from the oracle's list, bitwise, with many exactly tied powers
    (integer-valued FOP, low thresholds)."""
    print("case", T, N, H, n_cands, flush=True)
    rng = np.random.default_rng(T + N + H)
    x = torch.from_numpy(rng.integers(0, 5, size=(T, N)).astype(np.float32))
    ta = np.repeat(np.array([k + 1.5 for k in range(1, H + 1)], dtype=np.float32)[:, None], T, axis=1)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    out, counts = plan.detect(dev, torch.from_numpy(ta).cuda(), capacity=H * T * N)
    n = int(counts[-1].item())
    wi, wp, wc = oracle_detect_sorted(store, H, ta)
    assert n == len(wi) > 0
    for n_cand in n_cands:
        got, cnt = plan.select_top(out, n, n_cand)
        oi, op, oc = oracle.select_top(wi, wp, N, H, n_cand)
        assert np.array_equal(cnt.cpu().numpy(), oc), n_cand
        g = got.cpu().numpy()
        for k in range(H):
            c = int(oc[k])
            assert np.array_equal(g[k, :c, 0].view(np.uint32), oi[k, :c]), (n_cand, k)
            assert np.array_equal(g[k, :c, 1].view(np.uint32), op[k, :c].view(np.uint32)), (n_cand, k)
    # an empty list gives zero counts
    got, cnt = plan.select_top(out, 0, 4)
    assert np.array_equal(cnt.cpu().numpy(), np.zeros(H, dtype=np.int64))


def test_autotuned_plan_matches_oracle(tmp_path):
    """The autotuner picks among configurations with identical results: the
    tuned plan (from a fresh cache, then from the cache) gives the oracle's
    candidates."""
    from paper_1805_12258_amd import autotune as at
    T, N, H = 21, 256 * 96 + 5, 8
    x = exp_plane(T, N, 77)
    ta = random_thresholds(H, T, 78)
    dev, store = padded_device(x)
    cache = str(tmp_path / "tune.json")
    best, ms, tried = at.tune(T, N, H, fops=dev, ta=torch.from_numpy(ta).cuda(), reps=1, cache=cache)
    assert ms > 0 and len(tried) == len(at.candidates(True))
    plan, cfg = at.tuned_plan(T, N, H, cache=cache)
    assert cfg == best
    assert_same_candidates(gpu_detect(plan, dev, ta, capacity=H * T * N), oracle_detect_sorted(store, H, ta))


def test_detect_on_side_stream():
    """hs_detect on a non-default stream of the current device (the plan's
    tile schedule is copied for that device): the oracle's candidates."""
    T, N, H = 21, 256 * 64, 8
    x = exp_plane(T, N, 31)
    ta = random_thresholds(H, T, 32)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    s = torch.cuda.Stream()
    t = torch.from_numpy(np.ascontiguousarray(ta, dtype=np.float32)).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out, counts = plan.detect(dev, t, capacity=H * T * N, stream=s)
    s.synchronize()
    counts = counts.cpu().numpy()
    n = int(counts[-1])
    a = out[:n].cpu().numpy()
    got = (a[:, 0].view(np.uint32).copy(), a[:, 1].view(np.float32).copy(), counts)
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta))


def test_calls_on_a_stream_that_is_not_current():
    """stream=s without making s current: the wrappers allocate their
    temporaries on s, so work queued meanwhile on the current stream cannot
    reuse them while the kernels on s still run; the results equal the
    calls on the current stream."""
    T, N, H, tau = 21, 256 * 64, 8, 0.5
    x = exp_plane(T, N, 61)
    ta = random_thresholds(H, T, 62)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    t = torch.from_numpy(np.ascontiguousarray(ta, dtype=np.float32)).cuda()
    ref_out, ref_cnt = plan.detect(dev, t, capacity=H * T * N)
    lse = plan.lse(dev, tau)
    ref_g = plan.lse_backward(dev, lse, tau, gscale=0.5)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    out, cnt = plan.detect(dev, t, capacity=H * T * N, stream=s)
    g = plan.lse_backward(dev, lse, tau, gscale=0.5, stream=s)
    junk = [torch.randn(1 << 22, device="cuda") for _ in range(4)]   # current-stream work meanwhile
    s.synchronize()
    assert torch.equal(cnt, ref_cnt)
    n = int(cnt[-1])
    a = np.sort(out[:n, 0].cpu().numpy().view(np.uint32))
    b = np.sort(ref_out[:n, 0].cpu().numpy().view(np.uint32))
    assert np.array_equal(a, b)
    assert torch.equal(g, ref_g)
    del junk


def test_wrappers_reject_bad_device_buffers():
    """Bad shapes, dtypes, capacities and short FOP views raise ValueError
    before any launch."""
    T, N, H = 9, 1000, 4
    plan = hs.Plan(T, N, H)
    x = exp_plane(T, N, 3).cuda()
    ta = torch.zeros((H, T), device="cuda")
    with pytest.raises(ValueError):
        plan.detect(x, ta.double(), capacity=8)
    with pytest.raises(ValueError):
        plan.detect(x, ta[0], capacity=8)
    with pytest.raises(ValueError):
        plan.detect(x, ta, capacity=100, out=torch.zeros((50, 2), dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        plan.detect(x[:, :N - 1], ta, capacity=8)
    with pytest.raises(ValueError):
        plan.sum(x, out=torch.zeros((H, T, N - 1), device="cuda"))
    with pytest.raises(ValueError):
        plan.backward(torch.zeros((H, T, N), device="cuda"), dfop=torch.zeros((T, N), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.lse_backward(x, torch.zeros(H, dtype=torch.float32, device="cuda"), 0.5)


def _oracle_select(policy, wi, wp, N, H, n_cand):
    if policy == "top":
        return oracle.select_top(wi, wp, N, H, n_cand)
    return oracle.select_last(wi, wp, N, H, n_cand, order="alg2" if policy == "last_alg2" else "alg1")


def _check_select(plan, out, n, wi, wp, N, H, n_cand, policy):
    got, cnt = plan.select(out, n, n_cand, policy)
    oi, op, oc = _oracle_select(policy, wi, wp, N, H, n_cand)
    assert np.array_equal(cnt.cpu().numpy(), oc), (policy, n_cand)
    g = got.cpu().numpy()
    for k in range(H):
        c = int(oc[k])
        assert np.array_equal(g[k, :c, 0].view(np.uint32), oi[k, :c]), (policy, n_cand, k)
        assert np.array_equal(g[k, :c, 1].view(np.uint32), op[k, :c].view(np.uint32)), (policy, n_cand, k)


@pytest.mark.parametrize("policy", ["top", "last_alg2", "last_alg1"])
def test_select_policies_ties_and_caps(policy):
    """All three policies on a list with many exactly tied powers (integer
    FOP): bitwise equal to the oracle's lists for caps from 1 to the bounded
    selection's limit (1024); above it the top policy takes the sorting path
    and the others are refused."""
    T, N, H = 21, 1 << 14, 8
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.integers(0, 5, size=(T, N)).astype(np.float32))
    ta = np.repeat(np.array([k + 1.5 for k in range(1, H + 1)], dtype=np.float32)[:, None], T, axis=1)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    out, counts = plan.detect(dev, torch.from_numpy(ta).cuda(), capacity=H * T * N)
    n = int(counts[-1].item())
    wi, wp, wc = oracle_detect_sorted(store, H, ta)
    assert n == len(wi) > 100000
    for n_cand in (1, 7, 200, 1023, 1024):
        _check_select(plan, out, n, wi, wp, N, H, n_cand, policy)
    if policy == "top":
        _check_select(plan, out, n, wi, wp, N, H, 1025, policy)
    else:
        with pytest.raises(hs.HsError) as e:
            plan.select(out, n, 1025, policy)
        assert e.value.status == hs.HS_ERR_UNSUPPORTED
    got, cnt = plan.select(out, 0, 4, policy)
    assert np.array_equal(cnt.cpu().numpy(), np.zeros(H, dtype=np.int64))


def test_select_refines_crowded_digits():
    """Candidates crowded into a few bins of a long plane, so the leading
    10-bit digit of the last-N_cand keys cannot separate them: the
    selection refines with the next digits and still equals the oracle."""
    T, N, H = 21, 1 << 20, 8
    x = torch.zeros((T, N), dtype=torch.float32)
    x[:, :1024] = 100.0
    x[:, 5000] = 3.0
    ta = np.full((H, T), 50.0, dtype=np.float32)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    out, counts = plan.detect(dev, torch.from_numpy(ta).cuda(), capacity=1 << 20)
    n = int(counts[-1].item())
    wi, wp, wc = oracle_detect_sorted(store, H, ta)
    assert n == len(wi) > 8 * 2048
    for policy in ("last_alg2", "last_alg1", "top"):
        for n_cand in (1, 300, 1024):
            _check_select(plan, out, n, wi, wp, N, H, n_cand, policy)


@pytest.mark.parametrize("V", [2, 4, 8])
@pytest.mark.parametrize("name,dtype,H", [("f32", torch.float32, 8), ("f32", torch.float32, 16),
                                          ("f16", torch.float16, 5), ("bf16", torch.bfloat16, 13)])
def test_walk_bins_per_lane(V, name, dtype, H):
    """The strip walk with 2, 4 and 8 bins per lane (strips of 128, 256 and
    512 bins), over ragged strips and both row bands: candidates bitwise
    equal to the oracle's, for fp32 and 16-bit storage."""
    T, N = 85, 512 * 9 + 136
    print("case", V, name, H, flush=True)
    x = exp_plane(T, N, 1000 + V + H)
    ta = random_thresholds(H, T, 2000 + V)
    scale = 1.0 if name == "f32" else 0.125
    dev, store = padded_device(x, dtype=dtype, scale=scale)
    plan = hs.Plan(T, N, H, dtype=name, input_scale=scale, schedule=4, bins_per_lane=V)
    assert plan.info["detector"] == 1 and plan.info["bins_per_lane"] == V
    got = gpu_detect(plan, dev, ta, capacity=H * T * N)
    assert_same_candidates(got, oracle_detect_sorted(store, H, ta, scale=scale))


@pytest.mark.parametrize("n,grid", [(4 * 250007, 64), (4 * 250007, 8192), (4, 1), (1 << 22, 4096)])
def test_stream_read_sum(n, grid):
    """The read-ceiling kernel reads every word once: the block sums add up
    to the buffer's sum (fp64 reference, fp32 rounding tolerance), blocks
    past the data write zero."""
    print("case", n, grid, flush=True)
    g = torch.Generator().manual_seed(n + grid)
    x = torch.rand(n, generator=g, dtype=torch.float32)
    sink = torch.full((grid,), float("nan"), dtype=torch.float32, device="cuda")
    hs.hs_stream_read(x.cuda(), 4 * n, sink, grid)
    s = sink.cpu().double()
    assert torch.isfinite(s).all()
    ref = x.double().sum().item()
    assert abs(s.sum().item() - ref) <= 1e-5 * ref + 1e-6
