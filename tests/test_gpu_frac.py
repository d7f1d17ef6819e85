"""Fractional mapping on the GPU, HPF_k(i,j) = sum_{m=1..k} FOP(floor(m i/k),
floor(m j/k)): planes and candidate lists bitwise equal to the oracle's, for
fp32 and 16-bit storage, ragged and degenerate shapes, and the full
85 x 2^21 plane."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1805_12258_amd as hs
import synth
from tests.helpers import assert_same_candidates, gpu_detect, padded_device, random_thresholds, sort_cands

pytestmark = pytest.mark.gpu


def exp_plane(T, N, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.empty((T, N), dtype=torch.float32).exponential_(1.0, generator=g)


def oracle_frac_sorted(store, H, ta, scale=1.0):
    x = store.to(torch.float32).numpy()
    idx, pw, cnt = oracle.detect_frac_f32(x, H, ta, scale=scale, nthreads=min(16, os.cpu_count() or 1))
    idx, pw = sort_cands(idx, pw)
    return idx, pw, cnt


SHAPES = [(21, 1 << 16, 8), (9, 257, 16), (1, 1000, 3), (8, 256 * 7 + 5, 8),
          (85, 256 * 40 + 17, 8), (33, 999, 1), (4, 3, 16)]


@pytest.mark.parametrize("T,N,H", SHAPES)
def test_frac_planes_and_candidates(T, N, H):
    print("case", T, N, H, flush=True)
    x = exp_plane(T, N, 400 + T + N + H)
    ta = random_thresholds(H, T, 7 * T + N)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H, mapping="fractional")
    assert plan.info["mapping"] == hs.HS_MAP_FRACTIONAL and plan.info["detector"] == 2
    hp = plan.sum(dev).cpu().numpy()
    ref = oracle.sum_frac_f32(store.numpy(), H)
    assert np.array_equal(hp.view(np.uint32), ref.view(np.uint32))
    assert_same_candidates(gpu_detect(plan, dev, ta, capacity=H * T * N + 16), oracle_frac_sorted(store, H, ta))


def test_frac_tiny_workload():
    """The tiny workload: candidates equal the oracle's, and every injected
    signal is found at its k-th harmonic (k z0, k f0) in plane k, where the
    fractions m/k land on its harmonics m = 1..k."""
    x = synth.make_tiny()
    T, N, H = synth.TINY["n_temp"], synth.TINY["n_chan"], synth.TINY["n_hp"]
    ta = synth.thresholds(H, T)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H, mapping="fractional")
    got = gpu_detect(plan, dev, ta, capacity=1 << 18)
    assert_same_candidates(got, oracle_frac_sorted(store, H, ta))
    words = set(got[0].tolist())
    c = T // 2
    for (z0, f0, p0, nh) in synth.tiny_signals():
        for k in range(1, H + 1):
            if abs(k * z0) <= c:
                assert oracle.pack(k * z0 + c, k, k * f0, N, H) in words, (z0, f0, k)


@pytest.mark.parametrize("name,dtype", [("f16", torch.float16), ("bf16", torch.bfloat16)])
def test_frac_reduced_precision(name, dtype):
    T, N, H, s = 21, 256 * 30 + 9, 8, 0.125
    x = exp_plane(T, N, 77)
    ta = random_thresholds(H, T, 78)
    dev, store = padded_device(x, dtype=dtype, scale=s)
    plan = hs.Plan(T, N, H, dtype=name, input_scale=s, mapping="fractional")
    hp = plan.sum(dev).cpu().numpy()
    ref = oracle.sum_frac_f32(store.to(torch.float32).numpy(), H) * np.float32(1.0 / s)
    assert np.array_equal(hp.view(np.uint32), ref.view(np.uint32))
    assert_same_candidates(gpu_detect(plan, dev, ta, capacity=H * T * N),
                           oracle_frac_sorted(store, H, ta, scale=s))


def test_frac_capacity_overflow_counts_exact():
    T, N, H = 21, 4000, 8
    x = exp_plane(T, N, 91)
    ta = np.full((H, T), 1.0, dtype=np.float32)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H, mapping="fractional")
    want = oracle_frac_sorted(store, H, ta)
    gi, gp, gc = gpu_detect(plan, dev, ta, capacity=1000)
    assert np.array_equal(gc, want[2]) and len(gi) == 1000
    wset = set(zip(want[0].tolist(), want[1].view(np.uint32).tolist()))
    assert all(p in wset for p in zip(gi.tolist(), gp.view(np.uint32).tolist()))


def test_frac_ska_full_size():
    """The 85 x 2^21 plane with 50 injected signals, 8 planes: the full
    candidate list bitwise equal to the oracle's."""
    print("case ska frac", flush=True)
    x = synth.make_ska()
    T, N, H = synth.SKA["n_temp"], synth.SKA["n_chan"], synth.SKA["n_hp"]
    ta = synth.thresholds(H, T)
    dev = x.cuda()
    plan = hs.Plan(T, N, H, mapping="fractional")
    got = gpu_detect(plan, dev, ta, capacity=1 << 22)
    assert_same_candidates(got, oracle_frac_sorted(x, H, ta))


def test_frac_plan_other_calls_unsupported():
    T, N, H = 9, 600, 4
    plan = hs.Plan(T, N, H, mapping="fractional")
    x = exp_plane(T, N, 5).cuda()
    with pytest.raises(hs.HsError) as e:
        plan.lse(x, 0.5)
    assert e.value.status == hs.HS_ERR_UNSUPPORTED
    with pytest.raises(hs.HsError) as e:
        plan.backward(torch.zeros((H, T, N), device="cuda"))
    assert e.value.status == hs.HS_ERR_UNSUPPORTED
    with pytest.raises(hs.HsError) as e:
        plan.detect_singlehp(x, torch.zeros((H, T), device="cuda"), capacity=8)
    assert e.value.status == hs.HS_ERR_UNSUPPORTED
