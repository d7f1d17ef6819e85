"""Shared test helpers: device placement, running the library and the oracle."""
import numpy as np
import torch

import oracle
import synth


def padded_device(fop_cpu, dtype=torch.float32, scale=1.0, pad=None, fill=float("nan")):
    """Storage copy of x*scale on cuda:0 with ld > N; padding columns hold `fill`
    so that any read beyond the last bin shows up in the results."""
    T, N = fop_cpu.shape
    align = 4 if dtype == torch.float32 else 8
    pad = align if pad is None else pad
    ld = ((N + pad + align - 1) // align) * align
    store = (fop_cpu.to(torch.float32) * scale).to(dtype)
    dev = torch.full((T, ld), fill, dtype=dtype, device="cuda")
    dev[:, :N] = store.to("cuda")
    return dev, store


def sort_cands(idx, pw):
    o = np.argsort(idx, kind="stable")
    return idx[o], pw[o]


def gpu_detect(plan, fop_dev, ta_np, capacity=None):
    ta = torch.from_numpy(np.ascontiguousarray(ta_np, dtype=np.float32)).cuda()
    if capacity is None:
        capacity = max(1024, int(plan.n_hp * fop_dev.shape[0] * plan.n_chan * 0.01))
    out, counts = plan.detect(fop_dev[:, :], ta, capacity=capacity)
    torch.cuda.synchronize()
    counts = counts.cpu().numpy()
    n = min(int(counts[-1]), capacity)
    a = out[:n].cpu().numpy()
    idx = a[:, 0].view(np.uint32).copy()
    pw = a[:, 1].view(np.float32).copy()
    return idx, pw, counts


def oracle_detect_sorted(store_cpu, H, ta_np, scale=1.0, nthreads=8):
    x = store_cpu.to(torch.float32).numpy()
    idx, pw, counts = oracle.detect_f32(x, H, ta_np, scale=scale, nthreads=nthreads)
    idx, pw = sort_cands(idx, pw)
    return idx, pw, counts


def assert_same_candidates(got, want):
    gi, gp, gc = got
    wi, wp, wc = want
    assert np.array_equal(gc, wc), (gc, wc)
    gi, gp = sort_cands(gi, gp)
    assert len(np.unique(gi)) == len(gi), "duplicate candidate words"
    assert np.array_equal(gi, wi)
    assert np.array_equal(gp.view(np.uint32), wp.view(np.uint32))


def random_thresholds(H, T, seed, base=None):
    """Per-row, per-plane thresholds around k + 6 sqrt(k), some rows all-on
    (-inf) or all-off (+inf)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, H + 1, dtype=np.float64)[:, None]
    t = (k + 6 * np.sqrt(k)) * rng.uniform(0.85, 1.15, size=(H, T))
    t = t.astype(np.float32)
    if T >= 3:
        t[rng.integers(0, H), rng.integers(0, T)] = -np.inf
        t[rng.integers(0, H), rng.integers(0, T)] = np.inf
    return t


def make_batch(lens, T, H, seed0, dtype=torch.float32, scale=1.0):
    """Seeded FOPs of the given lengths on cuda:0 (ld > N, NaN padding) and
    their CPU storage copies."""
    devs, stores = [], []
    for f, n in enumerate(lens):
        x = synth.noise(T, n, seed0 + f)
        if n > 4 * H:
            synth.inject(x, synth.draw_signals(T, n, H, 2, seed0 + f))
        d, s = padded_device(x, dtype=dtype, scale=scale, pad=8 * (f % 3))
        devs.append(d)
        stores.append(s)
    return devs, stores


def batched_call(plan, devs, ta_np, caps):
    """Run hs_detect_batched; returns per-FOP (idx, pw, counts)."""
    import paper_1805_12258_amd as hs
    dev = devs[0].device
    fops = torch.tensor([d.data_ptr() for d in devs], dtype=torch.int64, device=dev)
    lds = torch.tensor([d.stride(0) for d in devs], dtype=torch.int64, device=dev)
    offs = np.concatenate([[0], np.cumsum(caps)[:-1]]).astype(np.int64)
    out = torch.empty((int(np.sum(caps)), 2), dtype=torch.int32, device=dev)
    counts = torch.empty((len(devs), plan.n_hp + 1), dtype=torch.int64, device=dev)
    ta = torch.from_numpy(np.ascontiguousarray(ta_np, dtype=np.float32)).to(dev)
    args = (fops, lds, ta, out, torch.from_numpy(offs).to(dev),
            torch.tensor(caps, dtype=torch.int64, device=dev), counts)
    hs.hs_detect_batched(plan.handle, *args)
    torch.cuda.synchronize()
    return args, offs


def unpack_batched(out, counts, offs, caps):
    res = []
    c = counts.cpu().numpy()
    o = out.cpu().numpy()
    for f in range(len(offs)):
        n = min(int(c[f, -1]), int(caps[f]))
        a = o[offs[f]:offs[f] + n]
        res.append((a[:, 0].view(np.uint32).copy(), a[:, 1].view(np.float32).copy(), c[f].copy()))
    return res
