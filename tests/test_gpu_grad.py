"""GPU parity of the transpose (hs_sum_backward), the log-sum-exp statistic
(hs_lse_forward / hs_lse_backward), the autograd wrappers and the canonical
candidate sort, through the C ABI, against the CPU oracle.

Tolerances come from the arithmetic:
* backward: each dFOP value is an fp32 sum of the suffix sums over at most
  sum_{m<=H} m^2 box points plus H plane terms, so
  |gpu - exact| <= (sum m^2 + 2H) * 2^-24 * (transpose of |g|);
* log-sum-exp: each thread sums a few hundred terms <= 1 and the partial
  pairs are merged in a tree, so the relative error of the sum of
  exponentials, i.e. the absolute error of lse, stays below
  4 (n_per_thread + 64) 2^-24;
* gradient of the statistic: 1e-5 relative per element plus 1e-8 of the
  largest element (weights that underflow), as the differentiation workload
  asks.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1805_12258_amd as hs
import synth
from oracle import lse as olse
from tests.helpers import gpu_detect, oracle_detect_sorted, padded_device

pytestmark = pytest.mark.gpu


def backward_bound(g, H):
    terms = sum(m * m for m in range(1, H + 1)) + 2 * H
    return terms * 2.0 ** -24 * oracle.vjp_f64(np.abs(g)) + 1e-30


@pytest.mark.parametrize("T,N,H", [(5, 64, 3), (21, 1000, 8), (85, 777, 16), (64, 4097, 8),
                                   (1, 300, 4), (33, 513, 1)])
def test_backward_vs_oracle(T, N, H):
    print("case", T, N, H, flush=True)
    rng = np.random.default_rng(T * 1000 + N + H)
    g = rng.standard_normal((H, T, N)).astype(np.float32)
    plan = hs.Plan(T, N, H)
    got = plan.backward(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    want = oracle.vjp_f64(g)
    err = np.abs(got - want)
    assert np.all(err <= backward_bound(g, H)), float((err / backward_bound(g, H)).max())


def test_backward_deterministic_and_touch_map():
    """g_8 = 1 and every other plane 0 on 64 x 2^12: the transpose is the
    read count of each FOP point when plane 8 is formed (Sec. IV-A), small
    integers, so it is exact; its maximum is the printed 204."""
    T, N, H = 64, 1 << 12, 8
    g = torch.zeros((H, T, N), dtype=torch.float32, device="cuda")
    g[H - 1] = 1.0
    plan = hs.Plan(T, N, H)
    a = plan.backward(g).cpu().numpy()
    b = plan.backward(g).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    touch = oracle.touch_counts(T, N, H)
    assert np.array_equal(a, touch.astype(np.float32))
    assert a.max() == 204


def test_backward_row_blocked():
    T, N, H = 85, 2000, 8
    rng = np.random.default_rng(5)
    g = rng.standard_normal((H, T, N)).astype(np.float32)
    for rows in (7, 30):
        plan = hs.Plan(T, N, H, tile_rows=rows)
        got = plan.backward(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - oracle.vjp_f64(g)) <= backward_bound(g, H)), rows


def lse_tol(T, N, lse_ref):
    per_thread = (T * N + 256 * 256 - 1) // (256 * 256)
    return 4 * (per_thread + 64) * 2.0 ** -24 + 1e-12 * np.abs(lse_ref)


@pytest.mark.parametrize("T,N,H,tau", [(21, 1 << 12, 8, 0.5), (9, 1004, 16, 1.7), (85, 3000, 8, 0.5)])
def test_lse_forward_and_gradient(T, N, H, tau):
    print("case", T, N, H, tau, flush=True)
    x = synth.noise(T, N, 600 + N)
    synth.inject(x, [(0, 40, 30.0, H)])
    plan = hs.Plan(T, N, H)
    dev = x.cuda()
    lse = plan.lse(dev, tau)
    S = oracle.sum_f32(x.numpy(), H)
    ref = olse.lse_f64(S, tau)
    got = lse.cpu().numpy()
    assert np.all(np.abs(got - ref) <= lse_tol(T, N, ref)), (got - ref)
    dfop = plan.lse_backward(dev, lse, tau, gscale=0.75).cpu().numpy().astype(np.float64)
    want = olse.grad_fop_f64(S, tau, gscale=0.75)
    assert np.all(np.abs(dfop - want) <= 1e-5 * np.abs(want) + 1e-8 * np.abs(want).max())


def test_lse_finite_differences():
    """GPU gradient against fp64 central differences (eps = 1e-3) of the
    oracle loss, on 16 points where the gradient is largest and 16 uniform
    ones: |fd - g| <= 1e-4 max|g| + 1e-3 |g|."""
    T, N, H, tau = 9, 256, 8, 0.5
    rng = np.random.default_rng(21)
    x = rng.exponential(1.0, size=(T, N)).astype(np.float32)
    plan = hs.Plan(T, N, H)
    dev = torch.from_numpy(x).cuda()
    g = plan.lse_backward(dev, plan.lse(dev, tau), tau).cpu().numpy().astype(np.float64)
    xd = x.astype(np.float64)

    def L(v):
        return olse.loss_f64(oracle.sum_f64(v, H), tau)

    flat = np.abs(g).ravel()
    pts = np.concatenate([np.argsort(flat)[::-1][:16], rng.choice(T * N, size=16, replace=False)])
    eps = 1e-3
    for p in pts:
        a, b = divmod(int(p), N)
        xp = xd.copy(); xp[a, b] += eps
        xm = xd.copy(); xm[a, b] -= eps
        fd = (L(xp) - L(xm)) / (2 * eps)
        assert abs(fd - g[a, b]) <= 1e-4 * flat.max() + 1e-3 * abs(g[a, b]), (a, b, fd, g[a, b])


def test_autograd_wrappers():
    T, N, H, tau = 21, 2000, 8, 0.5
    x = synth.noise(T, N, 77).cuda()
    plan = hs.Plan(T, N, H)
    # HarmonicSum: d/dFOP of sum(planes * w) is the transpose of w
    w = torch.randn((H, T, N), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    xa = x.clone().requires_grad_(True)
    (hs.HarmonicSum.apply(xa, plan) * w).sum().backward()
    assert torch.equal(xa.grad, plan.backward(w))
    # HarmonicLSE: loss value and gradient equal the direct calls
    xb = x.clone().requires_grad_(True)
    loss = hs.HarmonicLSE.apply(xb, plan, tau)
    assert loss.is_cuda and loss.dtype == torch.float64 and loss.dim() == 0
    (2.0 * loss).backward()
    lse, L = plan.lse(x, tau, with_loss=True)
    assert torch.equal(loss.detach(), L)                     # the library's scalar
    assert float(L) == pytest.approx(float(tau * lse.sum()), rel=1e-12)
    g2 = torch.full((), 2.0, dtype=torch.float64, device="cuda")
    assert torch.equal(xb.grad, plan.lse_backward(x, lse, tau, gscale=g2))
    assert torch.equal(xb.grad, plan.lse_backward(x, lse, tau, gscale=2.0))
    S = oracle.sum_f32(x.cpu().numpy(), H)
    assert float(loss.detach()) == pytest.approx(olse.loss_f64(S, tau), abs=H * tau * 1e-5)


def test_differentiation_workload_sampled():
    """One FOP of the differentiation workload at full size (85 x 2^20,
    8 planes, tau = 0.5): lse against the oracle, and the gradient at 48
    sampled points (the 24 largest and 24 uniform) against the per-point
    oracle transpose."""
    cfg = synth.DIFF
    T, N, H, tau = cfg["n_temp"], cfg["n_chan"], cfg["n_hp"], cfg["tau"]
    x = synth.make_diff_fop(0)
    plan = hs.Plan(T, N, H)
    dev = x.cuda()
    lse = plan.lse(dev, tau)
    g = plan.lse_backward(dev, lse, tau).cpu().numpy()
    S = oracle.sum_f32(x.numpy(), H)
    ref = olse.lse_f64(S, tau)
    got = lse.cpu().numpy()
    assert np.all(np.abs(got - ref) <= lse_tol(T, N, ref))
    rng = np.random.default_rng(8)
    flat = np.abs(g).ravel()
    pts = np.concatenate([np.argpartition(flat, -24)[-24:], rng.choice(T * N, size=24, replace=False)])
    gmax = olse.grad_point_f64(S, ref, tau, *divmod(int(np.argmax(flat)), N))
    for p in pts:
        a, b = divmod(int(p), N)
        want = olse.grad_point_f64(S, ref, tau, a, b)
        assert abs(g[a, b] - want) <= 1e-5 * abs(want) + 1e-8 * gmax, (a, b, g[a, b], want)


@pytest.mark.parametrize("T,N,H", [(21, 1 << 16, 8), (85, 5000, 16)])
def test_sort_candidates_canonical(T, N, H):
    x = synth.make_tiny() if N == 1 << 16 else synth.noise(T, N, 91)
    ta = synth.thresholds(H, T)
    dev, store = padded_device(x)
    plan = hs.Plan(T, N, H)
    out, counts = plan.detect(dev, torch.from_numpy(ta).cuda(), capacity=H * T * N)
    n = int(counts[-1].item())
    hs.sort_candidates(out, n)
    idx, pw = hs.split_candidates(out, n)
    wi, wp, wc = oracle_detect_sorted(store, H, ta)
    assert np.array_equal(idx, wi)
    assert np.array_equal(pw.view(np.uint32), wp.view(np.uint32))


@pytest.mark.parametrize("blocks", [1, 7, 13, 600])
def test_lse_fused_grids(blocks):
    """The fused statistic (fp32 plans) at several grid sizes, also below
    eight blocks (no tile schedule) and with several tiles per block."""
    T, N, H, tau = 33, 256 * 40 + 5, 8, 0.5
    x = synth.noise(T, N, 70 + blocks)
    synth.inject(x, [(0, 300, 25.0, H)])
    dev, store = padded_device(x)          # NaN padding: a read past the last bin shows
    plan = hs.Plan(T, N, H, persistent_blocks=blocks)
    got = plan.lse(dev, tau).cpu().numpy()
    ref = olse.lse_f64(oracle.sum_f32(store.numpy(), H), tau)
    assert np.all(np.abs(got - ref) <= lse_tol(T, N, ref)), (got - ref)


@pytest.mark.parametrize("name,dtype", [("f16", torch.float16), ("bf16", torch.bfloat16)])
def test_lse_reduced_precision_storage(name, dtype):
    """16-bit storage: lse (through materialised planes) and its gradient
    (fused) of the stored values, unscaled, against the oracle on the same
    values."""
    T, N, H, tau, scale = 21, 3000, 8, 0.7, 0.125
    x = synth.noise(T, N, 44)
    store = synth.quantize(x, dtype, scale)
    plan = hs.Plan(T, N, H, dtype=name, input_scale=scale)
    dev = store.cuda()
    lse = plan.lse(dev, tau)
    got = lse.cpu().numpy()
    S = oracle.sum_f32(store.to(torch.float32).numpy(), H) / scale
    ref = olse.lse_f64(S, tau)
    assert np.all(np.abs(got - ref) <= lse_tol(T, N, ref)), (got - ref)
    # the gradient (weights formed in the transpose's tile pass from the
    # 16-bit FOP), in unscaled units, against the oracle's on the same sums
    dfop = plan.lse_backward(dev, lse, tau, gscale=1.25).cpu().numpy().astype(np.float64)
    want = olse.grad_fop_f64(S, tau, gscale=1.25)
    assert np.all(np.abs(dfop - want) <= 1e-5 * np.abs(want) + 1e-8 * np.abs(want).max())


def test_lse_backward_deterministic_ragged():
    """The statistic's gradient on a plane whose rows and bins leave ragged
    tiles (85 rows over 16-row tiles, bins not a multiple of 256), 16 planes:
    within the bound of the oracle, and bitwise the same on a second call."""
    T, N, H, tau = 85, 256 * 9 + 76, 16, 0.9
    x = synth.noise(T, N, 71)
    synth.inject(x, [(1, 23, 25.0, H)])
    plan = hs.Plan(T, N, H)
    dev = x.cuda()
    lse = plan.lse(dev, tau)
    a = plan.lse_backward(dev, lse, tau)
    b = plan.lse_backward(dev, lse, tau)
    assert torch.equal(a, b)
    S = oracle.sum_f32(x.numpy(), H)
    want = olse.grad_fop_f64(S, tau)
    got = a.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-5 * np.abs(want) + 1e-8 * np.abs(want).max())


def test_backward_unaligned_cotangent():
    """g starting 4 bytes past a 16-byte boundary takes the scalar-load path
    of the transpose; same bound against the oracle."""
    T, N, H = 21, 1024, 8
    rng = np.random.default_rng(12)
    g = rng.standard_normal((H, T, N)).astype(np.float32)
    buf = torch.empty(H * T * N + 4, dtype=torch.float32, device="cuda")
    gv = buf[1:1 + H * T * N].view(H, T, N)
    gv.copy_(torch.from_numpy(g))
    assert gv.data_ptr() % 16 == 4
    got = hs.Plan(T, N, H).backward(gv).cpu().numpy().astype(np.float64)
    err = np.abs(got - oracle.vjp_f64(g))
    assert np.all(err <= backward_bound(g, H)), float((err / backward_bound(g, H)).max())
