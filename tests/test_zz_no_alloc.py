"""The allocation-free statistic (hs_lse_forward_noalloc) against the entry
point it mirrors (hs_lse_forward): bitwise equal lse and loss, on two calls
in a row, the second on a smaller plane, called through the C ABI."""
import numpy as np
import pytest
import torch

import paper_1805_12258_amd as hs
import synth

pytestmark = pytest.mark.gpu


def _pair(plan, x, tau):
    ld = x.stride(0)
    lse_a = torch.empty(plan.n_hp, dtype=torch.float64, device="cuda")
    loss_a = torch.empty((), dtype=torch.float64, device="cuda")
    work = torch.empty(hs.hs_lse_workspace_bytes(plan.handle), dtype=torch.uint8, device="cuda")
    hs.hs_lse_forward(plan.handle, x, ld, tau, lse_a, loss_a, work)
    lse_b = torch.full((plan.n_hp,), -1.0, dtype=torch.float64, device="cuda")
    loss_b = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    hs.hs_lse_forward_noalloc(plan.handle, x, ld, tau, lse_b, loss_b)
    torch.cuda.synchronize()
    return lse_a.cpu().numpy(), loss_a.item(), lse_b.cpu().numpy(), loss_b.item()


def test_noalloc_lse_matches_workspace_entry_point():
    tau = 0.5
    # first call: a larger plane, 16 planes (the most pairs per block)
    T1, N1, H1 = 85, 1 << 18, 16
    p1 = hs.Plan(T1, N1, H1)
    x1 = synth.noise(T1, N1, 501).cuda()
    a, la, b, lb = _pair(p1, x1, tau)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)) and la == lb
    assert np.all(np.isfinite(b))
    # second call: a smaller plane and fewer planes (the scratch keeps the
    # first call's pairs past this call's grid; they must not leak in)
    T2, N2, H2 = 21, 5000, 3
    p2 = hs.Plan(T2, N2, H2)
    x2 = synth.noise(T2, N2, 502).cuda()
    a, la, b, lb = _pair(p2, x2, tau)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)) and la == lb
    # and the first plane again after the smaller one
    a, la, b, lb = _pair(p1, x1, tau)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)) and la == lb


def test_noalloc_rejects_what_it_does_not_cover():
    x = synth.noise(9, 600, 3)
    lse = torch.empty(4, dtype=torch.float64, device="cuda")
    p16 = hs.Plan(9, 600, 4, dtype="f16", input_scale=0.125)
    x16 = x.to(torch.float16).cuda()
    with pytest.raises(hs.HsError) as e:
        hs.hs_lse_forward_noalloc(p16.handle, x16, x16.stride(0), 0.5, lse, None)
    assert e.value.status == hs.HS_ERR_UNSUPPORTED
    pf = hs.Plan(9, 600, 4, mapping="fractional")
    xf = x.cuda()
    with pytest.raises(hs.HsError) as e:
        hs.hs_lse_forward_noalloc(pf.handle, xf, xf.stride(0), 0.5, lse, None)
    assert e.value.status == hs.HS_ERR_UNSUPPORTED
    p = hs.Plan(9, 600, 4)
    with pytest.raises(hs.HsError) as e:
        hs.hs_lse_forward_noalloc(p.handle, xf, xf.stride(0), -1.0, lse, None)
    assert e.value.status == hs.HS_ERR_INVALID
