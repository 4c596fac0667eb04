"""ccm_dev_noalloc: the cross map of ccm_dev with its device buffers taken
from a static workspace, for callers that cannot allocate device memory.

Its results must equal ccm_dev's bit for bit (same plan, kernels and merge
order) on two calls in a row, the second with a smaller input than the first
(the workspace keeps the first call's contents), and a call needing more
than the workspace holds is refused with CCM_E_NOMEM.
"""
import numpy as np
import pytest

from paper_1905_00565_amd import capi, synth

pytestmark = pytest.mark.gpu


def run_dev(ctx, torch, x, y, E, tau, L, r, seed, noalloc, **kw):
    dx = torch.tensor(x, device="cuda:0")
    dy = torch.tensor(y, device="cuda:0")
    a = torch.full((len(L), r), -7.0, dtype=torch.float64, device="cuda:0")
    b = torch.full_like(a, -7.0)
    s = torch.cuda.current_stream()
    f = ctx.ccm_dev_noalloc if noalloc else ctx.ccm_dev
    le = f(dx, dy, E, tau, L, r, seed, a, b, stream=s, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), np.asarray(le)


def test_noalloc_equals_ccm_dev_two_calls():
    import torch
    ctx = capi.Context(0)
    try:
        w = synth.workload_small()                     # N = 1000, E = 2, r = 100
        big = (w.X, w.Y, 2, 1, w.L, w.r, w.seed)
        x2, y2 = synth.coupled_logistic(300, 0.3, 0.6)
        small = (x2, y2, 3, 2, [12, 80, 296], 7, 5)
        for args, kw in ((big, {}), (small, {"exclusion_radius": 3})):
            want = run_dev(ctx, torch, *args, False, **kw)
            got = run_dev(ctx, torch, *args, True, **kw)
            for u, v in zip(want, got):
                assert u.shape == v.shape
                assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
            assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
    finally:
        ctx.close()


def test_noalloc_refuses_oversize_and_flags():
    import torch
    ctx = capi.Context(0)
    try:
        w = synth.workload_sweep()                     # N = 10^4, r = 250: too large
        with pytest.raises(capi.CCMError) as ei:
            run_dev(ctx, torch, w.X, w.Y, 5, 1, w.L, 250, 2, True)
        assert ei.value.status == capi.CCM_E_NOMEM
        assert "workspace" in capi.ccm_last_error(ctx.handle)
        x, y = synth.coupled_logistic(400)
        with pytest.raises(capi.CCMError) as ei:
            run_dev(ctx, torch, x, y, 2, 1, [50, 400], 3, 1, True, flags=capi.CCM_FLAG_TABLE)
        assert ei.value.status == capi.CCM_E_INVAL
        # the workspace is still usable after the refusals
        want = run_dev(ctx, torch, x, y, 2, 1, [50, 400], 3, 1, False)
        got = run_dev(ctx, torch, x, y, 2, 1, [50, 400], 3, 1, True)
        assert all(np.array_equal(u, v) for u, v in zip(want, got))
    finally:
        ctx.close()
