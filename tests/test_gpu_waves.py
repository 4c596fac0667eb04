"""Memory-bounded batched calls: realizations run in waves whose drawn and
gathered libraries fit a byte limit (ccm_set_wave_limit).

The waves only change which realizations share the library pools at a time;
every realization's items, tiles and merge order are unchanged, so every
form must give bitwise the same rho at any limit.  The sweep at r = 2500 --
ten times the bench's, about 300 GB of libraries if held at once -- runs
under the default limit and is checked against the oracle at sampled
realizations.
"""
import numpy as np
import pytest

from paper_1905_00565_amd import capi, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = capi.Context(0)
    yield c
    c.set_wave_limit(0)
    c.close()


def bitwise_equal(a, b):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))


def run(ctx, fn, limit):
    ctx.set_wave_limit(limit)
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    out = fn()
    p = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    ctx.set_wave_limit(0)
    return out, p["waves"]


SWEEP = dict(E=[1, 3, 6, 10], tau=[1, 2], L=[30, 300, 2000], r=5, seed=4)


@pytest.mark.parametrize("flags,excl,qs", [
    (0, 0, 0), (capi.CCM_FLAG_PERSISTENT, 0, 0), (capi.CCM_FLAG_NO_GRAPH, 2, 0),
    (capi.CCM_FLAG_PLAIN, 0, 1), (capi.CCM_FLAG_TABLE, -1, 0), (capi.CCM_FLAG_NESTED, 0, 0),
    (capi.CCM_FLAG_SHARED_E, 0, 0)])
def test_sweep_forms_any_limit(ctx, flags, excl, qs):
    x, y = synth.coupled_logistic(2000)
    w = SWEEP

    def fn():
        return ctx.ccm_sweep(x, y, w["E"], w["tau"], w["L"], w["r"], w["seed"],
                             exclusion_radius=excl, query_set=qs, flags=flags)
    ref, nw = run(ctx, fn, 1 << 40)
    assert nw == 1
    for limit in (1 << 20, 200 << 10, 1):
        got, nw = run(ctx, fn, limit)
        assert nw > 1, limit
        assert bitwise_equal(ref, got), (flags, excl, qs, limit)


def test_matrix_any_limit(ctx):
    S, _ = synth.logistic_network(6, 1500, seed=5)

    def fn():
        return ctx.ccm_matrix(S, 3, 1, [40, 400, 1500], 4, 9)
    ref, nw = run(ctx, fn, 1 << 40)
    assert nw == 1
    for limit in (100 << 10, 1):
        got, nw = run(ctx, fn, limit)
        assert nw > 1
        assert bitwise_equal(ref, got), limit


def test_device_form_small_limit(ctx):
    import torch
    x, y = synth.coupled_logistic(1500)
    L, r = [40, 1500], 3
    ref = ctx.ccm(x, y, 4, 2, L, r, 8)
    dx, dy = torch.tensor(x, device="cuda:0"), torch.tensor(y, device="cuda:0")
    a = torch.empty((2, r), dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    ctx.set_wave_limit(1)
    try:
        ctx.ccm_dev(dx, dy, 4, 2, L, r, 8, a, b, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
    finally:
        ctx.set_wave_limit(0)
    assert bitwise_equal(ref[0], a.cpu().numpy()) and bitwise_equal(ref[1], b.cpu().numpy())


def test_full_sweep_smaller_limit(ctx):
    """The bench's sweep under a 2 GiB limit (its E = 9 and 10 groups need
    more, so they split) equals it under the default, bit for bit."""
    w = synth.workload_sweep()

    def fn():
        return ctx.ccm_sweep(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed)
    ref, nw0 = run(ctx, fn, 0)
    got, nw1 = run(ctx, fn, 2 << 30)
    assert nw1 > nw0 >= 1
    assert bitwise_equal(ref, got)


def test_sweep_r2500(ctx, orc):
    """The sweep at r = 2500 (5 million realizations) under the default
    limit: finite everywhere, full-library realizations equal across r, and
    sampled realizations of every E equal to the oracle."""
    w = synth.workload_sweep(r=2500)
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    rho = ctx.ccm_sweep(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed)
    p = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    assert p["realizations"] == 2 * 10 * 5 * 20 * 2500
    assert p["waves"] > 1
    assert np.isfinite(rho).all()
    full = rho[:, :, :, -1, :]
    assert np.array_equal(full, np.repeat(full[..., :1], w.r, axis=-1))
    rng = np.random.default_rng(2500)
    picks, tasks = [], []
    for ie, e in enumerate(w.E):
        it, il = int(rng.integers(5)), int(rng.integers(14))
        ri, d = int(rng.integers(250, 2500)), ie % 2
        S, T = (w.Y, w.X) if d == 0 else (w.X, w.Y)
        picks.append((d, ie, it, il, ri))
        tasks.append((S, T, e, w.tau[it], w.L[il], ri, w.seed, 0, 0))
    want = orc.realizations_threaded(tasks)
    got = [rho[q] for q in picks]
    assert np.max(np.abs(np.asarray(got) - np.asarray(want))) < TOL
