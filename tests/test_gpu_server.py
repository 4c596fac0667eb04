"""Served form: continuous batching of jobs, admission by HBM footprint.

Every job's rho must be bitwise equal to the same job run alone through
ccm() (and within 1e-5 of the oracle), with or without distance indexing
tables; failure paths are forced from the host (a budget too small, a
malformed job, options that are not served, a zero timeout, a cancel).
"""
import time

import numpy as np
import pytest

import oracle
from paper_1905_00565_amd import capi, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = capi.Context(0)
    yield c
    c.close()


def make_jobs(n, seed=0, n_lo=300, n_hi=3000, r=4, E_fixed=None, tau_fixed=None):
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(n):
        N = int(rng.integers(n_lo, n_hi))
        E = int(rng.integers(1, 11)) if E_fixed is None else E_fixed
        tau = int(rng.integers(1, 5)) if tau_fixed is None else tau_fixed
        x0, y0 = rng.uniform(0.1, 0.9, 2)
        X, Y = synth.coupled_logistic(N, x0, y0)
        ne = N - (E - 1) * tau
        L = sorted(set(synth.geometric_grid(max(E + 2, 20), ne, 4)))
        jobs.append(dict(X=X, Y=Y, E=E, tau=tau, L=L, r=r, seed=100 + k))
    return jobs


def run_alone(ctx, j):
    return ctx.ccm(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])


def test_server_single_job_bitwise_and_oracle(ctx):
    j = make_jobs(1, seed=1)[0]
    with capi.Server(ctx) as srv:
        t = srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
        assert srv.wait(t) == capi.CCM_OK
        rxy, ryx, st = srv.result(t, len(j["L"]), j["r"])
    axy, ayx, _ = run_alone(ctx, j)
    assert np.array_equal(rxy, axy, equal_nan=True) and np.array_equal(ryx, ayx, equal_nan=True)
    oxy, oyx, _ = oracle.default().ccm(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
    assert np.max(np.abs(rxy - oxy)) < 1e-5 and np.max(np.abs(ryx - oyx)) < 1e-5
    assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
    assert st["realizations"] == 2 * len(j["L"]) * j["r"]


def test_server_mix_equals_alone(ctx, orc):
    jobs = make_jobs(14, seed=2)
    with capi.Server(ctx, epoch_target_ms=2.0) as srv:
        tickets = [srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
                   for j in jobs]
        got = []
        for t, j in zip(tickets, jobs):
            assert srv.wait(t) == capi.CCM_OK
            got.append(srv.result(t, len(j["L"]), j["r"]))
    spans = []
    for (rxy, ryx, st), j in zip(got, jobs):
        axy, ayx, _ = run_alone(ctx, j)
        assert np.array_equal(rxy, axy, equal_nan=True)
        assert np.array_equal(ryx, ayx, equal_nan=True)
        # every rho of every job of the mix against the oracle
        oxy, oyx = orc.ccm_threaded(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
        assert np.max(np.abs(rxy - oxy)) < 1e-5 and np.max(np.abs(ryx - oyx)) < 1e-5
        spans.append((st["t_admit"], st["t_done"]))
    # continuous batching: some jobs were on the device at the same time
    overlaps = sum(1 for a in range(len(spans)) for b in range(a + 1, len(spans))
                   if spans[a][0] < spans[b][1] and spans[b][0] < spans[a][1])
    assert overlaps > 0


def test_server_budget_forces_queueing(ctx):
    jobs = make_jobs(5, seed=3, n_lo=2000, n_hi=2040, E_fixed=6, tau_fixed=2)
    # learn each job's footprint, then give a budget that fits only one
    foot = []
    with capi.Server(ctx) as srv:
        for j in jobs:
            t = srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
            assert srv.wait(t) == capi.CCM_OK
            foot.append(srv.result(t, len(j["L"]), j["r"])[2]["device_bytes"])
    srt = sorted(foot)
    assert srt[-1] < 1.5 * srt[0]
    budget = srt[-1] + srt[0] // 4          # fits the largest, not any two
    with capi.Server(ctx, hbm_budget_bytes=budget) as srv:
        tickets = [srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
                   for j in jobs]
        res = []
        for t, j in zip(tickets, jobs):
            assert srv.wait(t) == capi.CCM_OK
            res.append(srv.result(t, len(j["L"]), j["r"]))
    for (rxy, ryx, st), j in zip(res, jobs):
        axy, ayx, _ = run_alone(ctx, j)
        assert np.array_equal(rxy, axy, equal_nan=True)
        assert np.array_equal(ryx, ayx, equal_nan=True)
    spans = sorted((st["t_admit"], st["t_done"]) for _, _, st in res)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0          # one job on the device at a time


def test_server_job_larger_than_budget(ctx):
    jobs = make_jobs(2, seed=4)
    with capi.Server(ctx, hbm_budget_bytes=2 << 20) as srv:
        X, Y = synth.coupled_logistic(50000)
        with pytest.raises(capi.CCMError) as ei:
            srv.submit(X, Y, 5, 1, [1000, 49996], 10, 1)
        assert ei.value.status == capi.CCM_E_NOMEM
        j = make_jobs(1, seed=5, n_lo=100, n_hi=150, r=2)[0]
        t = srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
        assert srv.wait(t) == capi.CCM_OK
        rxy, _, _ = srv.result(t, len(j["L"]), j["r"])
    assert np.array_equal(rxy, run_alone(ctx, j)[0], equal_nan=True)
    assert jobs


def test_server_malformed_timeout_cancel(ctx):
    x, y = synth.coupled_logistic(40000)
    with capi.Server(ctx, hbm_budget_bytes=256 << 20, max_jobs=1) as srv:
        with pytest.raises(capi.CCMError) as ei:
            srv.submit(x, y, 0, 1, [100], 2, 1)          # E = 0
        assert ei.value.status == capi.CCM_E_INVAL
        with pytest.raises(capi.CCMError):
            srv.submit(x, y, 2, 1, [3], 2, 1)            # L < E + 2
        for flag in (capi.CCM_FLAG_NESTED, capi.CCM_FLAG_SHARED_E):   # other draws: not served
            with pytest.raises(capi.CCMError) as ei:
                srv.submit(x, y, 2, 1, [100], 2, 1, flags=flag)
            assert ei.value.status == capi.CCM_E_INVAL
        long_t = srv.submit(x, y, 8, 1, [5000, 39993], 20, 3)
        assert srv.wait(long_t, 0) == capi.CCM_E_TIMEOUT
        queued = srv.submit(x[:500], y[:500], 2, 1, [50, 499], 3, 4)   # waits: max_jobs=1
        assert srv.cancel(queued) == capi.CCM_OK
        assert srv.wait(queued) == capi.CCM_E_NOTFOUND
        ok = srv.submit(x[:800], y[:800], 3, 2, [40, 796], 3, 5)
        assert srv.wait(long_t) == capi.CCM_OK
        assert srv.wait(ok) == capi.CCM_OK
        rxy, ryx, _ = srv.result(ok, 2, 3)
        with pytest.raises(capi.CCMError) as ei:
            srv.result(queued, 2, 3)
        assert ei.value.status == capi.CCM_E_NOTFOUND
        srv.result(long_t, 2, 20)
    axy, ayx, _ = ctx.ccm(x[:800], y[:800], 3, 2, [40, 796], 3, 5)
    assert np.array_equal(rxy, axy, equal_nan=True) and np.array_equal(ryx, ayx, equal_nan=True)


def test_server_destroy_with_work_outstanding(ctx):
    x, y = synth.coupled_logistic(20000)
    srv = capi.Server(ctx)
    for k in range(3):
        srv.submit(x, y, 4, 1, [1000, 19997], 10, k)
    srv.close()          # cancels and waits; must not hang or fault
    # the context is still usable afterwards
    rxy, _, _ = ctx.ccm(x[:400], y[:400], 2, 1, [50], 2, 1)
    assert np.isfinite(rxy).all()


def test_server_table_jobs_bitwise(ctx):
    """Jobs with CCM_FLAG_TABLE served beside jobs without: every job's rho
    bitwise equal to the same job alone without tables (the walk selects the
    scan's neighbours)."""
    jobs = make_jobs(6, seed=7, n_lo=2000, n_hi=6000, r=3)
    with capi.Server(ctx, epoch_target_ms=2.0) as srv:
        tickets = [srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"],
                              flags=capi.CCM_FLAG_TABLE if k % 2 == 0 else 0)
                   for k, j in enumerate(jobs)]
        for t in tickets:
            assert srv.wait(t) == capi.CCM_OK
        out = [srv.result(t, len(j["L"]), j["r"]) for t, j in zip(tickets, jobs)]
    for (rxy, ryx, _), j in zip(out, jobs):
        axy, ayx, _ = run_alone(ctx, j)
        assert np.array_equal(rxy, axy, equal_nan=True)
        assert np.array_equal(ryx, ayx, equal_nan=True)


def test_server_cancel_running_job(ctx):
    """Cancel a job while its work is on the device, then wait for it and
    collect it: the ticket stays busy until the in-flight work retires (the
    scheduler still holds the job), wait then reports it cancelled, and jobs
    submitted afterwards run to the same results as alone."""
    x, y = synth.coupled_logistic(50000)
    with capi.Server(ctx, epoch_target_ms=5.0) as srv:
        # about 2e12 pairs: long enough to be mid-flight after 0.15 s
        big = srv.submit(x, y, 8, 1, [20000, 30000, 49993], 200, 3)
        time.sleep(0.15)
        assert srv.wait(big, 0) == capi.CCM_E_TIMEOUT
        assert srv.cancel(big) == capi.CCM_OK
        try:
            srv.result(big, 3, 200)
            early = capi.CCM_OK
        except capi.CCMError as e:
            early = e.status
        # busy while retiring; unknown once retired and released by this call
        assert early in (capi.CCM_E_BUSY, capi.CCM_E_NOTFOUND)
        assert srv.wait(big) == capi.CCM_E_NOTFOUND
        with pytest.raises(capi.CCMError) as ei:
            srv.result(big, 3, 200)
        assert ei.value.status == capi.CCM_E_NOTFOUND
        jobs = make_jobs(3, seed=11)
        tickets = [srv.submit(j["X"], j["Y"], j["E"], j["tau"], j["L"], j["r"], j["seed"])
                   for j in jobs]
        out = []
        for t, j in zip(tickets, jobs):
            assert srv.wait(t) == capi.CCM_OK
            out.append(srv.result(t, len(j["L"]), j["r"]))
    for (rxy, ryx, _), j in zip(out, jobs):
        axy, ayx, _ = run_alone(ctx, j)
        assert np.array_equal(rxy, axy, equal_nan=True)
        assert np.array_equal(ryx, ayx, equal_nan=True)


def test_server_job_stream_vs_oracle(ctx, orc):
    """The first six jobs of the bench's job stream (N up to 5*10^4, every
    tau, r = 100) served together: each equals the job alone bit for bit,
    and three realizations per job (a small, a middle and the full library,
    directions alternating) equal the oracle."""
    stream = synth.job_stream(6, 1.0, seed=4)
    series = [j["make"]() for j in stream]
    with capi.Server(ctx) as srv:
        tickets = [srv.submit(X, Y, j["E"], j["tau"], j["L"], j["r"], j["seed"])
                   for (X, Y), j in zip(series, stream)]
        out = []
        for t, j in zip(tickets, stream):
            assert srv.wait(t) == capi.CCM_OK
            out.append(srv.result(t, len(j["L"]), j["r"]))
    for k, ((rxy, ryx, _), (X, Y), j) in enumerate(zip(out, series, stream)):
        axy, ayx, _ = ctx.ccm(X, Y, j["E"], j["tau"], j["L"], j["r"], j["seed"])
        assert np.array_equal(rxy, axy, equal_nan=True)
        assert np.array_equal(ryx, ayx, equal_nan=True)
        for n, il in enumerate((2, 6, len(j["L"]) - 1)):
            ri = (7 * k + 31 * n) % j["r"]
            d = (k + n) % 2
            S, T = (Y, X) if d == 0 else (X, Y)
            want = orc.realization_split(S, T, j["E"], j["tau"], j["L"][il], ri, j["seed"])
            got = (rxy if d == 0 else ryx)[il, ri]
            assert abs(got - want) < 1e-5, (k, il, ri, d, got, want)
