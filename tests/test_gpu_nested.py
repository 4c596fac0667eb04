"""Nested libraries (CCM_FLAG_NESTED) against the oracle's nested mode.

The shuffled ordering must match the oracle bit for bit (integer work); rho
within 1e-5 of the oracle (the build's tolerance) for every library size,
including sizes that clamp to N_e and unsorted L lists; the batched forms
agree bit for bit among themselves; invalid combinations are rejected.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1905_00565_amd import capi, synth

pytestmark = pytest.mark.gpu
NESTED = capi.CCM_FLAG_NESTED
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = capi.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    oracle.build(force=False)
    return oracle.default()


def rho_close(a, b, tol=TOL):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(a)
    if ok.any():
        err = np.max(np.abs(a[ok] - b[ok]))
        assert err < tol, err


@pytest.mark.parametrize("key", [(1, 2, 1, 0, 20, 20), (1, 2, 1, 3, 999, 500),
                                 (12345678901234, 10, 5, 249, 9955, 9955),
                                 (7, 1, 1, 0, 1, 1), (3, 4, 2, 17, 50000, 1000)])
def test_nested_ordering_bit_exact(ctx, orc, key):
    seed, E, tau, r, ne, n = key
    assert np.array_equal(ctx.ccm_nested_library(ne, E, tau, r, seed, n),
                          orc.sample_nested(seed, E, tau, r, ne, n))


@pytest.mark.parametrize("N,E,tau,L,r,excl,kind", [
    (600, 2, 1, [50, 120, 599, 700], 4, 0, "logistic"),     # L clamps to N_e twice
    (900, 3, 2, [400, 60, 200], 3, 0, "logistic"),           # unsorted sizes
    (700, 1, 1, [20, 300, 699], 3, 0, "quantised"),          # ties, d_1 = 0
    (800, 5, 1, [30, 30, 500], 2, 0, "logistic"),            # repeated size
    (500, 4, 3, [80, 450], 3, 2, "logistic"),                # exclusion window
    (500, 2, 2, [60, 490], 3, -1, "gauss"),                  # query kept
    (2600, 10, 1, [100, 1000, 2591], 2, 0, "logistic"),      # several tiles per chain
])
def test_nested_vs_oracle(ctx, orc, N, E, tau, L, r, excl, kind):
    rng = np.random.default_rng(N + E)
    if kind == "logistic":
        X, Y = synth.coupled_logistic(N)
    elif kind == "quantised":
        X, Y = synth.quantised_series(N, 7, rng), synth.quantised_series(N, 5, rng)
    else:
        X, Y = rng.standard_normal(N), rng.standard_normal(N)
    gxy, gyx, gle = ctx.ccm(X, Y, E, tau, L, r, 21, exclusion_radius=excl, flags=NESTED)
    oxy, oyx, ole = orc.ccm_nested(X, Y, E, tau, L, r, 21, excl)
    assert np.array_equal(gle, ole)
    rho_close(gxy, oxy)
    rho_close(gyx, oyx)


def test_nested_sweep_vs_oracle_and_forms(ctx, orc):
    X, Y = synth.coupled_logistic(1500)
    E, tau, L, r = [1, 2, 4, 7], [1, 3], [40, 300, 1000, 1500], 3
    base = ctx.ccm_sweep(X, Y, E, tau, L, r, 8, flags=NESTED)
    for ie, e in enumerate(E):
        for it, t in enumerate(tau):
            oxy, oyx, _ = orc.ccm_nested(X, Y, e, t, L, r, 8)
            rho_close(base[0, ie, it], oxy)
            rho_close(base[1, ie, it], oyx)
    for flags in (capi.CCM_FLAG_NO_GRAPH, capi.CCM_FLAG_PERSISTENT):
        other = ctx.ccm_sweep(X, Y, E, tau, L, r, 8, flags=NESTED | flags)
        assert np.array_equal(base.view(np.uint64), other.view(np.uint64)), flags


def test_nested_full_library_equals_default(ctx):
    """At L = N_e every draw is the whole embedding, nested or not."""
    X, Y = synth.coupled_logistic(800)
    a = ctx.ccm(X, Y, 3, 1, [798], 3, 5, flags=NESTED)
    b = ctx.ccm(X, Y, 3, 1, [798], 3, 5)
    rho_close(a[0], b[0], 1e-12)
    rho_close(a[1], b[1], 1e-12)


def test_nested_work_and_invalid(ctx):
    X, Y = synth.coupled_logistic(2000)
    L = [100, 500, 1000, 1999]
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    ctx.ccm(X, Y, 2, 1, L, 2, 3, flags=NESTED)
    pn = ctx.profile_read(reset=True)
    ctx.ccm(X, Y, 2, 1, L, 2, 3)
    pi = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    assert pn["realizations"] == pi["realizations"] == 2 * len(L) * 2
    assert pn["pairs"] < 0.6 * pi["pairs"]            # N_e * max L vs N_e * sum L
    for kw in (dict(query_set=1, flags=NESTED),
               dict(flags=NESTED | capi.CCM_FLAG_TABLE),
               dict(flags=NESTED | capi.CCM_FLAG_PLAIN)):
        with pytest.raises(capi.CCMError) as ei:
            ctx.ccm(X, Y, 2, 1, L, 2, 3, **kw)
        assert ei.value.status == capi.CCM_E_INVAL
    S, _ = synth.logistic_network(3, 500, seed=5)
    with pytest.raises(capi.CCMError) as ei:
        ctx.ccm_matrix(S, 2, 1, [100], 2, 3, flags=NESTED)
    assert ei.value.status == capi.CCM_E_INVAL


def test_nested_full_sweep_sampled(ctx, orc):
    """The bench's nested call in full (N = 10^4, E = 1..10, tau = 1..5, 20 L,
    r = 250): sampled (E, tau) entries of its first two realizations at two
    library sizes against the oracle (an ordering depends on (seed, E, tau,
    r index) only, and a library is its prefix whatever the other sizes)."""
    w = synth.workload_sweep()
    got = ctx.ccm_sweep(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed, flags=NESTED)
    assert np.all(np.isfinite(got)) and np.all(np.abs(got) <= 1.0)
    picks = [(0, 0, (0, 19)), (3, 2, (5, 12)), (9, 4, (1, 8)), (6, 1, (10, 14))]
    with ThreadPoolExecutor(max_workers=len(picks)) as ex:
        outs = list(ex.map(lambda p: orc.ccm_nested(w.X, w.Y, w.E[p[0]], w.tau[p[1]],
                                                    [w.L[i] for i in p[2]], 2, w.seed), picks))
    for (ie, it, ils), (oxy, oyx, _) in zip(picks, outs):
        rho_close(got[0, ie, it, list(ils), :2], oxy)
        rho_close(got[1, ie, it, list(ils), :2], oyx)


def test_nested_minimum_sizes_and_constant_series(ctx, orc):
    """Boundaries: N_e = E + 2 (N = 42, E = 4, tau = 12) with L at the
    minimum and clamped (one segment); a constant series, whose predictions
    have no variance (rho NaN where the oracle's is)."""
    rng = np.random.default_rng(43)
    X, Y = synth.coupled_logistic(42, *rng.uniform(0.1, 0.9, 2))
    gxy, gyx, gle = ctx.ccm(X, Y, 4, 12, [6, 40], 3, 7, flags=NESTED)
    oxy, oyx, ole = orc.ccm_nested(X, Y, 4, 12, [6, 40], 3, 7)
    assert gle.tolist() == ole.tolist() == [6, 6]
    rho_close(gxy, oxy)
    rho_close(gyx, oyx)
    C = np.full(300, 0.25)
    Z = rng.standard_normal(300)
    gxy, gyx, _ = ctx.ccm(C, Z, 3, 2, [50, 296], 2, 9, flags=NESTED)
    oxy, oyx, _ = orc.ccm_nested(C, Z, 3, 2, [50, 296], 2, 9)
    assert np.isnan(oxy).any() or np.isnan(oyx).any()
    rho_close(gxy, oxy)
    rho_close(gyx, oyx)
