"""E-sweep sharing (CCM_FLAG_SHARED_E) against the oracle's shared-E mode.

Every E of a sweep is the default cross map of the series shifted by
(E_max - E) tau over the N_c points of E_max's embedding, with one library
per (tau, L, r) keyed by E = 0; the kernel computes all of them from one scan.
rho must agree with the oracle within 1e-5 (the build's tolerance) for every
E, tau, L and r, including E lists with gaps, repeats and no order, ties,
every exclusion mode and tiles with a ragged tail; at the full library every
E equals the default path on the shifted series; the batched forms agree bit
for bit; invalid combinations are rejected.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1905_00565_amd import capi, synth

pytestmark = pytest.mark.gpu
SHARED = capi.CCM_FLAG_SHARED_E
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


def oracle_sweep(orc, X, Y, E, tau, L, r, seed, excl=0):
    """rho[2][nE][ntau][nL][r] from the oracle, one call per (tau, L) in threads
    (the libraries of one L do not depend on the others)."""
    out = np.empty((2, len(E), len(tau), len(L), r))
    le = np.empty((len(tau), len(L)), dtype=np.int64)
    jobs = [(it, il) for it in range(len(tau)) for il in range(len(L))]

    def one(job):
        it, il = job
        return job, orc.ccm_shared_e(X, Y, E, tau[it], [L[il]], r, seed, excl)

    with ThreadPoolExecutor(max_workers=8) as ex:
        for (it, il), (rxy, ryx, l_eff) in ex.map(one, jobs):
            out[0, :, it, il] = rxy[:, 0]
            out[1, :, it, il] = ryx[:, 0]
            le[it, il] = l_eff[0]
    return out, le


def series(kind, n, rng):
    if kind == "logistic":
        return synth.coupled_logistic(n, *rng.uniform(0.1, 0.9, 2))
    if kind == "quantised":
        return synth.quantised_series(n, 7, rng), synth.quantised_series(n, 5, rng)
    return rng.standard_normal(n), rng.standard_normal(n)


# (N, E list, tau list, L, r, exclusion radius, kind)
CASES = [
    (1200, [1, 2, 3], [1], [20, 300, 1200], 3, 0, "logistic"),
    (1500, [10, 1, 4, 7], [1, 3], [60, 700, 1500], 2, 0, "logistic"),   # gaps, unordered
    (900, [2, 5, 5, 3], [2], [40, 899], 2, 0, "logistic"),              # repeated E
    (800, [1, 2, 3], [1], [30, 400, 800], 3, 0, "quantised"),           # ties, d_1 = 0
    (700, [1, 3, 6], [2], [80, 650], 2, 3, "logistic"),                 # exclusion window
    (700, [2, 4], [1, 2], [50, 690], 2, -1, "gauss"),                   # query kept
    (2600, list(range(1, 11)), [1], [100, 1000, 2600], 2, 0, "logistic"),  # several tiles
]


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[0]}-E{c[1]}-tau{c[2]}-x{c[5]}-{c[6]}"
                                             for c in CASES])
def test_shared_e_vs_oracle(ctx, orc, case):
    N, E, tau, L, r, excl, kind = case
    rng = np.random.default_rng(N + 7 * len(E) + excl)
    X, Y = series(kind, N, rng)
    got = ctx.ccm_sweep(X, Y, E, tau, L, r, 17, exclusion_radius=excl, flags=SHARED)
    want, _ = oracle_sweep(orc, X, Y, E, tau, L, r, 17, excl)
    rho_close(got, want)


def test_shared_e_single_call_and_leff(ctx, orc):
    X, Y = synth.coupled_logistic(1000)
    gxy, gyx, gle = ctx.ccm(X, Y, 4, 3, [30, 500, 2000], 3, 9, flags=SHARED)
    oxy, oyx, ole = orc.ccm_shared_e(X, Y, [4], 3, [30, 500, 2000], 3, 9)
    assert np.array_equal(gle, ole) and gle[-1] == 1000 - 3 * 3
    rho_close(gxy, oxy[0])
    rho_close(gyx, oyx[0])


def test_shared_e_full_library_equals_shifted_default(ctx):
    """At L = N_c every draw is every common point: E's rho is the default
    cross map of the series shifted by (E_max - E) tau."""
    N, tau, Emax = 1400, 2, 6
    X, Y = synth.coupled_logistic(N)
    nc = N - (Emax - 1) * tau
    E = [1, 3, 6]
    got = ctx.ccm_sweep(X, Y, E, [tau], [nc], 2, 3, flags=SHARED)
    for ie, e in enumerate(E):
        d = (Emax - e) * tau
        a = ctx.ccm(X[d:], Y[d:], e, tau, [nc], 2, 3)
        rho_close(got[0, ie, 0], a[0], 1e-12)
        rho_close(got[1, ie, 0], a[1], 1e-12)


def test_shared_e_forms_bitwise(ctx):
    X, Y = synth.coupled_logistic(3000)
    E, tau, L = [1, 2, 5, 8], [1, 2], [50, 600, 3000]
    base = ctx.ccm_sweep(X, Y, E, tau, L, 3, 8, flags=SHARED)
    for flags in (capi.CCM_FLAG_NO_GRAPH, capi.CCM_FLAG_PERSISTENT):
        other = ctx.ccm_sweep(X, Y, E, tau, L, 3, 8, flags=SHARED | flags)
        assert np.array_equal(base.view(np.uint64), other.view(np.uint64)), flags
    again = ctx.ccm_sweep(X, Y, E, tau, L, 3, 8, flags=SHARED)
    assert np.array_equal(base.view(np.uint64), again.view(np.uint64))


def test_shared_e_work_and_invalid(ctx):
    X, Y = synth.coupled_logistic(2000)
    E, L = [1, 2, 3, 4], [100, 1000, 1990]
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    ctx.ccm_sweep(X, Y, E, [1], L, 2, 3, flags=SHARED)
    ps = ctx.profile_read(reset=True)
    ctx.ccm_sweep(X, Y, E, [1], L, 2, 3)
    pi = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    assert ps["realizations"] == pi["realizations"] == 2 * len(E) * len(L) * 2
    assert ps["pairs"] < 0.3 * pi["pairs"]          # one scan for the four E
    for kw in (dict(query_set=1, flags=SHARED),
               dict(flags=SHARED | capi.CCM_FLAG_TABLE),
               dict(flags=SHARED | capi.CCM_FLAG_NESTED),
               dict(flags=SHARED | capi.CCM_FLAG_PLAIN)):
        with pytest.raises(capi.CCMError) as ei:
            ctx.ccm_sweep(X, Y, E, [1], L, 2, 3, **kw)
        assert ei.value.status == capi.CCM_E_INVAL
    # the rules of E_max apply: L >= E_max + 2 and N_c >= E_max + 2
    with pytest.raises(capi.CCMError):
        ctx.ccm_sweep(X, Y, [1, 10], [1], [11], 1, 3, flags=SHARED)
    with pytest.raises(capi.CCMError):
        ctx.ccm_sweep(X[:40], Y[:40], [1, 10], [4], [20], 1, 3, flags=SHARED)
    S, _ = synth.logistic_network(3, 500, seed=5)
    with pytest.raises(capi.CCMError) as ei:
        ctx.ccm_matrix(S, 2, 1, [100], 2, 3, flags=SHARED)
    assert ei.value.status == capi.CCM_E_INVAL


def test_shared_e_long_series_sample(ctx, orc):
    """N = 10^5 (noisy series, 390 query tiles): every rho of three E and two
    library sizes against the oracle."""
    w = synth.workload_long(r=1)
    E = [1, 3, 10]
    L = [500, 2000]
    got = ctx.ccm_sweep(w.X, w.Y, E, [2], L, 1, w.seed, flags=SHARED)
    assert np.all(np.isfinite(got)) and np.all(np.abs(got) <= 1.0)
    want, _ = oracle_sweep(orc, w.X, w.Y, E, [2], L, 1, w.seed)
    rho_close(got, want)


def test_shared_e_full_sweep_sampled(ctx, orc):
    """The bench's shared-E call in full (N = 10^4, E = 1..10, tau = 1..5, 20 L,
    r = 250): sampled (tau, L) entries of its first two realizations against
    the oracle (a realization's library depends on its index, not on r); every
    value finite and within [-1, 1]."""
    w = synth.workload_sweep()
    got = ctx.ccm_sweep(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed, flags=SHARED)
    assert got.shape == (2, 10, 5, len(w.L), w.r)
    assert np.all(np.isfinite(got)) and np.all(np.abs(got) <= 1.0)
    picks = [(0, 0), (2, 9), (4, 13), (1, 15)]      # (tau index, L index)
    with ThreadPoolExecutor(max_workers=len(picks)) as ex:
        outs = list(ex.map(lambda p: orc.ccm_shared_e(w.X, w.Y, w.E, w.tau[p[0]], [w.L[p[1]]],
                                                       2, w.seed), picks))
    for (it, il), (rxy, ryx, _) in zip(picks, outs):
        rho_close(got[0, :, it, il, :2], rxy[:, 0, :])
        rho_close(got[1, :, it, il, :2], ryx[:, 0, :])


def test_shared_e_minimum_sizes_and_constant_series(ctx, orc):
    """Boundaries: N_c = E_max + 2 at the largest tau (N = 42, E_max = 4,
    tau = 12) with L at the minimum and clamped; a constant series, whose
    predictions have no variance (rho NaN where the oracle's is)."""
    rng = np.random.default_rng(42)
    X, Y = synth.coupled_logistic(42, *rng.uniform(0.1, 0.9, 2))
    E, tau, L = [1, 2, 4], [1, 12], [6, 40]
    got = ctx.ccm_sweep(X, Y, E, tau, L, 3, 7, flags=SHARED)
    want, le = oracle_sweep(orc, X, Y, E, tau, L, 3, 7)
    assert le[1].tolist() == [6, 6]
    rho_close(got, want)
    C = np.full(300, 0.25)
    Z = rng.standard_normal(300)
    got = ctx.ccm_sweep(C, Z, [1, 3], [2], [50, 296], 2, 9, flags=SHARED)
    want, _ = oracle_sweep(orc, C, Z, [1, 3], [2], [50, 296], 2, 9)
    assert np.isnan(want).any()
    rho_close(got, want)
