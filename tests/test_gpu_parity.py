"""GPU path (through the C ABI) against the CPU oracle.

Neighbour indices and squared distances must match bit for bit; predictions
and rho within 1e-5 absolute (the accuracy the build targets; in practice the
two differ by rounding order only, ~1e-15).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1905_00565_amd import capi, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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
    nan_a, nan_b = np.isnan(a), np.isnan(b)
    assert np.array_equal(nan_a, nan_b)
    if (~nan_a).any():
        err = np.max(np.abs(a[~nan_a] - b[~nan_a]))
        assert err < tol, err


def test_sampler_bit_exact(ctx, orc):
    keys = [(1, 2, 1, 100, 0, 999), (2, 10, 5, 7848, 249, 9955), (3, 3, 2, 50000, 17, 99996),
            (12345678901234, 1, 1, 5, 3, 7), (5, 4, 1, 19997, 99, 19997), (9, 7, 3, 2, 1, 3),
            # one candidate; chunk edges of the sampler's 64-candidate steps; all taken
            (7, 2, 1, 1, 0, 1), (7, 2, 1, 1, 0, 64), (7, 2, 1, 63, 0, 64), (7, 2, 1, 64, 5, 65),
            (8, 3, 2, 127, 4, 128), (8, 3, 2, 3, 4, 129), (2**63 + 5, 5, 4, 300, 7, 1000),
            (11, 6, 2, 5000, 3, 5000)]
    rng = np.random.default_rng(77)
    for _ in range(40):
        ne = int(rng.integers(1, 20000))
        keys.append((int(rng.integers(0, 2**63)), int(rng.integers(1, 11)),
                     int(rng.integers(1, 6)), int(rng.integers(1, ne + 1)),
                     int(rng.integers(0, 300)), ne))
    for seed, E, tau, le, ri, ne in keys:
        g = ctx.ccm_library(ne, E, tau, le, ri, seed)
        o = orc.sample_library(seed, E, tau, le, ri, ne)
        assert np.array_equal(g, o), (seed, E, tau, le, ri, ne)


def test_golden_dyadic_neighbors(ctx):
    g = json.load(open(os.path.join(GOLDEN, "dyadic_e2_neighbors.json")))
    S = np.asarray(g["series_times_8"], dtype=np.float64) / 8.0
    T = np.arange(len(S), dtype=np.float64)
    for case in g["cases"]:
        nbr, d2, _, _ = ctx.ccm_neighbors(S, T, g["E"], g["tau"], case["library"],
                                          exclusion_radius=case["exclusion_radius"])
        assert nbr.tolist() == case["neighbors"], case["name"]
        want = np.asarray(case["d2_times_64"], dtype=np.float32) / np.float32(64)
        assert np.array_equal(d2, want), case["name"]


def _fuzz_cases():
    rng = np.random.default_rng(2024)
    cases = []
    for n in range(40):
        E = 1 + n % 10
        tau = 1 + (n // 10) % 3
        N = int(rng.integers((E - 1) * tau + E + 12, 300))
        kind = n % 4
        cases.append((n, E, tau, N, kind))
    return cases


@pytest.mark.parametrize("n,E,tau,N,kind", _fuzz_cases())
def test_neighbors_fuzz(ctx, orc, n, E, tau, N, kind):
    rng = np.random.default_rng(1000 + n)
    if kind == 0:
        S = rng.random(N)
    elif kind == 1:
        S = synth.quantised_series(N, 5, rng)          # ties and d_1 = 0
    elif kind == 2:
        S = synth.dyadic_series(N, rng)
    else:
        S = rng.standard_normal(N) * 1e3
    T = rng.random(N)
    ne = N - (E - 1) * tau
    excl = [0, -1, 2, 0][n % 4]
    qs = (n // 4) % 2
    lo = E + 2 + (2 * excl + 1 if excl > 0 else 0)
    L = int(rng.integers(lo, ne + 1))
    lib = np.sort(rng.choice(ne, size=L, replace=False)).astype(np.int32)
    g = ctx.ccm_neighbors(S, T, E, tau, lib, exclusion_radius=excl, query_set=qs)
    o = orc.neighbors(S, T, E, tau, lib, excl=excl, query_set=qs)
    assert np.array_equal(g[0], o[0]), "neighbour indices differ"
    assert np.array_equal(g[1], o[1]), "squared distances differ"
    assert np.max(np.abs(g[2] - o[2])) < TOL
    rho_close(g[3], o[3])


def test_neighbors_tile_boundaries(ctx, orc):
    # query counts around the tile size (256 queries per tile here) and a
    # ragged library tail for every group size
    rng = np.random.default_rng(7)
    for ne in (255, 256, 257, 511, 513):
        for E in (1, 3, 6):
            N = ne + E - 1
            S = rng.random(N)
            T = rng.random(N)
            for L in (E + 2, E + 3, 37, ne):
                lib = np.sort(rng.choice(ne, size=L, replace=False)).astype(np.int32)
                g = ctx.ccm_neighbors(S, T, E, 1, lib)
                o = orc.neighbors(S, T, E, 1, lib)
                assert np.array_equal(g[0], o[0]) and np.array_equal(g[1], o[1]), (ne, E, L)
                assert np.max(np.abs(g[2] - o[2])) < TOL
                rho_close(g[3], o[3])


def test_neighbors_every_small_library(ctx, orc):
    """Every library size from E + 2 to E + 73 for E = 1..5 (the outward
    scan's one-sided remainder is software-pipelined there): odd and even
    numbers of remaining groups on either side, scan starts at both ends and
    inside, and the single-position tails.  Bit-exact neighbours."""
    rng = np.random.default_rng(23)
    for E in range(1, 6):
        N = 180 + E
        ne = N - (E - 1)
        S = rng.random(N)
        T = rng.random(N)
        for L in range(E + 2, E + 74):
            lib = np.sort(rng.choice(ne, size=L, replace=False)).astype(np.int32)
            g = ctx.ccm_neighbors(S, T, E, 1, lib)
            o = orc.neighbors(S, T, E, 1, lib)
            assert np.array_equal(g[0], o[0]) and np.array_equal(g[1], o[1]), (E, L)
            assert np.max(np.abs(g[2] - o[2])) < TOL


def test_small_workload_full(ctx, orc):
    """Coupled logistic N=1000, E=2, tau=1, L=100..1000, r=100: every rho."""
    w = synth.workload_small()
    gxy, gyx, gle = ctx.ccm(w.X, w.Y, 2, 1, w.L, w.r, w.seed)
    oxy, oyx = orc.ccm_threaded(w.X, w.Y, 2, 1, w.L, w.r, w.seed)
    assert gle.tolist() == [min(l, 999) for l in w.L]
    rho_close(gxy, oxy)
    rho_close(gyx, oyx)
    # known behaviour: X from M_Y dominates and converges
    assert np.all(gxy.mean(1) > gyx.mean(1))


def test_sweep_small_all_E_tau(ctx, orc):
    x, y = synth.coupled_logistic(700)
    E = list(range(1, 11))
    tau = [1, 2, 3]
    L = [12, 50, 333, 700]
    r = 3
    g = ctx.ccm_sweep(x, y, E, tau, L, r, 11)
    for ie, e in enumerate(E):
        for it, t in enumerate(tau):
            oxy, oyx = orc.ccm_threaded(x, y, e, t, L, r, 11)
            rho_close(g[0, ie, it], oxy)
            rho_close(g[1, ie, it], oyx)


@pytest.mark.parametrize("excl,qs", [(-1, 0), (3, 0), (0, 1), (-1, 1)])
def test_ccm_options(ctx, orc, excl, qs):
    x, y = synth.coupled_logistic(500)
    L = [30, 120, 500]
    g = ctx.ccm(x, y, 3, 2, L, 4, 5, exclusion_radius=excl, query_set=qs)
    o = orc.ccm(x, y, 3, 2, L, 4, 5, excl=excl, query_set=qs)
    rho_close(g[0], o[0])
    rho_close(g[1], o[1])


def test_forms_bitwise_equal(ctx):
    """Plain per-realization launches, batched (graph / no graph / persistent)
    and repeated calls give bitwise-identical rho."""
    x, y = synth.coupled_logistic(900)
    args = (x, y, [1, 4, 7], [1, 2], [40, 300, 900], 5, 99)
    ref = ctx.ccm_sweep(*args)
    for flags in (capi.CCM_FLAG_NO_GRAPH, capi.CCM_FLAG_PLAIN, capi.CCM_FLAG_PERSISTENT,
                  capi.CCM_FLAG_PERSISTENT | capi.CCM_FLAG_NO_GRAPH, 0):
        got = ctx.ccm_sweep(*args, flags=flags)
        assert np.array_equal(ref, got, equal_nan=True), flags
    again = ctx.ccm_sweep(*args)
    assert np.array_equal(ref, again, equal_nan=True)


def test_device_forms(ctx):
    import torch
    x, y = synth.coupled_logistic(800)
    E, tau, L, r = [2, 5], [1, 3], [50, 800], 4
    ref = ctx.ccm_sweep(x, y, E, tau, L, r, 3)
    dx = torch.tensor(x, device="cuda:0")
    dy = torch.tensor(y, device="cuda:0")
    out = torch.empty(ref.shape, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.current_stream()
    ctx.ccm_sweep_dev(dx, dy, E, tau, L, r, 3, out, stream=s)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref, equal_nan=True)
    rxy = torch.empty((len(L), r), dtype=torch.float64, device="cuda:0")
    ryx = torch.empty_like(rxy)
    le = ctx.ccm_dev(dx, dy, 5, 3, L, r, 3, rxy, ryx, stream=s)
    torch.cuda.synchronize()
    assert le.tolist() == [50, 788]
    assert np.array_equal(rxy.cpu().numpy(), ref[0, 1, 1], equal_nan=True)
    assert np.array_equal(ryx.cpu().numpy(), ref[1, 1, 1], equal_nan=True)


def test_invalid_inputs(ctx):
    x, y = synth.coupled_logistic(50)
    bad = [
        dict(E=0, tau=1, L=[10]), dict(E=11, tau=1, L=[20]), dict(E=2, tau=0, L=[10]),
        dict(E=2, tau=1, L=[3]), dict(E=2, tau=49, L=[10]),
        dict(E=2, tau=1, L=[10], exclusion_radius=20),
    ]
    for b in bad:
        kw = dict(b)
        E, tau, L = kw.pop("E"), kw.pop("tau"), kw.pop("L")
        with pytest.raises(capi.CCMError) as ei:
            ctx.ccm(x, y, E, tau, L, 2, 1, **kw)
        assert ei.value.status == capi.CCM_E_INVAL, b
    xn = x.copy()
    xn[5] = np.inf
    with pytest.raises(capi.CCMError):
        ctx.ccm(xn, y, 2, 1, [10], 2, 1)
    with pytest.raises(capi.CCMError):
        ctx.ccm(x, y, 2, 1, [10], 0, 1)
    # clamping is not an error
    _, _, le = ctx.ccm(x, y, 2, 1, [10**6], 1, 1)
    assert le.tolist() == [49]


def test_profiled_launches(ctx):
    """While profiling, every cross-map launch is timed (direct launches);
    results equal the graph path's, bit for bit."""
    x, y = synth.coupled_logistic(3000)
    args = (x, y, [2, 7], [1, 3], [100, 3000], 6, 21)
    ref = ctx.ccm_sweep(*args)
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    a = ctx.ccm_sweep(*args)
    b = ctx.ccm_sweep(*args, flags=capi.CCM_FLAG_PERSISTENT)
    p = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    for got in (a, b):
        assert np.array_equal(ref, got, equal_nan=True)
    assert p["launches"] == 4 and p["waves"] == 2        # one launch per E, per call
    assert p["kernel_ms"] > 0 and p["realizations"] == 2 * ref.size
