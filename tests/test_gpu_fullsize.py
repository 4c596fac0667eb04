"""The workloads at full size against the oracle, on the kernel instances the
batched calls launch.

The per-query hook (ccm_neighbors) runs the cross-map kernel with the batched
launches' queries per lane, candidate groups, query tiles, scan order and
moment merge order; only its export of every query's neighbours after the
scan differs.  So the hook's rho for a realization must equal, bit for bit,
the rho the batched call produced for it -- which ties the neighbours the
hook exports (checked bit for bit against the oracle at sampled queries) to
the batched launch.

Bars: neighbour indices and binary32 squared distances bit-exact, predictions
and rho within 1e-5 of the FP64 oracle.  Coverage: every E = 1..10 of the
sweep at tau = 1 and 5 (256 sampled queries each, small and large
libraries); one realization in every (E, tau, L) cell of the sweep, with the
direction alternating; every L of the long series (two realizations each, the
full library included); every L of the causal matrix (two ordered pairs
each).
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
    c.close()


@pytest.fixture(scope="module")
def sweep(ctx):
    """The bench's sweep (N = 10^4, E = 1..10, tau = 1..5, 20 L, r = 250) in
    its default launch configuration (batched, graph)."""
    w = synth.workload_sweep()
    rho = ctx.ccm_sweep(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed)
    return w, rho


def close(a, b, tol=TOL):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    assert a.shape == b.shape
    assert np.array_equal(np.isnan(a), np.isnan(b))
    m = ~np.isnan(a)
    if m.any():
        err = np.max(np.abs(a[m] - b[m]))
        assert err < tol, err


def bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def hook_vs_oracle(ctx, orc, S, T, E, tau, lib, n_queries, rng):
    """Hook outputs of one library: sampled queries bit-exact against the
    oracle; returns the hook's rho."""
    ne = len(S) - (E - 1) * tau
    nbr, d2, pred, rho = ctx.ccm_neighbors(S, T, E, tau, lib)
    q = np.sort(rng.choice(ne, size=min(n_queries, ne), replace=False))
    on, od, op = orc.neighbors_at(S, T, E, tau, lib, q)
    assert np.array_equal(nbr[q], on), "neighbour indices differ from the oracle"
    assert np.array_equal(bits(d2[q]), bits(od)), "squared distances differ from the oracle"
    close(pred[q], op)
    return rho


@pytest.mark.parametrize("E", list(range(1, 11)))
def test_sweep_benched_instance_every_E(ctx, orc, sweep, E):
    """Per E, tau in {1, 5}: a small and a large library of the sweep through
    the hook -- the library draw equals the oracle's, 256 sampled queries
    have the oracle's neighbours and distances bit for bit, and the hook's
    rho equals the batched sweep's rho of that realization bit for bit."""
    w, rho = sweep
    rng = np.random.default_rng(500 + E)
    for tau in (1, 5):
        ne = w.N - (E - 1) * tau
        for il in ((3 * E + tau) % 10, 10 + (E + tau) % 10):
            ri = (37 * E + 11 * tau + il) % w.r
            d = (E + il) % 2
            le = min(w.L[il], ne)
            lib = ctx.ccm_library(ne, E, tau, le, ri, w.seed)
            assert np.array_equal(lib, orc.sample_library(w.seed, E, tau, le, ri, ne))
            S, T = (w.Y, w.X) if d == 0 else (w.X, w.Y)
            h = hook_vs_oracle(ctx, orc, S, T, E, tau, lib, 256, rng)
            got = rho[d, E - 1, tau - 1, il, ri]
            assert np.float64(h).view(np.uint64) == np.float64(got).view(np.uint64), \
                (E, tau, il, ri, d, h, got)


def test_sweep_every_cell_vs_oracle(orc, sweep):
    """One realization in each of the sweep's 1000 (E, tau, L) cells against
    the oracle, directions alternating, r drawn per cell."""
    w, rho = sweep
    assert np.isfinite(rho).all()
    rng = np.random.default_rng(77)
    picks, tasks = [], []
    for ie, e in enumerate(w.E):
        for it, t in enumerate(w.tau):
            for il, l in enumerate(w.L):
                d = (ie + it + il) % 2
                ri = int(rng.integers(w.r))
                S, T = (w.Y, w.X) if d == 0 else (w.X, w.Y)
                picks.append((d, ie, it, il, ri))
                tasks.append((S, T, e, t, l, ri, w.seed, 0, 0))
    want = orc.realizations_threaded(tasks)
    close([rho[p] for p in picks], want)
    # L = 10^4 clamps to N_e: every r of that cell is the same full library
    full = rho[:, :, :, -1, :]
    assert np.array_equal(full, np.repeat(full[..., :1], w.r, axis=-1))


def test_long_series_every_L(ctx, orc):
    """Noisy coupled logistic map, N = 10^5, E = 3, tau = 2, r = 250: two
    realizations at each of the four library sizes (both directions),
    the hook at 256 sampled queries of L = 5*10^4 and of the full library."""
    w = synth.workload_long()
    rxy, ryx, le = ctx.ccm(w.X, w.Y, 3, 2, w.L, w.r, w.seed)
    assert le.tolist() == [1000, 10000, 50000, 99996]
    assert np.isfinite(rxy).all() and np.isfinite(ryx).all()
    picks = [(0, 0, 5), (1, 0, 200), (0, 1, 17), (1, 1, 131), (0, 2, 42), (1, 2, 249),
             (0, 3, 0), (1, 3, 248)]
    for d, il, ri in picks:
        S, T = (w.Y, w.X) if d == 0 else (w.X, w.Y)
        want = orc.realization_split(S, T, 3, 2, w.L[il], ri, w.seed)
        got = (rxy if d == 0 else ryx)[il, ri]
        assert abs(got - want) < TOL, (d, il, ri, got, want)
    rng = np.random.default_rng(3)
    ne = 99996
    for il, ri in ((2, 42), (3, 0)):
        lib = ctx.ccm_library(ne, 3, 2, le[il], ri, w.seed)
        assert np.array_equal(lib, orc.sample_library(w.seed, 3, 2, le[il], ri, ne))
        h = hook_vs_oracle(ctx, orc, w.Y, w.X, 3, 2, lib, 256, rng)
        assert np.float64(h).view(np.uint64) == np.float64(rxy[il, ri]).view(np.uint64)


def test_matrix_every_L(ctx, orc):
    """64-series logistic network, N = 2*10^4, E = 4, tau = 1, r = 100: two
    ordered pairs at each of the ten library sizes, and the hook on one
    library series at the largest size."""
    m = synth.workload_matrix()
    S = m["S"]
    M = S.shape[0]
    rho = ctx.ccm_matrix(S, m["E"], m["tau"], m["L"], m["r"], m["seed"])
    off = ~np.eye(M, dtype=bool)
    assert np.isfinite(rho[off]).all() and np.isnan(rho[~off]).all()
    rng = np.random.default_rng(55)
    picks, tasks = [], []
    for il, l in enumerate(m["L"]):
        for _ in range(2):
            a, b = rng.choice(M, 2, replace=False)
            ri = int(rng.integers(m["r"]))
            picks.append((a, b, il, ri))
            tasks.append((S[a], S[b], m["E"], m["tau"], l, ri, m["seed"], 0, 0))
    close([rho[p] for p in picks], orc.realizations_threaded(tasks))
    ne = S.shape[1] - (m["E"] - 1) * m["tau"]
    le = min(m["L"][-2], ne)
    lib = ctx.ccm_library(ne, m["E"], m["tau"], le, 9, m["seed"])
    h = hook_vs_oracle(ctx, orc, S[7], S[30], m["E"], m["tau"], lib, 256,
                       np.random.default_rng(6))
    assert abs(h - rho[7, 30, len(m["L"]) - 2, 9]) < 1e-12


def test_sweep_deterministic_sample_vs_oracle(orc, sweep):
    """The sample the bench times the oracle on (realizations whose library
    stream state is 0 mod 1000, both directions) against the sweep's rho."""
    w, rho = sweep
    tasks, picks = orc.deterministic_sample(w.X, w.Y, w.E, w.tau, w.L, w.r, w.seed, 1000)
    assert len(tasks) > 400
    close([rho[p] for p in picks], orc.realizations_threaded(tasks))
