"""Pins that tie the CPU oracle to facts outside itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with what the paper, the mathematics or a textbook
routine fixes.  ``test_oracle_pins.py`` runs them against the real oracle;
``test_oracle_mutants.py`` runs them against deliberately broken builds to show
that each plausible mistake is caught by at least one pin.

What each pin rests on:

* hand enumeration of a dyadic example (every binary32 operation exact);
* closed forms for a ramp series (E=1 and E=2);
* a textbook routine: numpy's stable argsort for E=1 neighbours, numpy's
  corrcoef for Pearson;
* brute force with an exact, independently written binary32 FMA (Python
  fractions) on tiny random inputs;
* special cases: self-map with the query kept gives rho = 1; zero-distance
  neighbours share the weight equally;
* invariances: affine target, power-of-two scaling of the library series,
  full-library realizations independent of the draw;
* known behaviour: the coupled logistic map's asymmetric convergence;
* the sampler's published generator (SplitMix64 known-answer values) and the
  statistical properties of selection sampling.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
from scipy import stats

from paper_1905_00565_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# exact binary32 arithmetic, written independently of the oracle
# ---------------------------------------------------------------------------

def f32_round(x: Fraction) -> float:
    """Round an exact rational to the nearest binary32 (ties to even)."""
    if x == 0:
        return 0.0
    sign = -1.0 if x < 0 else 1.0
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    ulp_e = max(e - 23, -149)
    scaled = a / (Fraction(2) ** ulp_e)
    q, r = divmod(scaled.numerator, scaled.denominator)
    if 2 * r > scaled.denominator or (2 * r == scaled.denominator and q % 2 == 1):
        q += 1
    return sign * math.ldexp(float(q), ulp_e)


def exact_sqdist(S32, ti, tj, E, tau):
    acc = 0.0
    for k in range(E):
        diff = f32_round(Fraction(float(S32[ti - k * tau])) - Fraction(float(S32[tj - k * tau])))
        acc = f32_round(Fraction(diff) * Fraction(diff) + Fraction(acc))
    return acc


def brute_neighbors(S, E, tau, lib, excl, query_set=0):
    """Neighbours by listing every candidate and sorting by (d2, j)."""
    S32 = np.asarray(S, dtype=np.float32)
    off = (E - 1) * tau
    Ne = len(S) - off
    queries = list(lib) if query_set else list(range(Ne))
    out_n, out_d = [], []
    for i in queries:
        cands = []
        for j in lib:
            if excl >= 0 and abs(int(j) - int(i)) <= excl:
                continue
            cands.append((exact_sqdist(S32, i + off, int(j) + off, E, tau), int(j)))
        cands.sort()
        out_n.append([c[1] for c in cands[:E + 1]])
        out_d.append([c[0] for c in cands[:E + 1]])
    return np.array(out_n, dtype=np.int32), np.array(out_d, dtype=np.float32)


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def pin_golden_dyadic(orc):
    """Hand-enumerated neighbours of a dyadic series (Section 3.2 definition)."""
    with open(os.path.join(GOLDEN, "dyadic_e2_neighbors.json")) as f:
        g = json.load(f)
    S = np.asarray(g["series_times_8"], dtype=np.float64) / 8.0
    T = np.arange(len(S), dtype=np.float64)
    for case in g["cases"]:
        nbr, d2, _, _ = orc.neighbors(S, T, g["E"], g["tau"], case["library"],
                                      excl=case["exclusion_radius"])
        assert nbr.tolist() == case["neighbors"], case["name"]
        want = np.asarray(case["d2_times_64"], dtype=np.float32) / np.float32(64)
        assert np.array_equal(d2, want), case["name"]


def _ramp_rho(t_obs, t_hat):
    return float(np.corrcoef(t_obs, t_hat)[0, 1])


def pin_ramp_e1(orc):
    """S = T = t, E=1, full library: interior prediction t, endpoints closed form."""
    N = 40
    t = np.arange(N, dtype=np.float64)
    e = math.e
    want = t.copy()
    want[0] = (e + 2) / (e + 1)
    want[-1] = N - 2 - 1 / (e + 1)
    _, _, pred, rho = orc.neighbors(t, t, 1, 1, np.arange(N))
    assert np.max(np.abs(pred - want)) < 1e-12
    assert abs(rho - _ramp_rho(t, want)) < 1e-12


def pin_ramp_e2(orc):
    """S = T = t, E=2, tau=1: neighbours (t-1, t+1, t-2) in the interior."""
    N = 40
    t = np.arange(N, dtype=np.float64)
    e = math.e
    times = np.arange(1, N)               # time of embedded point i is i+1
    want = times - 2 / (2 * e + 1)
    em1, em2, em3 = math.exp(-1), math.exp(-2), math.exp(-3)
    want[0] = (2 * em1 + 3 * em2 + 4 * em3) / (em1 + em2 + em3)        # t = 1
    want[1] = (4 * e + 4) / (2 * e + 1)                                 # t = 2
    want[-1] = ((N - 2) * em1 + (N - 3) * em2 + (N - 4) * em3) / (em1 + em2 + em3)
    nbr, _, pred, rho = orc.neighbors(t, t, 2, 1, np.arange(N - 1))
    # interior neighbour order: t-1, t+1, t-2  (embedded index = time - 1)
    i = 10
    assert nbr[i].tolist() == [i - 1, i + 1, i - 2]
    assert np.max(np.abs(pred - want)) < 1e-12
    assert abs(rho - _ramp_rho(times.astype(float), want)) < 1e-12


def pin_e1_stable_argsort(orc):
    """E=1 neighbours equal numpy's stable argsort of binary32 |d|^2."""
    rng = np.random.default_rng(11)
    for trial in range(6):
        N = int(rng.integers(20, 120))
        S = rng.random(N) if trial % 2 else synth.quantised_series(N, 7, rng)
        T = rng.random(N)
        lib = np.sort(rng.choice(N, size=int(rng.integers(3, N)), replace=False))
        nbr, d2, _, _ = orc.neighbors(S, T, 1, 1, lib)
        S32 = S.astype(np.float32)
        for i in range(N):
            cand = lib[lib != i]
            d = S32[i] - S32[cand]
            dd = (d * d).astype(np.float32)
            order = np.argsort(dd, kind="stable")      # cand ascending: ties keep lower j
            assert nbr[i].tolist() == cand[order[:2]].tolist()
            assert np.array_equal(d2[i], dd[order[:2]])


def pin_exact_fma_bruteforce(orc):
    """E=2..4 neighbours and d2 equal exact-FMA brute force on tiny inputs."""
    rng = np.random.default_rng(12)
    for trial in range(6):
        E = 2 + trial % 3
        tau = 1 + trial % 2
        N = int(rng.integers(14, 26))
        S = rng.random(N) * 3 - 1
        Ne = N - (E - 1) * tau
        lib = np.sort(rng.choice(Ne, size=int(rng.integers(E + 3, Ne + 1)), replace=False))
        excl = [0, -1, 1][trial % 3]
        if excl == 1 and len(lib) < E + 4:
            excl = 0
        nbr, d2, _, _ = orc.neighbors(S, S, E, tau, lib, excl=excl)
        bn, bd = brute_neighbors(S, E, tau, lib, excl)
        assert np.array_equal(nbr, bn), (trial, nbr, bn)
        assert np.array_equal(d2, bd), trial


def pin_query_set_library(orc):
    """Library-only queries: neighbours of each library point, in library order."""
    rng = np.random.default_rng(13)
    S = rng.random(30)
    lib = np.sort(rng.choice(28, size=12, replace=False))
    nbr, d2, _, _ = orc.neighbors(S, S, 3, 1, lib, query_set=1)
    bn, bd = brute_neighbors(S, 3, 1, lib, 0, query_set=1)
    assert np.array_equal(nbr, bn) and np.array_equal(d2, bd)


def pin_neighbors_at_matches_full(orc):
    """Per-query results at listed queries equal the full realization's rows."""
    rng = np.random.default_rng(15)
    S = rng.random(120)
    T = rng.random(120)
    lib = np.sort(rng.choice(118, size=40, replace=False))
    nbr, d2, pred, _ = orc.neighbors(S, T, 3, 1, lib)
    q = np.array([0, 5, 77, 117])
    n2, d22, p2 = orc.neighbors_at(S, T, 3, 1, lib, q)
    assert np.array_equal(n2, nbr[q]) and np.array_equal(d22, d2[q])
    assert np.array_equal(p2, pred[q])


def pin_pearson_numpy(orc):
    """Pearson correlation equals numpy.corrcoef (and scipy.stats.pearsonr)."""
    rng = np.random.default_rng(14)
    for n in (2, 3, 17, 1000):
        a = rng.random(n)
        b = 0.3 * a + rng.random(n)
        want = float(np.corrcoef(a, b)[0, 1])
        assert abs(orc.pearson(a, b) - want) < 1e-12
        if n > 2:
            assert abs(orc.pearson(a, b) - stats.pearsonr(a, b)[0]) < 1e-12
    assert math.isnan(orc.pearson(np.ones(5), rng.random(5)))


def pin_self_map_rho_one(orc):
    """Cross-mapping a series onto itself with the query kept gives rho = 1."""
    w = synth.workload_small()
    for E in (1, 2, 3):
        Ne = len(w.X) - (E - 1)
        _, _, pred, rho = orc.neighbors(w.X, w.X, E, 1, np.arange(Ne), excl=-1)
        assert abs(rho - 1.0) < 1e-12, (E, rho)
        assert np.array_equal(pred, w.X[E - 1:])


def pin_zero_distance_weights(orc):
    """d_1 = 0: equal weight over zero-distance neighbours, none elsewhere."""
    S = np.array([0.5, 0.25, 0.5, 0.75, 0.5, 1.0])
    T = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    e = math.e
    _, _, pred, _ = orc.neighbors(S, T, 1, 1, np.arange(6))
    want = [4.0, 2.0, 3.0, 2.0, 2.0, (4 * e + 1) / (e + 1)]
    assert np.max(np.abs(pred - np.array(want))) < 1e-12, pred
    _, _, pred, _ = orc.neighbors(S, T, 1, 1, np.arange(6), excl=-1)
    assert pred[1] == 2.0 and pred[3] == 4.0     # lone zero-distance neighbour: itself


def pin_invariances(orc):
    """Affine target, power-of-two scaling, full-library independence of the draw."""
    w = synth.workload_small()
    X, Y = w.X[:400], w.Y[:400]
    r1, _ = orc.realization(Y, X, 2, 1, 150, 3, 7)
    r2, _ = orc.realization(Y, 2.5 * X - 0.75, 2, 1, 150, 3, 7)
    assert abs(r1 - r2) < 1e-12
    for k in (-3, 2):
        r3, _ = orc.realization(Y * 2.0 ** k, X, 2, 1, 150, 3, 7)
        assert r3 == r1
        lib = orc.sample_library(7, 2, 1, 150, 3, 399)
        a = orc.neighbors(Y, X, 2, 1, lib)
        b = orc.neighbors(Y * 2.0 ** k, X, 2, 1, lib)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    full = [orc.realization(Y, X, 3, 2, 10**6, q, s)[0] for q in (0, 5) for s in (1, 99)]
    assert len(set(full)) == 1


def pin_coupled_logistic_convergence(orc):
    """Skill rises with L and X-from-M_Y dominates (x is driven by y weakly,
    y by x strongly, so M_Y carries more of x): Introduction, Section 2.1."""
    w = synth.workload_small()
    L = [100, 300, 600, 1000]
    rxy, ryx = orc.ccm_threaded(w.X, w.Y, 2, 1, L, 12, 1)
    mxy, myx = rxy.mean(1), ryx.mean(1)
    assert np.all(np.diff(mxy) > 0) and np.all(np.diff(myx) > 0), (mxy, myx)
    assert np.all(mxy > myx)
    assert mxy[-1] > 0.95 and myx[-1] < 0.8


def pin_splitmix64_known_answers(orc):
    """SplitMix64 from state 0 gives its published first outputs."""
    assert orc.sm64_stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                     0x06C45D188009454F]


def pin_sampler_structure(orc):
    """Ascending, distinct, in range, exact size; identity when L_eff = N_e;
    every key field changes the draw."""
    for (Ne, L) in ((10, 3), (100, 37), (1000, 999), (57, 57)):
        idx = orc.sample_library(5, 2, 1, L, 0, Ne)
        assert len(idx) == L
        assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < Ne
    assert np.array_equal(orc.sample_library(9, 3, 2, 400, 4, 400), np.arange(400))
    base = orc.sample_library(1, 2, 3, 50, 4, 500)
    for args in ((2, 2, 3, 50, 4), (1, 3, 3, 50, 4), (1, 2, 4, 50, 4),
                 (1, 2, 3, 50, 5), (1, 3, 2, 50, 4)):
        assert not np.array_equal(orc.sample_library(*args, 500), base), args
    assert np.array_equal(orc.sample_library(1, 2, 3, 50, 4, 500), base)


def pin_sampler_uniform(orc):
    """Selection sampling is uniform: inclusion counts and subset counts pass chi^2."""
    Ne, L, R = 50, 10, 4000
    counts = np.zeros(Ne)
    for q in range(R):
        counts[orc.sample_library(77, 1, 1, L, q, Ne)] += 1
    p = stats.chisquare(counts).pvalue
    assert p > 1e-4, p
    from itertools import combinations
    subsets = {c: 0 for c in combinations(range(5), 2)}
    for q in range(5000):
        subsets[tuple(orc.sample_library(3, 1, 1, 2, q, 5).tolist())] += 1
    p = stats.chisquare(list(subsets.values())).pvalue
    assert p > 1e-4, p


MASK64 = (1 << 64) - 1


def _py_splitmix_mix(z):
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & MASK64
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB & MASK64
    return z ^ (z >> 31)


def _py_nested(seed, E, tau, r_index, Ne, n):
    """The nested ordering restated with Python integers: key folded through
    the SplitMix64 mix, then forward Fisher-Yates steps driven by the stream."""
    st = 0
    for v in (seed, E, tau, r_index):
        st = _py_splitmix_mix(st ^ (v & MASK64))
    a = list(range(Ne))
    out = []
    for k in range(n):
        st = (st + 0x9E3779B97F4A7C15) & MASK64
        z = _py_splitmix_mix(st)
        j = k + ((z * (Ne - k)) >> 64)
        a[k], a[j] = a[j], a[k]
        out.append(a[k])
    return out


def _py_selection(seed, E, tau, L_eff, r_index, Ne):
    """Selection sampling restated with Python integers from Knuth's Algorithm
    S (TAOCP Vol. 2, Sec. 3.4.2): with t candidates seen and m chosen, take
    candidate t when a uniform integer below Ne - t falls below L_eff - m; the
    uniform integer is the high word of one 64-bit draw times (Ne - t).  The
    draws come from the SplitMix64 stream whose state is the key folded one
    field at a time, in the order (seed, E, tau, L_eff, r_index)."""
    st = 0
    for v in (seed, E, tau, L_eff, r_index):
        st = _py_splitmix_mix(st ^ (v & MASK64))
    chosen = []
    for t in range(Ne):
        if len(chosen) == L_eff:
            break
        st = (st + 0x9E3779B97F4A7C15) & MASK64
        u = (_py_splitmix_mix(st) * (Ne - t)) >> 64
        if u < L_eff - len(chosen):
            chosen.append(t)
    return chosen


def pin_sampler_python(orc):
    """The library draw equals an independent statement of the stream and of
    Algorithm S, on a grid of keys: seeds near 0 and near 2^64, every E, taus,
    sizes from 1 to the whole set, the sweep's and long series' sizes."""
    keys = [(1, 2, 1, 100, 0, 999), (2, 10, 5, 348, 249, 9955), (3, 3, 2, 1000, 17, 2500),
            (2**64 - 1, 1, 1, 1, 3, 40), (12345678901234567, 7, 3, 499, 1, 500),
            (0, 4, 1, 20, 99, 1997), (5, 6, 4, 137, 7, 1480), (2, 1, 1, 2976, 3, 10000)]
    for E in range(1, 11):
        keys.append((2, E, 1 + E % 5, 100 + 37 * E, E * 25, 10000 - (E - 1) * (1 + E % 5)))
    for seed, E, tau, le, ri, ne in keys:
        got = orc.sample_library(seed, E, tau, le, ri, ne).tolist()
        assert got == _py_selection(seed, E, tau, le, ri, ne), (seed, E, tau, le, ri, ne)
    st = 0
    for v in (9, 3, 2, 50, 4):
        st = _py_splitmix_mix(st ^ v)
    assert orc.library_state(9, 3, 2, 50, 4) == st


def pin_nested_structure(orc):
    """Nested ordering: distinct points in range, a permutation when complete,
    shorter draws are prefixes of longer ones, every key field matters, and
    the points match an independent statement of the shuffle."""
    for Ne, n in ((10, 3), (100, 37), (1000, 999), (57, 57)):
        idx = orc.sample_nested(5, 2, 1, 0, Ne, n)
        assert len(idx) == n and len(set(idx.tolist())) == n
        assert idx.min() >= 0 and idx.max() < Ne
    full = orc.sample_nested(9, 3, 2, 4, 400, 400)
    assert np.array_equal(np.sort(full), np.arange(400))
    for n1, n2 in ((1, 50), (17, 400), (399, 400)):
        assert np.array_equal(orc.sample_nested(9, 3, 2, 4, 400, n1),
                              orc.sample_nested(9, 3, 2, 4, 400, n2)[:n1])
    base = orc.sample_nested(1, 2, 3, 4, 500, 50)
    for args in ((2, 2, 3, 4), (1, 3, 3, 4), (1, 2, 4, 4), (1, 2, 3, 5), (1, 3, 2, 4)):
        assert not np.array_equal(orc.sample_nested(*args, 500, 50), base), args
    for key in ((1, 2, 3, 4, 500, 50), (12345678901234, 10, 5, 249, 9955, 200),
                (7, 1, 1, 0, 3, 3)):
        assert orc.sample_nested(*key).tolist() == _py_nested(*key), key


def pin_nested_uniform(orc):
    """Nested ordering is uniform: first point, first-4 inclusions and the
    ordered first pair all pass chi^2."""
    Ne, R = 12, 6600
    first = np.zeros(Ne)
    incl = np.zeros(Ne)
    pairs = np.zeros((Ne, Ne))
    for q in range(R):
        idx = orc.sample_nested(31, 2, 1, q, Ne, 4)
        first[idx[0]] += 1
        incl[idx] += 1
        pairs[idx[0], idx[1]] += 1
    assert stats.chisquare(first).pvalue > 1e-4
    assert stats.chisquare(incl).pvalue > 1e-4
    off = pairs[~np.eye(Ne, dtype=bool)]
    assert pairs.trace() == 0
    assert stats.chisquare(off).pvalue > 1e-4


def pin_nested_ccm(orc):
    """Nested cross map: each (L, r) is the realization over the first L_eff
    points of r's ordering; the libraries of one r are nested; the full
    library gives the same rho as the independent draws."""
    x, y = synth.coupled_logistic(260)
    E, tau, L, r, seed = 2, 1, [20, 75, 259, 300], 3, 17
    ne = 260 - (E - 1) * tau
    rxy, ryx, le = orc.ccm_nested(x, y, E, tau, L, r, seed)
    assert le.tolist() == [20, 75, 259, 259]
    for q in range(r):
        perm = orc.sample_nested(seed, E, tau, q, ne, 259)
        for il, l in enumerate(le):
            lib = np.sort(perm[:l])
            assert rxy[il, q] == orc.neighbors(y, x, E, tau, lib)[3]
            assert ryx[il, q] == orc.neighbors(x, y, E, tau, lib)[3]
        assert set(perm[:20].tolist()) <= set(perm[:75].tolist())
    ixy, iyx, _ = orc.ccm(x, y, E, tau, [259], r, seed)
    assert np.array_equal(rxy[2], ixy[0]) and np.array_equal(ryx[3], iyx[0])


def pin_shared_e(orc):
    """E-sweep sharing: one E alone with the full common range is the default
    cross map at the full library; every (E, L, r) is the realization over
    the series shifted by (E_max - E) tau with the library drawn over the
    N_c common points by the key without E."""
    x, y = synth.coupled_logistic(300)
    for E in (2, 4):
        ne = 300 - (E - 1) * 2
        sxy, syx, _ = orc.ccm_shared_e(x, y, [E], 2, [ne], 3, 5)
        dxy, dyx, _ = orc.ccm(x, y, E, 2, [ne], 3, 5)
        assert np.array_equal(sxy[0], dxy) and np.array_equal(syx[0], dyx)
    Es, tau, L, r, seed = [1, 3, 6], 2, [25, 120, 400], 2, 13
    rxy, ryx, le = orc.ccm_shared_e(x, y, Es, tau, L, r, seed)
    nc = 300 - (6 - 1) * tau
    assert le.tolist() == [25, 120, nc]
    for ie, E in enumerate(Es):
        d = (6 - E) * tau
        for il, l in enumerate(le):
            for q in range(r):
                lib = orc.sample_library(seed, 0, tau, int(l), q, nc)
                assert rxy[ie, il, q] == orc.neighbors(y[d:], x[d:], E, tau, lib)[3]
                assert ryx[ie, il, q] == orc.neighbors(x[d:], y[d:], E, tau, lib)[3]


def pin_shared_e_python(orc):
    """E = 1 inside a shared sweep, computed independently: common points at
    times c + (E_max - 1) tau, binary32 squared differences (the product
    diff * diff, which is the chain's first term), stable sort, exp weights,
    numpy Pearson."""
    x, y = synth.coupled_logistic(220)
    Es, tau, L, r, seed = [1, 4], 3, [60], 2, 29
    rxy, _, _ = orc.ccm_shared_e(x, y, Es, tau, L, r, seed)
    off = (4 - 1) * tau
    nc = 220 - off
    yf = y.astype(np.float32)
    for q in range(r):
        lib = orc.sample_library(seed, 0, tau, 60, q, nc)
        pred = np.empty(nc)
        for c in range(nc):
            cand = [j for j in lib if j != c]
            diff = np.array([yf[c + off] - yf[j + off] for j in cand], dtype=np.float32)
            d2 = diff * diff                       # binary32 product: RN(diff^2)
            order = np.argsort(d2, kind="stable")[:2]
            dist = np.sqrt(d2[order].astype(np.float64))
            u = np.exp(-dist / dist[0]) if dist[0] > 0 else (dist == 0).astype(float)
            w = u / u.sum()
            pred[c] = float(np.sum(w * x[np.asarray(cand)[order] + off]))
        rho = np.corrcoef(x[off:off + nc], pred)[0, 1]
        assert abs(rxy[0, 0, q] - rho) < 1e-12, (q, rxy[0, 0, q], rho)


def pin_input_rules(orc):
    """Invalid inputs are refused; L above N_e is clamped, not refused."""
    x = np.linspace(0.1, 0.9, 50)
    y = x[::-1].copy()
    assert orc.status_of_ccm(x, y, 50, 0, 1, [10], 1) != 0      # E < 1
    assert orc.status_of_ccm(x, y, 50, 11, 1, [20], 1) != 0     # E > 10
    assert orc.status_of_ccm(x, y, 50, 2, 0, [10], 1) != 0      # tau < 1
    assert orc.status_of_ccm(x, y, 50, 2, 1, [3], 1) != 0       # L < E + 2
    assert orc.status_of_ccm(x, y, 50, 2, 1, [10], 0) != 0      # r < 1
    bad = x.copy()
    bad[3] = np.nan
    assert orc.status_of_ccm(bad, y, 50, 2, 1, [10], 1) != 0    # non-finite
    assert orc.status_of_ccm(x, y, 50, 2, 1, [4000], 1) == 0    # clamped
    rxy, _, le = orc.ccm(x, y, 2, 1, [4000], 1, 1)
    assert le.tolist() == [49]


ALL_PINS = [
    pin_golden_dyadic,
    pin_ramp_e1,
    pin_ramp_e2,
    pin_e1_stable_argsort,
    pin_exact_fma_bruteforce,
    pin_query_set_library,
    pin_neighbors_at_matches_full,
    pin_pearson_numpy,
    pin_self_map_rho_one,
    pin_zero_distance_weights,
    pin_invariances,
    pin_coupled_logistic_convergence,
    pin_splitmix64_known_answers,
    pin_sampler_structure,
    pin_sampler_uniform,
    pin_sampler_python,
    pin_nested_structure,
    pin_nested_uniform,
    pin_nested_ccm,
    pin_shared_e,
    pin_shared_e_python,
    pin_input_rules,
]
