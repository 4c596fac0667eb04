"""Seeded synthetic inputs for convergent cross mapping workloads.

This module only *generates input series and parameter grids*.  It holds none
of the cross-map arithmetic (no embedding, distances, neighbour search,
weights or correlation), so both the CPU oracle and the HIP path can draw
their inputs from it without sharing any part of the method.

Workloads (all series are float64, all generators are seeded):

* ``coupled_logistic``: the two-species coupled logistic map commonly used to
  illustrate CCM (x is weakly forced by y, y more strongly by x), iterated with
  a simultaneous update in exactly the written evaluation order (plain Python
  floats, no fused multiply-add).
* ``add_observation_noise``: i.i.d. Gaussian observation noise added after the
  fact (not fed back into the dynamics).
* ``logistic_network``: M logistic maps coupled through a sparse random
  interaction matrix, redrawn until every value stays inside (0, 1).
* ``job_stream``: a Poisson stream of independent CCM jobs for serving.

The paper runs its experiments on an unnamed 4000-point series (Section 4,
baseline scenario); these generators stand in for it with series of the same
kind (coupled nonlinear dynamics) and the sizes each workload calls for.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "coupled_logistic",
    "add_observation_noise",
    "logistic_network",
    "geometric_grid",
    "Workload",
    "workload_small",
    "workload_sweep",
    "workload_long",
    "workload_matrix",
    "job_stream",
    "embedded_count",
]


def coupled_logistic(n: int, x0: float = 0.4, y0: float = 0.2,
                     rx: float = 3.8, ry: float = 3.5,
                     bxy: float = 0.02, byx: float = 0.1):
    """Iterate x[t+1] = x(rx - rx x - bxy y), y[t+1] = y(ry - ry y - byx x).

    Simultaneous update, evaluated left to right exactly as written, in IEEE
    double precision without contraction (Python floats never fuse).  Returns
    two float64 arrays of length ``n`` starting at (x0, y0).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    xs = [0.0] * n
    ys = [0.0] * n
    x, y = float(x0), float(y0)
    for t in range(n):
        xs[t] = x
        ys[t] = y
        x, y = x * (rx - rx * x - bxy * y), y * (ry - ry * y - byx * x)
    return np.asarray(xs, dtype=np.float64), np.asarray(ys, dtype=np.float64)


def add_observation_noise(s: np.ndarray, sigma: float, rng: np.random.Generator):
    """Return ``s + sigma * eps`` with eps ~ N(0, 1) i.i.d. from ``rng``."""
    return np.asarray(s, dtype=np.float64) + sigma * rng.standard_normal(len(s))


def logistic_network(m: int, n: int, seed: int, density: float = 0.05,
                     beta_lo: float = 0.02, beta_hi: float = 0.1,
                     r_lo: float = 3.5, r_hi: float = 3.8,
                     x_lo: float = 0.2, x_hi: float = 0.6,
                     max_redraws: int = 64):
    """M logistic maps x_i[t+1] = x_i (r_i - r_i x_i - sum_j beta_ij x_j).

    The off-diagonal edge mask is Bernoulli(``density``); present edges carry
    beta ~ U[beta_lo, beta_hi].  If any value leaves (0, 1) the whole draw is
    repeated from the next sub-seed.  Returns (S [m][n] float64, beta [m][m]).
    """
    for attempt in range(max_redraws):
        rng = np.random.default_rng([seed, attempt])
        r = rng.uniform(r_lo, r_hi, m)
        mask = rng.random((m, m)) < density
        np.fill_diagonal(mask, False)
        beta = np.where(mask, rng.uniform(beta_lo, beta_hi, (m, m)), 0.0)
        x = rng.uniform(x_lo, x_hi, m)
        out = np.empty((m, n), dtype=np.float64)
        ok = True
        for t in range(n):
            out[:, t] = x
            x = x * (r - r * x - beta @ x)
            if not np.all((x > 0.0) & (x < 1.0)):
                ok = False
                break
        if ok:
            return out, beta
    raise RuntimeError("logistic_network: no bounded draw found")


def geometric_grid(lo: float, hi: float, n: int):
    """``n`` values geometrically spaced from lo to hi, rounded to integers."""
    if n == 1:
        return [int(round(hi))]
    return [int(round(lo * (hi / lo) ** (i / (n - 1)))) for i in range(n)]


def embedded_count(n: int, e: int, tau: int) -> int:
    """Number of lagged-coordinate vectors a series of length n yields."""
    return n - (e - 1) * tau


@dataclass
class Workload:
    """One cross-map workload: series plus its parameter grid."""
    name: str
    X: np.ndarray
    Y: np.ndarray
    E: list
    tau: list
    L: list
    r: int
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return len(self.X)


def workload_small() -> Workload:
    """Coupled logistic map, N=1000, E=2, tau=1, L=100..1000 step 100, r=100."""
    x, y = coupled_logistic(1000)
    return Workload("coupled-logistic N=1000 E=2 tau=1 L=100..1000 r=100",
                    x, y, [2], [1], list(range(100, 1001, 100)), 100, 1)


def workload_sweep(n: int = 10000, r: int = 250) -> Workload:
    """Parameter sweep: E=1..10, tau=1..5, 20 L log-spaced 100..10^4, r=250."""
    x, y = coupled_logistic(n)
    return Workload(f"coupled-logistic sweep N={n} E=1..10 tau=1..5 "
                    f"L=20 log-spaced 100..{n} r={r}",
                    x, y, list(range(1, 11)), list(range(1, 6)),
                    geometric_grid(100, n, 20), r, 2)


def workload_long(n: int = 100000, r: int = 250) -> Workload:
    """Long noisy series: N=10^5 + N(0, 0.01^2) noise, E=3, tau=2."""
    x, y = coupled_logistic(n)
    rng = np.random.default_rng(103)
    x = add_observation_noise(x, 0.01, rng)
    y = add_observation_noise(y, 0.01, rng)
    return Workload(f"noisy coupled-logistic N={n} E=3 tau=2 L=1e3,1e4,5e4,1e5 r={r}",
                    x, y, [3], [2], [1000, 10000, 50000, 100000], r, 3)


def workload_matrix(m: int = 64, n: int = 20000, r: int = 100):
    """64-series logistic network, E=4, tau=1, 10 L values 500..20000."""
    s, beta = logistic_network(m, n, seed=5)
    return {"name": f"logistic network M={m} N={n} E=4 tau=1 L=10 geometric 500..{n} r={r}",
            "S": s, "beta": beta, "E": 4, "tau": 1,
            "L": geometric_grid(500, n, 10), "r": r, "seed": 5}


def job_stream(n_jobs: int, rate_hz: float, seed: int = 4,
               n_lo: int = 1000, n_hi: int = 50000, r: int = 100):
    """Poisson stream of CCM jobs on seeded coupled-logistic pairs.

    Per job (seeded by its id): N ~ U{n_lo..n_hi}, E ~ U{1..10},
    tau ~ U{1..4}, x0, y0 ~ U(0.1, 0.9); a 10-point geometric L grid from
    100 to the embedded count; r realizations.  Arrival gaps are exponential
    with mean 1/rate_hz.  Series are generated lazily by ``job['make']()``.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_jobs) if rate_hz > 0 else np.zeros(n_jobs)
    t = np.cumsum(gaps)
    jobs = []
    for j in range(n_jobs):
        jr = np.random.default_rng([seed, 1000003, j])
        n = int(jr.integers(n_lo, n_hi + 1))
        e = int(jr.integers(1, 11))
        tau = int(jr.integers(1, 5))
        x0, y0 = (float(v) for v in jr.uniform(0.1, 0.9, 2))
        ne = embedded_count(n, e, tau)
        grid = sorted(set(geometric_grid(100, ne, 10)))

        def make(n=n, x0=x0, y0=y0):
            return coupled_logistic(n, x0, y0)

        jobs.append({"id": j, "t_arrival": float(t[j]), "N": n, "E": e, "tau": tau,
                     "x0": x0, "y0": y0, "L": grid, "r": r,
                     "seed": int(jr.integers(0, 2**63)), "make": make})
    return jobs


def quantised_series(n: int, levels: int, rng: np.random.Generator):
    """Series on a coarse grid k/levels: forces distance ties and d_1 = 0."""
    return np.floor(rng.random(n) * levels) / levels


def dyadic_series(n: int, rng: np.random.Generator, denom: int = 8):
    """Series of values k/denom: every float32 operation on them is exact."""
    return rng.integers(0, denom + 1, n).astype(np.float64) / denom

