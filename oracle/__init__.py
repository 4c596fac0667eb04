"""Python access to the CPU oracle (``ccm_oracle.c``) through ctypes.

TEST INFRASTRUCTURE ONLY: the oracle is the plain reference the HIP library
is checked against.  Only ``tests/``, the smoke check and the CPU-baseline leg
of ``bench.py`` may import this package; the product library never does.

Every method here is argument marshalling; the arithmetic is in the C file.
Realizations are independent, so ``ccm_threaded`` runs them on a thread pool
(ctypes releases the GIL during the foreign call).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "ccm_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=gnu11", "-Wall", "-Wextra", "-ffp-contract=off",
             "-fno-fast-math", "-fPIC", "-shared"]

MASK64 = (1 << 64) - 1


def compile_oracle(src: str, out: str) -> str:
    """Compile one oracle source file with gcc (contraction off, no fast-math)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIBRARY):
        compile_oracle(SOURCE, LIBRARY)
    return LIBRARY


class OracleError(RuntimeError):
    pass


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


class Oracle:
    """One loaded build of the oracle shared library."""

    def __init__(self, path: str = LIBRARY):
        if path == LIBRARY and not os.path.exists(path):
            build()
        L = C.CDLL(path)
        i32, i64, u64, dbl = C.c_int32, C.c_int64, C.c_uint64, C.c_double
        P = C.c_void_p
        L.oracle_sm64_mix.argtypes = [u64]
        L.oracle_sm64_mix.restype = u64
        L.oracle_sm64_next.argtypes = [C.POINTER(u64)]
        L.oracle_sm64_next.restype = u64
        L.oracle_library_state.argtypes = [u64, i32, i32, i64, i32]
        L.oracle_library_state.restype = u64
        L.oracle_sample_library.argtypes = [u64, i32, i32, i64, i32, i64, P]
        L.oracle_sample_library.restype = i64
        L.oracle_pearson.argtypes = [P, P, i64]
        L.oracle_pearson.restype = dbl
        L.oracle_neighbors.argtypes = [P, P, i64, i32, i32, P, i64, i32, i32,
                                       P, P, P, P]
        L.oracle_neighbors.restype = C.c_int
        L.oracle_neighbors_at.argtypes = [P, P, i64, i32, i32, P, i64, i32, P, i64,
                                          P, P, P]
        L.oracle_neighbors_at.restype = C.c_int
        L.oracle_realization.argtypes = [P, P, i64, i32, i32, i64, i32, u64,
                                         i32, i32, P, P]
        L.oracle_realization.restype = C.c_int
        L.oracle_ccm.argtypes = [P, P, i64, i32, i32, P, i32, i32, u64, i32,
                                 i32, P, P, P]
        L.oracle_ccm.restype = C.c_int
        L.oracle_nested_state.argtypes = [u64, i32, i32, i32]
        L.oracle_nested_state.restype = u64
        L.oracle_sample_nested.argtypes = [u64, i32, i32, i32, i64, i64, P]
        L.oracle_sample_nested.restype = C.c_int
        L.oracle_ccm_nested.argtypes = [P, P, i64, i32, i32, P, i32, i32, u64, i32,
                                        P, P, P]
        L.oracle_ccm_nested.restype = C.c_int
        L.oracle_ccm_shared_e.argtypes = [P, P, i64, P, i32, i32, P, i32, i32, u64, i32,
                                          P, P, P]
        L.oracle_ccm_shared_e.restype = C.c_int
        self.lib = L
        self.path = path

    @staticmethod
    def _check(st):
        if st != 0:
            raise OracleError(f"oracle status {st}")

    # -- sampler ---------------------------------------------------------
    def sm64_mix(self, z: int) -> int:
        return int(self.lib.oracle_sm64_mix(z & MASK64))

    def sm64_stream(self, state: int, n: int):
        st = C.c_uint64(state & MASK64)
        return [int(self.lib.oracle_sm64_next(C.byref(st))) for _ in range(n)]

    def library_state(self, seed, E, tau, L_eff, r_index) -> int:
        return int(self.lib.oracle_library_state(seed & MASK64, E, tau, L_eff, r_index))

    def sample_library(self, seed, E, tau, L_eff, r_index, N_e):
        out = np.empty(max(L_eff, 1), dtype=np.int32)
        n = self.lib.oracle_sample_library(seed & MASK64, E, tau, L_eff, r_index,
                                           N_e, _ptr(out))
        return out[:n].copy()

    def nested_state(self, seed, E, tau, r_index) -> int:
        return int(self.lib.oracle_nested_state(seed & MASK64, E, tau, r_index))

    def sample_nested(self, seed, E, tau, r_index, N_e, n_out):
        """First n_out points of the nested ordering of (E, tau, r_index)."""
        out = np.empty(max(n_out, 1), dtype=np.int32)
        self._check(self.lib.oracle_sample_nested(seed & MASK64, E, tau, r_index, N_e,
                                                  n_out, _ptr(out)))
        return out[:n_out].copy()

    # -- one realization ---------------------------------------------------
    def pearson(self, a, b) -> float:
        a, b = _f64(a), _f64(b)
        assert len(a) == len(b)
        return float(self.lib.oracle_pearson(_ptr(a), _ptr(b), len(a)))

    def neighbors(self, S, T, E, tau, lib_idx, excl=0, query_set=0):
        """(nbr [nq][E+1], d2 [nq][E+1] float32, pred [nq], rho) of one library."""
        S, T = _f64(S), _f64(T)
        li = np.ascontiguousarray(lib_idx, dtype=np.int32)
        N = len(S)
        Ne = N - (E - 1) * tau
        nq = len(li) if query_set else Ne
        nbr = np.empty((max(nq, 1), E + 1), dtype=np.int32)
        d2 = np.empty((max(nq, 1), E + 1), dtype=np.float32)
        pred = np.empty(max(nq, 1), dtype=np.float64)
        rho = C.c_double()
        self._check(self.lib.oracle_neighbors(_ptr(S), _ptr(T), N, E, tau, _ptr(li),
                                              len(li), excl, query_set, _ptr(nbr),
                                              _ptr(d2), _ptr(pred), C.byref(rho)))
        return nbr[:nq], d2[:nq], pred[:nq], rho.value

    def neighbors_at(self, S, T, E, tau, lib_idx, queries, excl=0):
        """(nbr [nq][E+1], d2 [nq][E+1], pred [nq]) at the listed embedded queries."""
        S, T = _f64(S), _f64(T)
        li = np.ascontiguousarray(lib_idx, dtype=np.int32)
        qs = np.ascontiguousarray(queries, dtype=np.int64)
        nq = len(qs)
        nbr = np.empty((max(nq, 1), E + 1), dtype=np.int32)
        d2 = np.empty((max(nq, 1), E + 1), dtype=np.float32)
        pred = np.empty(max(nq, 1), dtype=np.float64)
        self._check(self.lib.oracle_neighbors_at(_ptr(S), _ptr(T), len(S), E, tau, _ptr(li),
                                                 len(li), excl, _ptr(qs), nq, _ptr(nbr),
                                                 _ptr(d2), _ptr(pred)))
        return nbr[:nq], d2[:nq], pred[:nq]

    def realization(self, S, T, E, tau, L, r_index, seed, excl=0, query_set=0):
        """(rho, L_eff) of one sampled realization."""
        S, T = _f64(S), _f64(T)
        rho = C.c_double()
        le = C.c_int64()
        self._check(self.lib.oracle_realization(_ptr(S), _ptr(T), len(S), E, tau,
                                                int(L), r_index, seed & MASK64, excl,
                                                query_set, C.byref(le), C.byref(rho)))
        return rho.value, le.value

    # -- whole cross map ---------------------------------------------------
    def ccm(self, X, Y, E, tau, L, r, seed, excl=0, query_set=0):
        """rho_xy[l][r] (X predicted from Y's manifold), rho_yx[l][r], L_eff[l]."""
        X, Y = _f64(X), _f64(Y)
        Ls = np.ascontiguousarray(L, dtype=np.int64)
        nL = len(Ls)
        rxy = np.empty((nL, r))
        ryx = np.empty((nL, r))
        le = np.empty(nL, dtype=np.int64)
        self._check(self.lib.oracle_ccm(_ptr(X), _ptr(Y), len(X), E, tau, _ptr(Ls), nL,
                                        r, seed & MASK64, excl, query_set, _ptr(rxy),
                                        _ptr(ryx), _ptr(le)))
        return rxy, ryx, le

    def ccm_nested(self, X, Y, E, tau, L, r, seed, excl=0):
        """As ccm, with nested libraries (the first L_eff points of one ordering per r)."""
        X, Y = _f64(X), _f64(Y)
        Ls = np.ascontiguousarray(L, dtype=np.int64)
        nL = len(Ls)
        rxy = np.empty((nL, r))
        ryx = np.empty((nL, r))
        le = np.empty(nL, dtype=np.int64)
        self._check(self.lib.oracle_ccm_nested(_ptr(X), _ptr(Y), len(X), E, tau, _ptr(Ls),
                                               nL, r, seed & MASK64, excl, _ptr(rxy),
                                               _ptr(ryx), _ptr(le)))
        return rxy, ryx, le

    def ccm_shared_e(self, X, Y, Es, tau, L, r, seed, excl=0):
        """E-sweep sharing for one tau: rho_xy[e][l][r], rho_yx[e][l][r], L_eff[l]."""
        X, Y = _f64(X), _f64(Y)
        Ea = np.ascontiguousarray(Es, dtype=np.int32)
        Ls = np.ascontiguousarray(L, dtype=np.int64)
        nE, nL = len(Ea), len(Ls)
        rxy = np.empty((nE, nL, r))
        ryx = np.empty((nE, nL, r))
        le = np.empty(nL, dtype=np.int64)
        self._check(self.lib.oracle_ccm_shared_e(_ptr(X), _ptr(Y), len(X), _ptr(Ea), nE, tau,
                                                 _ptr(Ls), nL, r, seed & MASK64, excl,
                                                 _ptr(rxy), _ptr(ryx), _ptr(le)))
        return rxy, ryx, le

    def status_of_ccm(self, X, Y, N, E, tau, L, r, excl=0):
        """Raw status code of the whole cross map (for input-rule checks)."""
        X, Y = _f64(X), _f64(Y)
        Ls = np.ascontiguousarray(L, dtype=np.int64)
        nL = len(Ls)
        rxy = np.empty((max(nL, 1), max(r, 1)))
        ryx = np.empty_like(rxy)
        le = np.empty(max(nL, 1), dtype=np.int64)
        return int(self.lib.oracle_ccm(_ptr(X), _ptr(Y), N, E, tau, _ptr(Ls), nL, r, 1,
                                       excl, 0, _ptr(rxy), _ptr(ryx), _ptr(le)))

    def realization_split(self, S, T, E, tau, L, r_index, seed, excl=0, threads=None,
                          chunk=2048):
        """rho of one realization (every embedded point a query) with its queries
        split over threads: the library from ``sample_library``, each chunk's
        predictions from ``neighbors_at``, then the skill from ``pearson`` of
        the observed and predicted values -- the steps ``realization`` takes,
        in its query order, so the result is the same (pinned)."""
        S, T = _f64(S), _f64(T)
        N = len(S)
        off = (E - 1) * tau
        Ne = N - off
        le = min(int(L), Ne)
        lib = self.sample_library(seed, E, tau, le, r_index, Ne)
        qs = np.arange(Ne, dtype=np.int64)
        parts = [qs[a:a + chunk] for a in range(0, Ne, chunk)]
        threads = threads or default_threads()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            preds = list(ex.map(lambda q: self.neighbors_at(S, T, E, tau, lib, q, excl)[2],
                                parts))
        return self.pearson(T[off:off + Ne], np.concatenate(preds))

    def deterministic_sample(self, X, Y, Es, taus, Ls, r, seed, modulus):
        """The realizations of a sweep whose library stream state (the fold of
        (seed, E, tau, L_eff, r_index) that keys the draw) is 0 mod
        ``modulus``, both directions of each: a fixed sample for timing the
        oracle and checking the GPU.  Returns (tasks, picks): ``realization``
        argument tuples and their (direction, iE, itau, iL, r_index) indices
        in the sweep's rho."""
        N = len(X)
        tasks, picks = [], []
        for ie, e in enumerate(Es):
            for it, t in enumerate(taus):
                ne = N - (e - 1) * t
                for il, l in enumerate(Ls):
                    le = min(int(l), ne)
                    for ri in range(r):
                        if self.library_state(seed, e, t, le, ri) % modulus:
                            continue
                        for d, (S, T) in enumerate(((Y, X), (X, Y))):
                            tasks.append((S, T, e, t, l, ri, seed, 0, 0))
                            picks.append((d, ie, it, il, ri))
        return tasks, picks

    def realizations_threaded(self, tasks, threads=None):
        """rho of many realizations; ``tasks`` holds ``realization`` argument tuples."""
        threads = threads or default_threads()

        def one(t):
            return self.realization(*t)[0]

        if threads == 1:
            return [one(t) for t in tasks]
        with ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(one, tasks))

    def ccm_threaded(self, X, Y, E, tau, L, r, seed, excl=0, query_set=0, threads=None):
        """Same result as ``ccm`` with the realizations spread over threads."""
        X, Y = _f64(X), _f64(Y)
        tasks = []
        for l in L:
            for q in range(r):
                tasks.append((Y, X, E, tau, l, q, seed, excl, query_set))
                tasks.append((X, Y, E, tau, l, q, seed, excl, query_set))
        res = self.realizations_threaded(tasks, threads)
        arr = np.asarray(res).reshape(len(L), r, 2)
        return arr[:, :, 0].copy(), arr[:, :, 1].copy()


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def __getattr__(name):
    # module-level shortcuts: oracle.ccm(...), oracle.neighbors(...), ...
    if name.startswith("_"):
        raise AttributeError(name)
    return getattr(default(), name)
