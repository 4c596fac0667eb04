"""ctypes binding of libccm (include/ccm.h), function for function.

Argument marshalling only: every step of the cross map runs in the HIP
library.  There is no CPU path: if ``libccm.so`` is missing the import of a
function raises, and if no GPU is present ``ccm_create`` fails.

Host-array functions take numpy arrays; device-pointer functions
(``ccm_dev``, ``ccm_sweep_dev``) take torch CUDA tensors (or raw integer
addresses) plus an optional stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CCM_LIBRARY may name another build of the same library (e.g. a tuning variant).
LIBRARY = os.environ.get("CCM_LIBRARY") or os.path.join(_HERE, "libccm.so")

CCM_OK = 0
CCM_E_INVAL = -1
CCM_E_NOMEM = -2
CCM_E_DEVICE = -3
CCM_E_BUSY = -4
CCM_E_NOTFOUND = -5
CCM_E_TIMEOUT = -6

CCM_FLAG_PLAIN = 1
CCM_FLAG_NO_GRAPH = 2
CCM_FLAG_PERSISTENT = 4
CCM_FLAG_TABLE = 8
CCM_FLAG_NESTED = 16
CCM_FLAG_SHARED_E = 32
CCM_TABLE_WIDTH = 1024

# Every symbol include/ccm.h declares (checked by the ABI test).
EXPORTS = [
    "ccm_create", "ccm_destroy", "ccm_last_error", "ccm_set_wave_limit", "ccm", "ccm_sweep",
    "ccm_matrix", "ccm_dev", "ccm_dev_noalloc", "ccm_sweep_dev", "ccm_matrix_dev", "ccm_library",
    "ccm_nested_library", "ccm_neighbors",
    "ccm_profile_enable", "ccm_profile_read",
    "ccm_server_create", "ccm_submit", "ccm_wait", "ccm_result", "ccm_cancel",
    "ccm_server_destroy",
]


class ccm_opts(C.Structure):
    _fields_ = [("exclusion_radius", C.c_int32), ("query_set", C.c_int32),
                ("flags", C.c_uint32)]


class ccm_profile(C.Structure):
    _fields_ = [("kernel_ms", C.c_double), ("launches", C.c_int64),
                ("pairs", C.c_double), ("flops", C.c_double),
                ("predictions", C.c_double), ("realizations", C.c_double),
                ("table_realizations", C.c_double), ("waves", C.c_double)]


class ccm_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_jobs", C.c_int32),
                ("epoch_target_ms", C.c_double)]


class ccm_job(C.Structure):
    _fields_ = [("X", C.c_void_p), ("Y", C.c_void_p), ("N", C.c_int64), ("E", C.c_int32),
                ("tau", C.c_int32), ("L", C.c_void_p), ("nL", C.c_int32), ("r", C.c_int32),
                ("seed", C.c_uint64), ("opts", ccm_opts)]


class ccm_job_stats(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("pairs", C.c_uint64), ("predictions", C.c_uint64),
                ("realizations", C.c_uint64), ("device_bytes", C.c_uint64)]


class CCMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"ccm status {status}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libccm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(f"{LIBRARY} is missing: build it with "
                               "`python -m paper_1905_00565_amd.build`")
        try:
            # One HIP runtime per process: torch bundles its own copy (same
            # SONAME); loading it first makes libccm bind to that copy.
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIBRARY)
        P, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.ccm_create.argtypes = [C.c_int, C.POINTER(P)]
        L.ccm_destroy.argtypes = [P]
        L.ccm_destroy.restype = None
        L.ccm_last_error.argtypes = [P]
        L.ccm_last_error.restype = C.c_char_p
        L.ccm_set_wave_limit.argtypes = [P, u64]
        L.ccm.argtypes = [P, P, P, i64, i32, i32, P, i32, i32, u64, P, P, P, P]
        L.ccm_sweep.argtypes = [P, P, P, i64, P, i32, P, i32, P, i32, i32, u64, P, P]
        L.ccm_dev.argtypes = [P, P, P, i64, i32, i32, P, i32, i32, u64, P, P, P, P, P]
        L.ccm_dev_noalloc.argtypes = [P, P, P, i64, i32, i32, P, i32, i32, u64, P, P, P, P, P]
        L.ccm_sweep_dev.argtypes = [P, P, P, i64, P, i32, P, i32, P, i32, i32, u64, P, P, P]
        L.ccm_matrix.argtypes = [P, P, i32, i64, i32, i32, P, i32, i32, u64, P, P]
        L.ccm_matrix_dev.argtypes = [P, P, i32, i64, i32, i32, P, i32, i32, u64, P, P, P]
        L.ccm_library.argtypes = [P, i64, i32, i32, i64, i32, u64, P]
        L.ccm_neighbors.argtypes = [P, P, P, i64, i32, i32, P, i64, P, P, P, P, P]
        L.ccm_server_create.argtypes = [P, C.POINTER(ccm_server_cfg), C.POINTER(P)]
        L.ccm_submit.argtypes = [P, C.POINTER(ccm_job), C.POINTER(u64)]
        L.ccm_wait.argtypes = [P, u64, i64]
        L.ccm_result.argtypes = [P, u64, P, P, C.POINTER(ccm_job_stats)]
        L.ccm_cancel.argtypes = [P, u64]
        L.ccm_server_destroy.argtypes = [P]
        L.ccm_server_destroy.restype = None
        L.ccm_profile_enable.argtypes = [P, C.c_int]
        L.ccm_profile_read.argtypes = [P, C.POINTER(ccm_profile), C.c_int]
        for name in EXPORTS:
            if name not in ("ccm_destroy", "ccm_last_error", "ccm_server_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dev_ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return C.c_void_p(t)
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _opts(exclusion_radius=0, query_set=0, flags=0):
    return ccm_opts(int(exclusion_radius), int(query_set), int(flags))


def _check(ctx, st):
    if st != CCM_OK:
        msg = lib().ccm_last_error(ctx).decode() if ctx else ""
        raise CCMError(st, msg)


# ---------------------------------------------------------------------------
# functions mirroring the C ABI
# ---------------------------------------------------------------------------

def ccm_create(device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    st = lib().ccm_create(device, C.byref(h))
    if st != CCM_OK:
        raise CCMError(st, f"ccm_create(device={device}) failed")
    return h


def ccm_destroy(ctx) -> None:
    lib().ccm_destroy(ctx)


def ccm_last_error(ctx) -> str:
    return lib().ccm_last_error(ctx).decode()


def ccm_set_wave_limit(ctx, nbytes: int) -> None:
    """Device bytes of libraries held at once by a batched call (0: default)."""
    _check(ctx, lib().ccm_set_wave_limit(ctx, int(nbytes)))


def ccm(ctx, X, Y, E, tau, L, r, seed, exclusion_radius=0, query_set=0, flags=0):
    """(rho_X_from_MY [nL][r], rho_Y_from_MX [nL][r], L_eff [nL])."""
    X, Y = _f64(X), _f64(Y)
    if len(X) != len(Y):
        raise ValueError("X and Y must have the same length")
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    nL = len(Ls)
    rxy = np.empty((nL, r))
    ryx = np.empty((nL, r))
    le = np.empty(nL, dtype=np.int64)
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm(ctx, _ptr(X), _ptr(Y), len(X), E, tau, _ptr(Ls), nL, r,
                          seed & (2**64 - 1), C.byref(o), _ptr(rxy), _ptr(ryx), _ptr(le)))
    return rxy, ryx, le


def ccm_sweep(ctx, X, Y, E, tau, L, r, seed, exclusion_radius=0, query_set=0, flags=0):
    """rho [2][nE][ntau][nL][r] ([0]: X from M_Y, [1]: Y from M_X)."""
    X, Y = _f64(X), _f64(Y)
    if len(X) != len(Y):
        raise ValueError("X and Y must have the same length")
    Es = np.ascontiguousarray(E, dtype=np.int32)
    Ts = np.ascontiguousarray(tau, dtype=np.int32)
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    rho = np.empty((2, len(Es), len(Ts), len(Ls), r))
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_sweep(ctx, _ptr(X), _ptr(Y), len(X), _ptr(Es), len(Es), _ptr(Ts),
                                len(Ts), _ptr(Ls), len(Ls), r, seed & (2**64 - 1),
                                C.byref(o), _ptr(rho)))
    return rho


def ccm_dev(ctx, X, Y, E, tau, L, r, seed, rho_xy, rho_yx, stream=None,
            exclusion_radius=0, query_set=0, flags=0, N=None):
    """Device form: X, Y, rho_xy, rho_yx are torch CUDA tensors (or addresses)."""
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    le = np.empty(len(Ls), dtype=np.int64)
    n = int(N if N is not None else X.numel())
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_dev(ctx, _dev_ptr(X), _dev_ptr(Y), n, E, tau, _ptr(Ls), len(Ls),
                              r, seed & (2**64 - 1), C.byref(o), _dev_ptr(rho_xy),
                              _dev_ptr(rho_yx), _ptr(le), _stream_ptr(stream)))
    return le


def ccm_dev_noalloc(ctx, X, Y, E, tau, L, r, seed, rho_xy, rho_yx, stream=None,
                    exclusion_radius=0, query_set=0, flags=0, N=None):
    """ccm_dev with its device buffers in the library's static workspace."""
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    le = np.empty(len(Ls), dtype=np.int64)
    n = int(N if N is not None else X.numel())
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_dev_noalloc(ctx, _dev_ptr(X), _dev_ptr(Y), n, E, tau, _ptr(Ls),
                                      len(Ls), r, seed & (2**64 - 1), C.byref(o),
                                      _dev_ptr(rho_xy), _dev_ptr(rho_yx), _ptr(le),
                                      _stream_ptr(stream)))
    return le


def ccm_sweep_dev(ctx, X, Y, E, tau, L, r, seed, rho, stream=None,
                  exclusion_radius=0, query_set=0, flags=0, N=None):
    """Device form of ccm_sweep: rho is a device double[2][nE][ntau][nL][r]."""
    Es = np.ascontiguousarray(E, dtype=np.int32)
    Ts = np.ascontiguousarray(tau, dtype=np.int32)
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    n = int(N if N is not None else X.numel())
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_sweep_dev(ctx, _dev_ptr(X), _dev_ptr(Y), n, _ptr(Es), len(Es),
                                    _ptr(Ts), len(Ts), _ptr(Ls), len(Ls), r,
                                    seed & (2**64 - 1), C.byref(o), _dev_ptr(rho),
                                    _stream_ptr(stream)))


def ccm_matrix(ctx, S, E, tau, L, r, seed, exclusion_radius=0, query_set=0, flags=0):
    """rho [M][M][nL][r]: rho[a][b] predicts series b from the manifold of a."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    if S.ndim != 2:
        raise ValueError("S must be [M][N]")
    M, N = S.shape
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    rho = np.empty((M, M, len(Ls), r))
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_matrix(ctx, _ptr(S), M, N, E, tau, _ptr(Ls), len(Ls), r,
                                 seed & (2**64 - 1), C.byref(o), _ptr(rho)))
    return rho


def ccm_matrix_dev(ctx, S, E, tau, L, r, seed, rho, stream=None, exclusion_radius=0,
                   query_set=0, flags=0, M=None, N=None):
    """Device form of ccm_matrix: S is a device double[M][N], rho double[M][M][nL][r]."""
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    m = int(M if M is not None else S.shape[0])
    n = int(N if N is not None else S.shape[1])
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_matrix_dev(ctx, _dev_ptr(S), m, n, E, tau, _ptr(Ls), len(Ls), r,
                                     seed & (2**64 - 1), C.byref(o), _dev_ptr(rho),
                                     _stream_ptr(stream)))


def ccm_library(ctx, N_e, E, tau, L_eff, r_index, seed):
    out = np.empty(max(int(L_eff), 1), dtype=np.int32)
    _check(ctx, lib().ccm_library(ctx, N_e, E, tau, L_eff, r_index, seed & (2**64 - 1),
                                  _ptr(out)))
    return out[:L_eff]


def ccm_nested_library(ctx, N_e, E, tau, r_index, seed, n_out):
    """First n_out points of the nested ordering of (E, tau, r_index)."""
    out = np.empty(n_out, dtype=np.int32)
    _check(ctx, lib().ccm_nested_library(ctx, C.c_int64(N_e), E, tau, r_index,
                                         C.c_uint64(seed & (2**64 - 1)), C.c_int64(n_out),
                                         _ptr(out)))
    return out


def ccm_neighbors(ctx, lib_series, target, E, tau, lib_idx, exclusion_radius=0,
                  query_set=0, flags=0):
    """(nbr [Nq][E+1], d2 [Nq][E+1] float32, pred [Nq], rho) of one library."""
    S, T = _f64(lib_series), _f64(target)
    li = np.ascontiguousarray(lib_idx, dtype=np.int32)
    N = len(S)
    ne = N - (E - 1) * tau
    nq = len(li) if query_set else ne
    nbr = np.empty((max(nq, 1), E + 1), dtype=np.int32)
    d2 = np.empty((max(nq, 1), E + 1), dtype=np.float32)
    pred = np.empty(max(nq, 1), dtype=np.float64)
    rho = C.c_double()
    o = _opts(exclusion_radius, query_set, flags)
    _check(ctx, lib().ccm_neighbors(ctx, _ptr(S), _ptr(T), N, E, tau, _ptr(li), len(li),
                                    C.byref(o), _ptr(nbr), _ptr(d2), _ptr(pred),
                                    C.byref(rho)))
    return nbr[:nq], d2[:nq], pred[:nq], rho.value


def ccm_profile_enable(ctx, on=True):
    _check(ctx, lib().ccm_profile_enable(ctx, 1 if on else 0))


def ccm_profile_read(ctx, reset=True) -> dict:
    p = ccm_profile()
    _check(ctx, lib().ccm_profile_read(ctx, C.byref(p), 1 if reset else 0))
    return {f: getattr(p, f) for f, _ in ccm_profile._fields_}


def ccm_server_create(ctx, hbm_budget_bytes=0, max_jobs=0, epoch_target_ms=0.0):
    cfg = ccm_server_cfg(int(hbm_budget_bytes), int(max_jobs), float(epoch_target_ms))
    h = C.c_void_p()
    _check(ctx, lib().ccm_server_create(ctx, C.byref(cfg), C.byref(h)))
    return h


def ccm_submit(srv, X, Y, E, tau, L, r, seed, exclusion_radius=0, query_set=0, flags=0,
               ctx=None):
    """Queue a job; returns its ticket.  Arrays are copied by the call."""
    X, Y = _f64(X), _f64(Y)
    if len(X) != len(Y):
        raise ValueError("X and Y must have the same length")
    Ls = np.ascontiguousarray(L, dtype=np.int64)
    job = ccm_job(_ptr(X), _ptr(Y), len(X), E, tau, _ptr(Ls), len(Ls), r,
                  seed & (2**64 - 1), _opts(exclusion_radius, query_set, flags))
    t = C.c_uint64()
    _check(ctx, lib().ccm_submit(srv, C.byref(job), C.byref(t)))
    return t.value


def ccm_wait(srv, ticket, timeout_ns=-1) -> int:
    """Status of the wait (CCM_OK, CCM_E_TIMEOUT, ...); does not raise."""
    return int(lib().ccm_wait(srv, ticket, timeout_ns))


def ccm_result(srv, ticket, nL, r):
    """(rho_xy [nL][r], rho_yx [nL][r], stats dict); raises on a failed job."""
    rxy = np.empty((nL, r))
    ryx = np.empty((nL, r))
    st = ccm_job_stats()
    status = lib().ccm_result(srv, ticket, _ptr(rxy), _ptr(ryx), C.byref(st))
    if status != CCM_OK:
        raise CCMError(status, f"job {ticket}")
    return rxy, ryx, {f: getattr(st, f) for f, _ in ccm_job_stats._fields_}


def ccm_cancel(srv, ticket) -> int:
    return int(lib().ccm_cancel(srv, ticket))


def ccm_server_destroy(srv) -> None:
    lib().ccm_server_destroy(srv)


class Server:
    """Owns one server; methods forward to the functions above."""

    def __init__(self, ctx, **cfg):
        self.ctx = ctx.handle if isinstance(ctx, Context) else ctx
        self.handle = ccm_server_create(self.ctx, **cfg)

    def submit(self, *a, **k):
        return ccm_submit(self.handle, *a, ctx=self.ctx, **k)

    def wait(self, ticket, timeout_ns=-1):
        return ccm_wait(self.handle, ticket, timeout_ns)

    def result(self, ticket, nL, r):
        return ccm_result(self.handle, ticket, nL, r)

    def cancel(self, ticket):
        return ccm_cancel(self.handle, ticket)

    def close(self):
        if self.handle:
            ccm_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Context:
    """Owns one ccm context; methods forward to the functions above."""

    def __init__(self, device: int = 0):
        self.handle = ccm_create(device)

    def close(self):
        if self.handle:
            ccm_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_wave_limit(self, nbytes):
        ccm_set_wave_limit(self.handle, nbytes)

    def ccm(self, *a, **k):
        return ccm(self.handle, *a, **k)

    def ccm_sweep(self, *a, **k):
        return ccm_sweep(self.handle, *a, **k)

    def ccm_dev(self, *a, **k):
        return ccm_dev(self.handle, *a, **k)

    def ccm_dev_noalloc(self, *a, **k):
        return ccm_dev_noalloc(self.handle, *a, **k)

    def ccm_sweep_dev(self, *a, **k):
        return ccm_sweep_dev(self.handle, *a, **k)

    def ccm_matrix(self, *a, **k):
        return ccm_matrix(self.handle, *a, **k)

    def ccm_matrix_dev(self, *a, **k):
        return ccm_matrix_dev(self.handle, *a, **k)

    def ccm_library(self, *a, **k):
        return ccm_library(self.handle, *a, **k)

    def ccm_nested_library(self, *a, **k):
        return ccm_nested_library(self.handle, *a, **k)

    def ccm_neighbors(self, *a, **k):
        return ccm_neighbors(self.handle, *a, **k)

    def profile_enable(self, on=True):
        ccm_profile_enable(self.handle, on)

    def profile_read(self, reset=True):
        return ccm_profile_read(self.handle, reset)
