"""FP64 CPU oracle for SpAMM and coupled Newton-Schulz square-root iteration.

TEST INFRASTRUCTURE ONLY.  The arithmetic lives in ``spamm_oracle.c`` (plain C,
FP64, written from the paper; see its header for what each function follows).
This module only compiles it with gcc, loads it with ctypes and marshals NumPy
arrays.  It imports nothing from the GPU package, and the GPU package never
imports it: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spamm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK, NOT_CONVERGED, STAGNATED = 0, 1, 2
EINVAL, ENOMEM, EDIVERGED = -1, -2, -3


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, so the arithmetic is as written)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64, dp, ip = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
            lp = ctypes.POINTER(ctypes.c_int64)
            lib.oracle_pyramid_len.argtypes = [i64, i64]
            lib.oracle_pyramid_len.restype = i64
            lib.oracle_norms.argtypes = [dp, i64, i64, dp]
            lib.oracle_spamm.argtypes = [dp, dp, dp, i64, i64, ctypes.c_double, ip, i64, lp]
            lib.oracle_spamm_tiles.argtypes = [dp, dp, i64, i64, ctypes.c_double, ip, i64, dp, lp]
            lib.oracle_ns_step.argtypes = [dp, dp, dp, dp, i64, i64, ctypes.c_double, ctypes.c_double]
            lib.oracle_ns_sqrt.argtypes = [dp, dp, dp, i64, i64, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, dp, dp, lp, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_double)]
            lib.oracle_ns_single_step.argtypes = [dp, dp, dp, dp, i64, i64, ctypes.c_double, ctypes.c_double]
            lib.oracle_product_rep.argtypes = [dp, dp, i64, i64, dp, ctypes.c_int, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, ip, ip]
            lib.oracle_product_rep.restype = ctypes.c_int
            lib.oracle_damping.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
            lib.oracle_damping.restype = None
            for f in (lib.oracle_norms, lib.oracle_spamm, lib.oracle_spamm_tiles, lib.oracle_ns_sqrt,
                      lib.oracle_ns_step, lib.oracle_ns_single_step):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("expected a square matrix")
    return a


def depth(n: int, leaf: int) -> int:
    nb = -(-n // leaf)
    L = 0
    while (1 << L) < nb:
        L += 1
    return L


def norms(a, leaf: int) -> list[np.ndarray]:
    """Norm pyramid as a list of levels, leaves first: level d has shape (2^(L-d), 2^(L-d))."""
    a = _f64(a)
    n = a.shape[0]
    lib = _load()
    out = np.zeros(lib.oracle_pyramid_len(n, leaf), dtype=np.float64)
    st = lib.oracle_norms(_dptr(a), n, leaf, _dptr(out))
    if st:
        raise OracleError(f"oracle_norms status {st}")
    L = depth(n, leaf)
    levels, off = [], 0
    for d in range(L, -1, -1):
        side = 1 << d
        levels.append(out[off:off + side * side].reshape(side, side))
        off += side * side
    return levels


def spamm(a, b, leaf: int, tau: float, want_triples: bool = True, cap: int | None = None):
    """C = a (x)_tau b.  Returns (C, R, count) with R an (|R|, 3) int array of
    (i, j, k) sorted lexicographically (None when not requested)."""
    a, b = _f64(a), _f64(b)
    n = a.shape[0]
    nb = -(-n // leaf)
    lib = _load()
    c = np.zeros_like(a)
    if cap is None:
        cap = nb ** 3 if want_triples else 0
    trip = np.zeros((max(cap, 1), 3), dtype=np.int32)
    cnt = ctypes.c_int64(0)
    st = lib.oracle_spamm(_dptr(a), _dptr(b), _dptr(c), n, leaf, float(tau),
                          trip.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if want_triples else None,
                          cap, ctypes.byref(cnt))
    if st:
        raise OracleError(f"oracle_spamm status {st}")
    R = None
    if want_triples:
        if cnt.value > cap:
            raise OracleError("triple capacity exceeded")
        R = trip[:cnt.value]
        R = R[np.lexsort((R[:, 2], R[:, 1], R[:, 0]))]
    return c, R, cnt.value


def spamm_tiles(a, b, leaf: int, tau: float, tiles):
    """Only the listed C tiles of a (x)_tau b: returns (tiles_out[t, leaf, leaf], counts[t])."""
    a, b = _f64(a), _f64(b)
    n = a.shape[0]
    t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32).reshape(-1, 2))
    out = np.zeros((t.shape[0], leaf, leaf), dtype=np.float64)
    counts = np.zeros(t.shape[0], dtype=np.int64)
    st = _load().oracle_spamm_tiles(_dptr(a), _dptr(b), n, leaf, float(tau),
                                    t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), t.shape[0], _dptr(out),
                                    counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if st:
        raise OracleError(f"oracle_spamm_tiles status {st}")
    return out, counts


def ns_sqrt(s, leaf: int, tau: float, tol: float, maxit: int, tau_s: float = -1.0, mu_rel: float = 0.0,
            stagnation_stop: bool = False, damped: bool = False, single: bool = False) -> dict:
    """Coupled Newton-Schulz, dual channel or (single=True) the single
    channel instance, optionally with the damped map of Sec. 4.2.  Returns a
    dict with Y, Z, status, iterations, scale and the r, t and |R| histories."""
    s = _f64(s)
    n = s.shape[0]
    lib = _load()
    Y = np.zeros_like(s)
    Z = np.zeros_like(s)
    r = np.zeros(maxit + 1)
    t = np.zeros(maxit + 1)
    nr = np.zeros((maxit + 1, 3), dtype=np.int64)
    it = ctypes.c_int(0)
    sc = ctypes.c_double(0.0)
    st = lib.oracle_ns_sqrt(_dptr(s), _dptr(Y), _dptr(Z), n, leaf, float(tau), float(tau_s), float(tol),
                            int(maxit), float(mu_rel), int(bool(stagnation_stop)), int(bool(damped)),
                            int(bool(single)),
                            _dptr(r), _dptr(t),
                            nr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(it),
                            ctypes.byref(sc))
    k = it.value
    return dict(status=st, Y=Y, Z=Z, iterations=k, scale=sc.value, r=r[:k + 1].copy(), t=t[:k + 1].copy(),
                nR=nr[:k + 1].copy())


def damping(t: float, damped: bool = True) -> tuple[float, float]:
    """(alpha, eps) of the map at relative trace error t (Sec. 4.2), as the
    damped iteration uses them."""
    a, e = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _load().oracle_damping(int(bool(damped)), float(t), ctypes.byref(a), ctypes.byref(e))
    return a.value, e.value


def ns_step(y, z, leaf: int, tau: float, tau_s: float = -1.0):
    """One dual-channel update from (y, z): returns (h (x)_{tau_s} y, z (x)_tau h) with
    h = 1.5 I - 0.5 (y (x)_tau z)."""
    y, z = _f64(y), _f64(z)
    n = y.shape[0]
    yo = np.zeros_like(y)
    zo = np.zeros_like(z)
    st = _load().oracle_ns_step(_dptr(y), _dptr(z), _dptr(yo), _dptr(zo), n, leaf, float(tau), float(tau_s))
    if st:
        raise OracleError(f"oracle_ns_step status {st}")
    return yo, zo


def ns_single_step(s, z, leaf: int, tau: float, tau_s: float = -1.0):
    """One single-channel step from any (s', z): returns (y, z_next) with
    y = s' (x)_{tau_s} z and z_next = z (x)_tau h[z^T (x)_tau y] (plain map)."""
    s, z = _f64(s), _f64(z)
    n = s.shape[0]
    y = np.zeros_like(s)
    zn = np.zeros_like(s)
    st = _load().oracle_ns_single_step(_dptr(s), _dptr(z), _dptr(y), _dptr(zn), n, leaf, float(tau), float(tau_s))
    if st:
        raise OracleError(f"oracle_ns_single_step status {st}")
    return y, zn


def product_rep(s, leaf: int, mu_rel, tau_slice: float, tau_r: float, tol: float, maxit: int,
                tau_s_slice: float = -1.0, stagnation_stop: bool = True, damped: bool = False) -> dict:
    """Inverse factor W of s + mu_rel[-1] c0 I as a product of regularised
    slices (Secs. 6.1, 6.3).  Returns dict(status, W, statuses, iterations)."""
    s = _f64(s)
    n = s.shape[0]
    mu = np.ascontiguousarray(np.asarray(mu_rel, dtype=np.float64))
    W = np.zeros_like(s)
    sts = np.zeros(len(mu), dtype=np.int32)
    its = np.zeros(len(mu), dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int32)
    st = _load().oracle_product_rep(_dptr(s), _dptr(W), n, leaf, _dptr(mu), len(mu), float(tau_slice),
                                    float(tau_s_slice), float(tau_r), float(tol), int(maxit),
                                    int(bool(stagnation_stop)), int(bool(damped)), sts.ctypes.data_as(ip),
                                    its.ctypes.data_as(ip))
    return dict(status=st, W=W, statuses=sts.tolist(), iterations=its.tolist())
