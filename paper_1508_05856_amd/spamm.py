"""Thin ctypes binding over ``libspamm.so`` (the C ABI declared in include/spamm.h).

Argument marshalling only: torch CUDA tensors become device pointers and the
current HIP stream, statuses become exceptions.  Every step of the computation
runs in the library's HIP kernels; there is no CPU or PyTorch fallback, and
loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspamm.so")

OK, NOT_CONVERGED, STAGNATED = 0, 1, 2
EINVAL, ENOMEM, EDIVERGED, EHIP, ECAPACITY = -1, -2, -3, -4, -5
F64, F32, BF16X3, BF16X6 = 0, 1, 2, 3
_PREC = {"f64": F64, "fp64": F64, "f32": F32, "fp32": F32, "bf16x3": BF16X3, "bf16x6": BF16X6}

STATUS_NAMES = {OK: "OK", NOT_CONVERGED: "NOT_CONVERGED", STAGNATED: "STAGNATED", EINVAL: "EINVAL",
                ENOMEM: "ENOMEM", EDIVERGED: "EDIVERGED", EHIP: "EHIP", ECAPACITY: "ECAPACITY"}

# Every symbol include/spamm.h declares.
EXPORTS = ("spamm_create", "spamm_destroy", "spamm_last_error", "spamm_pyramid_len", "spamm_norms",
           "spamm_multiply", "ns_sqrt", "spamm_ns_history", "spamm_solve_footprint", "spamm_solve_begin",
           "spamm_solve_step", "spamm_solve_poll", "spamm_solve_finish", "spamm_set_graphs", "spamm_profile_enable",
           "spamm_profile_read", "spamm_profile_reset", "spamm_solve_triples", "spamm_product_rep",
           "spamm_multiply_noalloc", "spamm_alloc_count", "spamm_set_pool_limit")
MAX_SLICES = 16
KIND_GEMM, KIND_CULL, KIND_PYRAMID = 0, 1, 2


class SpammError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("retained", ctypes.c_int64), ("possible", ctypes.c_int64), ("thr", ctypes.c_double),
                ("flops", ctypes.c_double)]


class NsOpts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int), ("prec", ctypes.c_int), ("tau_s", ctypes.c_double),
                ("mu_rel", ctypes.c_double), ("stagnation_stop", ctypes.c_int), ("damped", ctypes.c_int),
                ("single", ctypes.c_int)]


class ProdRepOpts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int), ("prec", ctypes.c_int), ("nslices", ctypes.c_int),
                ("mu_rel", ctypes.POINTER(ctypes.c_double)), ("tau_slice", ctypes.c_double),
                ("tau_s_slice", ctypes.c_double), ("tau_r", ctypes.c_double), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("stagnation_stop", ctypes.c_int), ("damped", ctypes.c_int)]


class ProdRepResult(ctypes.Structure):
    _fields_ = [("nslices_done", ctypes.c_int), ("status", ctypes.c_int * 16), ("iterations", ctypes.c_int * 16)]


class NsResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("resid", ctypes.c_double), ("trace_err", ctypes.c_double),
                ("scale", ctypes.c_double), ("triples_total", ctypes.c_int64), ("flops_total", ctypes.c_double)]


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libspamm.so and declare the C ABI; raises if it is missing."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with paper_1508_05856_amd.build.build() "
                               "(there is no CPU fallback)")
        lib = ctypes.CDLL(path)
        vp, i64, i32p, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        lib.spamm_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
        lib.spamm_destroy.argtypes = [vp]
        lib.spamm_last_error.argtypes = []
        lib.spamm_last_error.restype = ctypes.c_char_p
        lib.spamm_pyramid_len.argtypes = [i64, ctypes.c_int]
        lib.spamm_pyramid_len.restype = i64
        lib.spamm_norms.argtypes = [vp, vp, i64, i64, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double), vp]
        lib.spamm_multiply.argtypes = [vp, vp, vp, vp, i64, i64, dbl, ctypes.c_int, ctypes.c_int, i32p, i64,
                                       ctypes.POINTER(Stats), vp]
        lib.spamm_multiply_noalloc.argtypes = [vp, vp, vp, vp, i64, i64, dbl, ctypes.c_int, ctypes.c_int, vp]
        lib.spamm_multiply_noalloc.restype = ctypes.c_int
        lib.ns_sqrt.argtypes = [vp, vp, vp, vp, i64, i64, dbl, dbl, ctypes.c_int, ctypes.POINTER(NsOpts),
                                ctypes.POINTER(NsResult), vp]
        lib.spamm_ns_history.argtypes = [vp, vp, vp, vp, ctypes.c_int]
        lib.spamm_solve_footprint.argtypes = [i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.spamm_solve_footprint.restype = ctypes.c_size_t
        lib.spamm_solve_begin.argtypes = [vp, vp, i64, i64, dbl, dbl, ctypes.c_int, ctypes.POINTER(NsOpts),
                                          ctypes.POINTER(ctypes.c_void_p), vp]
        lib.spamm_solve_step.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, vp]
        lib.spamm_solve_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(NsResult)]
        lib.spamm_solve_finish.argtypes = [vp, vp, vp, vp, i64, vp]
        lib.spamm_solve_triples.argtypes = [vp, vp, ctypes.c_int, vp, i64, ctypes.POINTER(ctypes.c_int64), vp]
        lib.spamm_product_rep.argtypes = [vp, vp, vp, i64, i64, ctypes.POINTER(ProdRepOpts),
                                          ctypes.POINTER(ProdRepResult), vp]
        lib.spamm_profile_enable.argtypes = [vp, ctypes.c_int]
        lib.spamm_set_graphs.argtypes = [vp, ctypes.c_int]
        lib.spamm_set_graphs.restype = ctypes.c_int
        lib.spamm_profile_reset.argtypes = [vp]
        lib.spamm_profile_read.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
        lib.spamm_alloc_count.argtypes = [vp]
        lib.spamm_alloc_count.restype = ctypes.c_int64
        lib.spamm_set_pool_limit.argtypes = [vp, ctypes.c_size_t]
        lib.spamm_set_pool_limit.restype = ctypes.c_int
        for f in (lib.spamm_create, lib.spamm_destroy, lib.spamm_norms, lib.spamm_multiply, lib.ns_sqrt,
                  lib.spamm_ns_history, lib.spamm_profile_enable, lib.spamm_profile_reset,
                  lib.spamm_profile_read, lib.spamm_solve_begin, lib.spamm_solve_step, lib.spamm_solve_poll,
                  lib.spamm_solve_finish):
            f.restype = ctypes.c_int
        _lib = lib
        return lib


def _check(status: int, allow_warning: bool = True) -> int:
    if status < 0:
        raise SpammError(status, load_library().spamm_last_error().decode())
    return status


def _stream_ptr(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _mat(t: torch.Tensor, name: str) -> tuple[int, int]:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or t.dim() != 2 or t.shape[0] != t.shape[1] or t.stride(1) != 1:
        raise ValueError(f"{name} must be a square float64 row-major matrix")
    return t.data_ptr(), t.stride(0)


class Context:
    """Owns one spamm_ctx (device scratch, pinned scalars, last solve's history)."""

    def __init__(self, device: int | None = None):
        self.lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(self.lib.spamm_create(ctypes.byref(h), self.device))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(self.lib.spamm_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points --------------------------------------------------------
    def pyramid_len(self, n: int, leaf: int) -> int:
        return int(self.lib.spamm_pyramid_len(n, leaf))

    def spamm_norms(self, A: torch.Tensor, leaf: int, want_root: bool = True) -> tuple[torch.Tensor, float | None]:
        """Norm pyramid of A; the root norm (which synchronises) only if want_root."""
        pa, ld = _mat(A, "A")
        n = A.shape[0]
        out = torch.empty(self.pyramid_len(n, leaf), dtype=torch.float64, device=A.device)
        root = ctypes.c_double(0.0)
        _check(self.lib.spamm_norms(self.handle, pa, n, ld, leaf, out.data_ptr(),
                                    ctypes.byref(root) if want_root else None, _stream_ptr(A.device)))
        return out, (root.value if want_root else None)

    def spamm_multiply(self, A: torch.Tensor, B: torch.Tensor, tau: float, leaf: int, prec="f64",
                       C: torch.Tensor | None = None, triples: bool = False, cap: int | None = None):
        """C = A (x)_tau B.  Returns (C, stats dict, triples or None)."""
        pa, ld = _mat(A, "A")
        pb, ldb = _mat(B, "B")
        n = A.shape[0]
        if B.shape != A.shape or ldb != ld:
            raise ValueError("A and B must have the same shape and leading dimension")
        if C is None:
            C = torch.empty_like(A)
        pc, ldc = _mat(C, "C")
        if ldc != ld:
            raise ValueError("C must share A's leading dimension")
        nb = -(-n // leaf)
        trip = None
        if triples:
            if cap is None:
                cap = nb ** 3
            trip = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=A.device)
        st = Stats()
        status = self.lib.spamm_multiply(self.handle, pa, pb, pc, n, ld, float(tau), leaf,
                                         _PREC[prec] if isinstance(prec, str) else int(prec),
                                         trip.data_ptr() if trip is not None else None, cap or 0,
                                         ctypes.byref(st), _stream_ptr(A.device))
        _check(status)
        stats = dict(retained=st.retained, possible=st.possible, thr=st.thr, flops=st.flops)
        if trip is not None:
            trip = trip[:st.retained]
        return C, stats, trip

    def spamm_multiply_noalloc(self, A: torch.Tensor, B: torch.Tensor, tau: float, leaf: int, prec="f64",
                               C: torch.Tensor | None = None) -> torch.Tensor:
        """C = A (x)_tau B through the allocation-free entry point (static
        device scratch; enqueued on the current stream, not synchronised).
        C must be preallocated by callers that cannot allocate."""
        pa, ld = _mat(A, "A")
        pb, ldb = _mat(B, "B")
        if B.shape != A.shape or ldb != ld:
            raise ValueError("A and B must have the same shape and leading dimension")
        if C is None:
            C = torch.empty_like(A)
        pc, ldc = _mat(C, "C")
        if ldc != ld:
            raise ValueError("C must share A's leading dimension")
        _check(self.lib.spamm_multiply_noalloc(self.handle, pa, pb, pc, A.shape[0], ld, float(tau), leaf,
                                               _PREC[prec] if isinstance(prec, str) else int(prec),
                                               _stream_ptr(A.device)))
        return C

    def ns_sqrt(self, s: torch.Tensor, tau: float, tol: float, maxit: int, leaf: int = 32, prec="f64",
                tau_s: float = -1.0, mu_rel: float = 0.0, stagnation_stop: bool = False, damped: bool = False,
                single: bool = False, Y: torch.Tensor | None = None, Z: torch.Tensor | None = None,
                raise_on_error: bool = True):
        """Y ~ s^{1/2}, Z ~ s^{-1/2}.  Returns (Y, Z, info dict)."""
        ps, ld = _mat(s, "s")
        n = s.shape[0]
        Y = torch.empty_like(s) if Y is None else Y
        Z = torch.empty_like(s) if Z is None else Z
        py, ldy = _mat(Y, "Y")
        pz, ldz = _mat(Z, "Z")
        if ldy != ld or ldz != ld:
            raise ValueError("Y and Z must share s's leading dimension")
        opts = NsOpts(leaf, _PREC[prec] if isinstance(prec, str) else int(prec), float(tau_s), float(mu_rel),
                      int(bool(stagnation_stop)), int(bool(damped)), int(bool(single)))
        res = NsResult()
        status = self.lib.ns_sqrt(self.handle, ps, py, pz, n, ld, float(tau), float(tol), int(maxit),
                                  ctypes.byref(opts), ctypes.byref(res), _stream_ptr(s.device))
        if status < 0 and raise_on_error:
            _check(status)
        info = dict(status=status, iterations=res.iterations, resid=res.resid, trace_err=res.trace_err,
                    scale=res.scale, triples_total=res.triples_total, flops_total=res.flops_total)
        if status < 0:
            info["error"] = self.lib.spamm_last_error().decode()
        return Y, Z, info

    def product_rep(self, s: torch.Tensor, mu_rel, tau_slice: float, tau_r: float, tol: float, maxit: int,
                    leaf: int = 32, prec="f64", tau_s_slice: float = -1.0, stagnation_stop: bool = True,
                    damped: bool = False, W: torch.Tensor | None = None, raise_on_error: bool = True):
        """Inverse factor W (W^T (s + mu_rel[-1] c0 I) W ~ I) as a product of
        regularised slices.  Returns (W, info dict with per-slice status and
        update counts)."""
        ps, ld = _mat(s, "s")
        n = s.shape[0]
        W = torch.empty_like(s) if W is None else W
        pw, ldw = _mat(W, "W")
        if ldw != ld:
            raise ValueError("W must share s's leading dimension")
        mu = (ctypes.c_double * len(mu_rel))(*[float(m) for m in mu_rel])
        opts = ProdRepOpts(leaf, _PREC[prec] if isinstance(prec, str) else int(prec), len(mu_rel), mu,
                           float(tau_slice), float(tau_s_slice), float(tau_r), float(tol), int(maxit),
                           int(bool(stagnation_stop)), int(bool(damped)))
        res = ProdRepResult()
        status = self.lib.spamm_product_rep(self.handle, ps, pw, n, ld, ctypes.byref(opts), ctypes.byref(res),
                                            _stream_ptr(s.device))
        if status < 0 and raise_on_error:
            _check(status)
        k = res.nslices_done
        return W, dict(status=status, statuses=list(res.status[:k]), iterations=list(res.iterations[:k]))

    # -- step API (batched and served solves) --------------------------------
    def footprint(self, n: int, leaf: int, prec="f64", maxit: int = 40, single: bool = False) -> int:
        return int(self.lib.spamm_solve_footprint(n, leaf, _PREC[prec] if isinstance(prec, str) else int(prec),
                                                  maxit, int(bool(single))))

    def solve_begin(self, s: torch.Tensor, tau: float, tol: float, maxit: int, leaf: int = 32, prec="f64",
                    tau_s: float = -1.0, mu_rel: float = 0.0, stagnation_stop: bool = False,
                    damped: bool = False, single: bool = False) -> "Solve":
        ps, ld = _mat(s, "s")
        opts = NsOpts(leaf, _PREC[prec] if isinstance(prec, str) else int(prec), float(tau_s), float(mu_rel),
                      int(bool(stagnation_stop)), int(bool(damped)), int(bool(single)))
        h = ctypes.c_void_p()
        _check(self.lib.spamm_solve_begin(self.handle, ps, s.shape[0], ld, float(tau), float(tol), int(maxit),
                                          ctypes.byref(opts), ctypes.byref(h), _stream_ptr(s.device)))
        return Solve(self, h, s.shape[0], s.device)

    def solve_step(self, solves, iterations: int = 1) -> int:
        """Advance every running solve in the list by `iterations`; returns how many still run."""
        arr = (ctypes.c_void_p * max(len(solves), 1))(*[x.handle for x in solves])
        dev = solves[0].device if solves else torch.device("cuda", self.device)
        return _check(self.lib.spamm_solve_step(self.handle, arr, len(solves), int(iterations), _stream_ptr(dev)))

    def set_graphs(self, enable: bool = True):
        _check(self.lib.spamm_set_graphs(self.handle, int(bool(enable))))

    def profile(self, enable: bool = True):
        _check(self.lib.spamm_profile_enable(self.handle, int(bool(enable))))

    def set_pool_limit(self, nbytes: int):
        """Device bytes the context keeps pooled at most (beyond it, returned
        memory is freed)."""
        _check(self.lib.spamm_set_pool_limit(self.handle, int(nbytes)))

    def alloc_count(self) -> int:
        """Device and pinned allocations this context has made so far."""
        return int(self.lib.spamm_alloc_count(self.handle))

    def profile_reset(self):
        _check(self.lib.spamm_profile_reset(self.handle))

    def profile_read(self, kind: int = KIND_GEMM):
        """Durations (ms) of the recorded launches of one kind, in launch order."""
        import numpy as np
        m = _check(self.lib.spamm_profile_read(self.handle, kind, None, 0))
        out = np.zeros(max(m, 1))
        _check(self.lib.spamm_profile_read(self.handle, kind, out.ctypes.data, m))
        return out[:m]

    def ns_history(self, cap: int = 4096):
        """(r, t, nR) of the most recent ns_sqrt on this context, as lists."""
        import numpy as np
        r = np.zeros(cap)
        t = np.zeros(cap)
        nR = np.zeros((cap, 3), dtype=np.int64)
        m = _check(self.lib.spamm_ns_history(self.handle, r.ctypes.data, t.ctypes.data, nR.ctypes.data, cap))
        m = min(m, cap)
        return r[:m], t[:m], nR[:m]


class Solve:
    """One Newton-Schulz solve on the device (spamm_solve)."""

    def __init__(self, ctx: Context, handle, n: int, device):
        self.ctx, self.handle, self.n, self.device = ctx, handle, n, device

    def triples(self, which: int) -> torch.Tensor:
        """Retained (i, j, k) triples of the latest product of one channel
        (0 = x, 1 = y, 2 = z), sorted, as a device int32 tensor (|R|, 3)."""
        cnt = ctypes.c_int64(0)
        # a zero-capacity call reports the count (ECAPACITY when non-empty)
        self.ctx.lib.spamm_solve_triples(self.ctx.handle, self.handle, int(which), None, 0, ctypes.byref(cnt),
                                         _stream_ptr(self.device))
        m = int(cnt.value)
        out = torch.empty((max(m, 1), 3), dtype=torch.int32, device=self.device)
        _check(self.ctx.lib.spamm_solve_triples(self.ctx.handle, self.handle, int(which), out.data_ptr(), m,
                                                ctypes.byref(cnt), _stream_ptr(self.device)))
        return out[:m]

    def poll(self) -> dict:
        done = ctypes.c_int(0)
        res = NsResult()
        st = self.ctx.lib.spamm_solve_poll(self.handle, ctypes.byref(done), ctypes.byref(res))
        return dict(done=bool(done.value), status=st, iterations=res.iterations, resid=res.resid,
                    trace_err=res.trace_err, scale=res.scale, triples_total=res.triples_total,
                    flops_total=res.flops_total)

    def finish(self, Y: torch.Tensor | None = None, Z: torch.Tensor | None = None, want_outputs: bool = True):
        """Egress (Y, Z), free the solve; returns (Y, Z, info)."""
        if self.handle is None:
            raise RuntimeError("solve already finished")
        info = self.poll()
        if want_outputs:
            if Y is None:
                Y = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
            if Z is None:
                Z = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
            py, ld = _mat(Y, "Y")
            pz, ldz = _mat(Z, "Z")
            if ldz != ld:
                raise ValueError("Y and Z must share a leading dimension")
        else:
            py = pz = None
            ld = self.n
        st = self.ctx.lib.spamm_solve_finish(self.ctx.handle, self.handle, py, pz, ld, _stream_ptr(self.device))
        self.handle = None
        info["status"] = st
        if st < 0:
            info["error"] = self.ctx.lib.spamm_last_error().decode()
        return Y, Z, info


_default_ctx: dict[int, Context] = {}


def default_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def spamm_norms(A, leaf):
    return default_context(A.device.index).spamm_norms(A, leaf)


def spamm_multiply(A, B, tau, leaf, prec="f64", **kw):
    return default_context(A.device.index).spamm_multiply(A, B, tau, leaf, prec, **kw)


def ns_sqrt(s, tau, tol, maxit, **kw):
    return default_context(s.device.index).ns_sqrt(s, tau, tol, maxit, **kw)


def exported_symbols(path: str = LIB_PATH) -> list[str]:
    """Names from EXPORTS that the shared library defines (no GPU needed)."""
    lib = ctypes.CDLL(path)
    return [name for name in EXPORTS if hasattr(lib, name)]
