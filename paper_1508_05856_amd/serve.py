"""Continuous-batching server for Newton-Schulz square-root solves on one GPU.

Requests (s, tau, tol, ...) arrive from any thread.  Each lane of the server
is an engine thread with its own library context and HIP stream; a request
goes to the lane of its size class.  A lane admits pending requests as solver
slots while the device footprint of everything admitted (spamm_solve_footprint,
over all lanes) fits the HBM budget, then advances every admitted solve by a
few iterations per step in shared launches (spamm_solve_step); solves that stop
leave at the step boundary, their results are written out and their memory is
released, and newly arrived requests join the next step.  Lanes run on
separate streams, so small solves need not wait for the steps of large ones.
Each solve's arithmetic does not depend on which others share its launches or
its lane, so a result is the same alone and in any mix.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import torch

from . import spamm


def exact_residual(ctx: "spamm.Context", Y: torch.Tensor, Z: torch.Tensor) -> float:
    """||I - Y Z||_F from the library's dense (tau = 0) FP64 product on the
    current stream."""
    C, _, _ = ctx.spamm_multiply(Y, Z, 0.0, 64)
    C.diagonal().sub_(1.0)
    return float(torch.linalg.norm(C))


@dataclass
class Request:
    s: torch.Tensor                 # device, float64, symmetric
    tau: float
    tol: float
    maxit: int = 40
    leaf: int = 64
    prec: str = "f64"
    tau_s: float = -1.0
    mu_rel: float = 0.0
    stagnation_stop: bool = True
    damped: bool = False
    single: bool = False
    verify: bool = False            # also return the exact ||I - Y Z||_F (a dense product) as info["resid_exact"];
                                    # the product's workspace stays with the lane's context, outside the budget
    t_submit: float = 0.0
    future: Future = field(default_factory=Future)
    footprint: int = 0
    ready: object = None  # torch.cuda.Event recorded on the submitter's stream after s was written


@dataclass
class Result:
    """Y and Z are complete when the result is set (the lane synchronised its
    stream); a caller that hands them to work on another stream and then
    drops them should call record_stream first, as for any tensor."""
    Y: torch.Tensor
    Z: torch.Tensor
    info: dict
    latency_s: float   # submit to result ready
    queued_s: float    # submit to admission
    t_done: float      # time.perf_counter() when the result was ready


class _Lane:
    def __init__(self, server: "Server", device: int, nmax: int | None, iters: int):
        self.nmax = nmax  # largest n this lane takes (None: no bound)
        self.iters = iters  # iterations per step
        self.ctx = spamm.Context(device)
        self.stream = torch.cuda.Stream(device)  # default priority
        self.pending: collections.deque[Request] = collections.deque()
        self.active: list[tuple[Request, spamm.Solve, float]] = []
        self.thread = threading.Thread(target=server._loop, args=(self,), name="spamm-engine", daemon=True)


class Server:
    def __init__(self, device: int = 0, hbm_budget: int | None = None, iters_per_step=2,
                 max_active: int = 512, autostart: bool = True, lanes: tuple = (None,),
                 pool_share: float = 0.2):
        """lanes: the largest n of each lane in increasing order, the last one
        None (no bound); the default is one lane for every size.
        iters_per_step: iterations per step, one number or one per lane.  pool_share:
        the fraction of the budget that each lane's context may keep pooled
        (memory of finished solves kept for the next ones instead of freed)."""
        lanes = tuple(lanes)
        if not lanes or lanes[-1] is not None or any(a is None for a in lanes[:-1]) or any(
                a >= b for a, b in zip(lanes[:-2], lanes[1:-1])):
            raise ValueError("lanes must be increasing size bounds ending with None")
        self.device = torch.device("cuda", device)
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(device)
            hbm_budget = int(free * 0.45)  # the rest holds pooled memory, queued inputs and returned outputs
        self.hbm_budget = hbm_budget
        its = tuple(iters_per_step) if isinstance(iters_per_step, (tuple, list)) else (iters_per_step,) * len(lanes)
        if len(its) != len(lanes) or min(its) < 1:
            raise ValueError("iters_per_step must be >= 1, one value or one per lane")
        self.iters_per_step = its
        self.max_active = max_active
        self._lock = threading.Condition()
        self._stop = False
        self._lanes = [_Lane(self, device, nmax, it) for nmax, it in zip(lanes, its)]
        # each lane's context keeps the memory of finished solves pooled for
        # the next ones, up to its share of the budget
        for lane in self._lanes:
            lane.ctx.set_pool_limit(int(hbm_budget * pool_share))
        self.ctx = self._lanes[0].ctx  # for footprint queries
        self.in_use = 0
        self.pending_bytes = 0
        self.stats = dict(steps=0, admitted=0, completed=0, failed=0, max_active=0, max_pending=0, peak_bytes=0)
        if autostart:
            self.start()

    def start(self):
        """Start the engine threads (for a server made with autostart=False)."""
        for lane in self._lanes:
            if not lane.thread.is_alive():
                lane.thread.start()

    # -- client side ----------------------------------------------------------
    def submit(self, s: torch.Tensor, tau: float, tol: float, **kw) -> Future:
        req = Request(s=s, tau=tau, tol=tol, **kw)
        req.footprint = self.reservation(s.shape[0], req.leaf, req.prec, req.maxit, req.single)
        if req.footprint == 0 or req.footprint > self.hbm_budget:
            req.future.set_exception(ValueError(f"request needs {req.footprint} bytes; budget {self.hbm_budget}"))
            return req.future
        req.ready = torch.cuda.Event()
        req.ready.record(torch.cuda.current_stream(s.device))
        req.t_submit = time.perf_counter()
        lane = next(ln for ln in self._lanes if ln.nmax is None or s.shape[0] <= ln.nmax)
        with self._lock:
            if self._stop:
                req.future.set_exception(RuntimeError("server is closed"))
                return req.future
            lane.pending.append(req)
            self.pending_bytes += s.numel() * s.element_size()
            npend = sum(len(ln.pending) for ln in self._lanes)
            self.stats["max_pending"] = max(self.stats["max_pending"], npend)
            self._lock.notify_all()
        return req.future

    def reservation(self, n: int, leaf: int, prec: str = "f64", maxit: int = 40, single: bool = False) -> int:
        """Device bytes admission reserves for a request: its footprint plus
        what a pooled memory block may hold beyond it (a quarter and 16 MiB);
        0 for invalid arguments."""
        fp = self.ctx.footprint(n, leaf, prec, maxit, single)
        return fp + fp // 4 + (16 << 20) if fp > 0 else 0

    def backlog(self) -> tuple[int, int]:
        """(requests, input bytes) submitted and not yet admitted."""
        with self._lock:
            return sum(len(ln.pending) for ln in self._lanes), self.pending_bytes

    def close(self):
        """Finish every submitted request, then stop the engines."""
        self.start()
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for lane in self._lanes:
            lane.thread.join()
        for lane in self._lanes:
            lane.ctx.close()

    # -- engine threads -------------------------------------------------------
    def _admit(self, lane: _Lane) -> bool:
        """Admit what fits; False when a pending request waits for memory."""
        while True:
            with self._lock:
                if not lane.pending or len(lane.active) >= self.max_active:
                    return True
                req = lane.pending[0]
                if self.in_use + req.footprint > self.hbm_budget and self.in_use > 0:
                    return False  # memory frees up at some lane's step boundary
                lane.pending.popleft()
                self.pending_bytes -= req.s.numel() * req.s.element_size()
                self.in_use += req.footprint  # reserved before the lock is released
                self.stats["peak_bytes"] = max(self.stats["peak_bytes"], self.in_use)
            t_admit = time.perf_counter()
            try:
                lane.stream.wait_event(req.ready)
                sv = lane.ctx.solve_begin(req.s, req.tau, req.tol, req.maxit, leaf=req.leaf, prec=req.prec,
                                          tau_s=req.tau_s, mu_rel=req.mu_rel,
                                          stagnation_stop=req.stagnation_stop, damped=req.damped,
                                          single=req.single)
            except Exception as e:  # invalid input or no memory: fail this request only
                req.s = None
                self._release(req.footprint)
                req.future.set_exception(e)
                continue
            req.s = None  # the solve holds its own blocked copy of s (begin synchronised its stream)
            lane.active.append((req, sv, t_admit))
            with self._lock:
                self.stats["admitted"] += 1

    def _release(self, nbytes: int):
        with self._lock:
            self.in_use -= nbytes
            self._lock.notify_all()

    def _fail_active(self, lane: _Lane, err: Exception):
        """A shared launch failed: every solve in it fails, and its memory is released."""
        for req, sv, _ in lane.active:
            try:
                sv.finish(want_outputs=False)
            except Exception:
                pass
            self._release(req.footprint)
            req.future.set_exception(err)
            with self._lock:
                self.stats["failed"] += 1
        lane.active = []

    def _loop(self, lane: _Lane):
        torch.cuda.set_stream(lane.stream)  # this thread's library calls go to the lane's stream
        while True:
            with self._lock:
                while not self._stop and not lane.pending and not lane.active:
                    self._lock.wait()
                if self._stop and not lane.active and not lane.pending:
                    return
            fits = self._admit(lane)
            if not lane.active:
                if not fits:
                    with self._lock:
                        self._lock.wait(timeout=0.01)
                continue
            with self._lock:
                self.stats["max_active"] = max(self.stats["max_active"], sum(len(ln.active) for ln in self._lanes))
            try:
                lane.ctx.solve_step([sv for _, sv, _ in lane.active], lane.iters)
            except Exception as e:
                self._fail_active(lane, e)
                continue
            with self._lock:
                self.stats["steps"] += 1
            still = []
            for req, sv, t_admit in lane.active:
                if not sv.poll()["done"]:
                    still.append((req, sv, t_admit))
                    continue
                try:
                    # finish() writes Y, Z and waits for them, so the result is ready at `now`
                    Y, Z, info = sv.finish()
                except Exception as e:  # e.g. no memory for the outputs
                    if sv.handle is not None:
                        sv.finish(want_outputs=False)
                    self._release(req.footprint)
                    req.future.set_exception(e)
                    with self._lock:
                        self.stats["failed"] += 1
                    continue
                if req.verify:
                    info["resid_exact"] = exact_residual(lane.ctx, Y, Z) if info["status"] >= 0 else None
                self._release(req.footprint)
                now = time.perf_counter()
                with self._lock:
                    self.stats["completed"] += 1
                req.future.set_result(Result(Y, Z, info, now - req.t_submit, t_admit - req.t_submit, now))
            lane.active = still
