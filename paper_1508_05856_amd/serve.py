"""Continuous-batching server for Newton-Schulz square-root solves on one GPU.

Requests (s, tau, tol, ...) arrive from any thread.  A single engine thread
admits pending requests as solver slots while their device footprint
(spamm_solve_footprint) fits the HBM budget, then advances every admitted
solve by a few iterations per step in shared launches (spamm_solve_step);
solves that stop leave at the step boundary, their results are written out
and their memory is released, and newly arrived requests join the next step.
Each solve's arithmetic does not depend on which others share its launches,
so a result is the same alone and in any mix.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import torch

from . import spamm


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
    t_submit: float = 0.0
    future: Future = field(default_factory=Future)
    footprint: int = 0


@dataclass
class Result:
    Y: torch.Tensor
    Z: torch.Tensor
    info: dict
    latency_s: float   # submit to result ready
    queued_s: float    # submit to admission
    t_done: float      # time.perf_counter() when the result was ready


class Server:
    def __init__(self, device: int = 0, hbm_budget: int | None = None, iters_per_step: int = 2,
                 max_active: int = 512, autostart: bool = True):
        self.ctx = spamm.Context(device)
        self.device = torch.device("cuda", device)
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(device)
            hbm_budget = int(free * 0.6)  # the rest holds queued inputs and returned outputs
        self.hbm_budget = hbm_budget
        self.iters_per_step = iters_per_step
        self.max_active = max_active
        self._pending: collections.deque[Request] = collections.deque()
        self._lock = threading.Condition()
        self._stop = False
        self._active: list[tuple[Request, spamm.Solve, float]] = []
        self.in_use = 0
        self.pending_bytes = 0
        self.stats = dict(steps=0, admitted=0, completed=0, failed=0, max_active=0, max_pending=0, peak_bytes=0)
        self._thread = threading.Thread(target=self._loop, name="spamm-engine", daemon=True)
        if autostart:
            self._thread.start()

    def start(self):
        """Start the engine thread (for a server made with autostart=False)."""
        if not self._thread.is_alive():
            self._thread.start()

    # -- client side ----------------------------------------------------------
    def submit(self, s: torch.Tensor, tau: float, tol: float, **kw) -> Future:
        req = Request(s=s, tau=tau, tol=tol, **kw)
        req.footprint = self.ctx.footprint(s.shape[0], req.leaf, req.prec, req.maxit, req.single)
        if req.footprint == 0 or req.footprint > self.hbm_budget:
            req.future.set_exception(ValueError(f"request needs {req.footprint} bytes; budget {self.hbm_budget}"))
            return req.future
        req.t_submit = time.perf_counter()
        with self._lock:
            if self._stop:
                req.future.set_exception(RuntimeError("server is closed"))
                return req.future
            self._pending.append(req)
            self.pending_bytes += s.numel() * s.element_size()
            self.stats["max_pending"] = max(self.stats["max_pending"], len(self._pending))
            self._lock.notify()
        return req.future

    def backlog(self) -> tuple[int, int]:
        """(requests, input bytes) submitted and not yet admitted."""
        with self._lock:
            return len(self._pending), self.pending_bytes

    def close(self):
        """Finish every submitted request, then stop the engine."""
        self.start()
        with self._lock:
            self._stop = True
            self._lock.notify()
        self._thread.join()
        self.ctx.close()

    # -- engine thread --------------------------------------------------------
    def _admit(self):
        while True:
            with self._lock:
                if not self._pending or len(self._active) >= self.max_active:
                    return
                req = self._pending[0]
                if self.in_use + req.footprint > self.hbm_budget and self._active:
                    return  # wait for memory to free up at a step boundary
                self._pending.popleft()
                self.pending_bytes -= req.s.numel() * req.s.element_size()
            t_admit = time.perf_counter()
            try:
                sv = self.ctx.solve_begin(req.s, req.tau, req.tol, req.maxit, leaf=req.leaf, prec=req.prec,
                                          tau_s=req.tau_s, mu_rel=req.mu_rel,
                                          stagnation_stop=req.stagnation_stop, damped=req.damped,
                                          single=req.single)
            except Exception as e:  # invalid input or no memory: fail this request only
                req.s = None
                req.future.set_exception(e)
                continue
            req.s = None  # the solve holds its own blocked copy of s
            self.in_use += req.footprint
            self.stats["peak_bytes"] = max(self.stats["peak_bytes"], self.in_use)
            self._active.append((req, sv, t_admit))
            self.stats["admitted"] += 1

    def _fail_active(self, err: Exception):
        """A shared launch failed: every solve in it fails, and its memory is released."""
        for req, sv, _ in self._active:
            try:
                sv.finish(want_outputs=False)
            except Exception:
                pass
            self.in_use -= req.footprint
            req.future.set_exception(err)
            self.stats["failed"] += 1
        self._active = []

    def _loop(self):
        while True:
            with self._lock:
                while not self._stop and not self._pending and not self._active:
                    self._lock.wait()
                if self._stop and not self._active and not self._pending:
                    return
            self._admit()
            if not self._active:
                continue
            self.stats["max_active"] = max(self.stats["max_active"], len(self._active))
            try:
                self.ctx.solve_step([sv for _, sv, _ in self._active], self.iters_per_step)
            except Exception as e:
                self._fail_active(e)
                continue
            self.stats["steps"] += 1
            still = []
            for req, sv, t_admit in self._active:
                if not sv.poll()["done"]:
                    still.append((req, sv, t_admit))
                    continue
                try:
                    # finish() writes Y, Z and waits for them, so the result is ready at `now`
                    Y, Z, info = sv.finish()
                except Exception as e:  # e.g. no memory for the outputs
                    if sv.handle is not None:
                        sv.finish(want_outputs=False)
                    self.in_use -= req.footprint
                    req.future.set_exception(e)
                    self.stats["failed"] += 1
                    continue
                self.in_use -= req.footprint
                now = time.perf_counter()
                self.stats["completed"] += 1
                req.future.set_result(Result(Y, Z, info, now - req.t_submit, t_admit - req.t_submit, now))
            self._active = still
