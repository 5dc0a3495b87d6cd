"""Request loop for single-source Helmholtz solves of mixed grid sizes and
frequencies on one GPU (continuous admission by device-memory footprint).

Each request carries its own slowness model, frequency and source. A request
is admitted as soon as a worker is free and the device memory it needs (its
operators and multigrid hierarchy plus its Krylov workspace, planned on the
host with ``hh_footprint_bytes`` before anything is allocated) fits in the
budget beside the requests already on the device; requests that arrive while
others run are admitted as slots and memory free up. Every admitted request
runs on its own HIP stream (one per worker), so the work of several requests
overlaps on the device; its state (model, hierarchy, basis) stays on the
device until it completes. Admission is first-fit in arrival order, with the
head of the queue reserved once it has waited ``starvation_s`` (so a large
request is not passed over indefinitely).

A request's arithmetic does not depend on what else runs: each solve uses only
its own buffers and stream, and its control flow is decided on the device, so
a result in the mix equals the result alone (tested).
"""
from __future__ import annotations

import dataclasses
import threading
import time
from collections import deque
from typing import Dict, List, Optional

import numpy as np
import torch

from . import hh


@dataclasses.dataclass
class Request:
    id: int
    slowness: np.ndarray          # (nz, nx) or (n,) float64, s/m
    h: float                      # grid spacing (m)
    freq_hz: float
    source: np.ndarray            # complex128, same shape as slowness
    alpha: float = 0.01
    tol: float = 1e-6
    restart: int = 30
    max_iters: int = 2000
    # dense limit of the coarsest grid; None: chosen by coarsest_limit()
    max_coarse: Optional[int] = None
    precond_f32: bool = False
    t_arrival: float = 0.0        # set by the server at submission (monotonic clock)


@dataclasses.dataclass
class Result:
    id: int
    u: np.ndarray
    iterations: int
    true_rel_res: float
    status: int
    footprint: int                # bytes admitted for the request
    t_arrival: float
    t_admit: float
    t_done: float
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def queued(self) -> float:
        return self.t_admit - self.t_arrival


def coarsest_limit(req: Request) -> Optional[int]:
    """Dense limit of the coarsest grid for a request (2D). A larger limit stops
    the coarsening before under-resolved levels, trading a larger LU and inverse
    at set-up for far fewer iterations. Measured on MI355X (set-up + solve,
    complex64 preconditioner): 801 x 401 at 20 Hz: 4096 -> 1250 iterations
    (146 ms), 8192 -> 154 (43 ms); 1601 x 601 at 10 Hz: 8192 -> 309 (141 ms),
    16384 -> 94 (131 ms); 1601 x 601 at 20 Hz: 8192 does not converge in 2000,
    16384 -> 220 (206 ms). Hence 8192, and 16384 for grids of 500k nodes or
    more."""
    if req.max_coarse is not None or req.slowness.ndim != 2:
        return req.max_coarse
    return 16384 if req.slowness.size >= 500_000 else 8192


def footprint(req: Request) -> int:
    """Device bytes a request needs (operators + workspace), planned on the host."""
    pb, wb = hh.footprint_bytes(req.slowness.shape, 2 * np.pi * req.freq_hz,
                                float(req.slowness.max()), req.h,
                                max_coarse=coarsest_limit(req),
                                restart=req.restart, nrhs=1, precond_f32=req.precond_f32)
    return pb + wb


def solve_one(req: Request, device, stream) -> Result:
    """Create, solve and release one request on `stream` (used by the workers,
    and alone for reference)."""
    with torch.cuda.stream(stream):
        m = torch.from_numpy(np.ascontiguousarray(req.slowness, dtype=np.float64)).to(
            device, non_blocking=False)
        f = torch.from_numpy(np.ascontiguousarray(req.source, dtype=np.complex128)).to(device)
        P = hh.Problem(m, 2 * np.pi * req.freq_hz, req.alpha, req.h, stream=stream,
                       max_coarse=coarsest_limit(req))
        try:
            r = P.solve(f, tol=req.tol, restart=req.restart, max_iters=req.max_iters,
                        precond_f32=req.precond_f32, stream=stream, hist_cap=1)
            u = r.u.cpu().numpy()
        finally:
            P.close()
    return Result(id=req.id, u=u, iterations=r.iterations, true_rel_res=r.true_rel_res,
                  status=r.status, footprint=0, t_arrival=req.t_arrival, t_admit=0.0,
                  t_done=0.0)


class Server:
    """Admission by footprint onto `workers` concurrent streams of one GPU.

    `solve_fn(request, device, stream) -> Result` and `footprint_fn(request)`
    default to the GPU solve and the host-side plan; the scheduler itself does
    not touch the device (device=None runs without streams, for tests of the
    admission logic)."""

    def __init__(self, budget_bytes: int, workers: int = 4, device="cuda:0",
                 starvation_s: float = 1.0, solve_fn=None, footprint_fn=None):
        if workers < 1:
            raise ValueError("workers must be >= 1")
        self.budget = int(budget_bytes)
        self.device = torch.device(device) if device is not None else None
        self.starvation_s = starvation_s
        self._solve = solve_fn or solve_one
        self._footprint = footprint_fn or footprint
        self._lock = threading.Condition()
        self._pending: deque = deque()          # (request, footprint)
        self._in_use = 0
        self._results: Dict[int, Result] = {}
        self._closed = False
        self.peak_in_use = 0
        self.max_concurrent = 0
        self._running = 0
        self._streams = [torch.cuda.Stream(device=self.device) if self.device is not None
                         else None for _ in range(workers)]
        self._work: List[deque] = [deque() for _ in range(workers)]
        self._threads = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                         for i in range(workers)]
        self._idle = set(range(workers))
        for t in self._threads:
            t.start()

    # -- client side -------------------------------------------------------
    def submit(self, req: Request):
        fp = self._footprint(req)
        if fp > self.budget:
            raise ValueError(f"request {req.id} needs {fp} bytes, more than the budget")
        with self._lock:
            req.t_arrival = time.monotonic()
            self._pending.append((req, fp))
            self._admit()

    def results(self, ids=None, timeout: Optional[float] = None) -> Dict[int, Result]:
        """Wait for the given request ids (default: everything submitted)."""
        t0 = time.monotonic()
        with self._lock:
            while True:
                want = set(ids) if ids is not None else None
                done = want is None and not self._pending and self._running == 0
                if want is not None:
                    done = want.issubset(self._results.keys())
                if done:
                    return dict(self._results)
                left = None if timeout is None else timeout - (time.monotonic() - t0)
                if left is not None and left <= 0:
                    raise TimeoutError("requests still running")
                self._lock.wait(timeout=left if left is not None else 1.0)

    def close(self):
        with self._lock:
            self._closed = True
            self._lock.notify_all()
        for t in self._threads:
            t.join()

    # -- scheduling (called with the lock held) ----------------------------
    def _admit(self):
        now = time.monotonic()
        while self._idle and self._pending:
            head, head_fp = self._pending[0]
            reserve = now - head.t_arrival >= self.starvation_s
            pick = None
            for i, (req, fp) in enumerate(self._pending):
                if self._in_use + fp <= self.budget:
                    pick = i
                    break
                if reserve:           # the head waits for memory: admit nothing else
                    break
            if pick is None:
                return
            req, fp = self._pending[pick]
            del self._pending[pick]
            w = self._idle.pop()
            self._in_use += fp
            self._running += 1
            self.peak_in_use = max(self.peak_in_use, self._in_use)
            self.max_concurrent = max(self.max_concurrent, self._running)
            self._work[w].append((req, fp, time.monotonic()))
            self._lock.notify_all()

    # -- workers -----------------------------------------------------------
    def _worker(self, w: int):
        if self.device is not None:
            torch.cuda.set_device(self.device)
        stream = self._streams[w]
        while True:
            with self._lock:
                while not self._work[w] and not self._closed:
                    self._lock.wait()
                if not self._work[w]:
                    return
                req, fp, t_admit = self._work[w].popleft()
            err = None
            try:
                res = self._solve(req, self.device, stream)
            except Exception as e:       # reported per request; the loop goes on
                err = f"{type(e).__name__}: {e}"
                res = Result(id=req.id, u=np.zeros(0), iterations=0, true_rel_res=float("nan"),
                             status=-99, footprint=fp, t_arrival=req.t_arrival,
                             t_admit=t_admit, t_done=0.0, error=err)
            res.footprint = fp
            res.t_arrival = req.t_arrival
            res.t_admit = t_admit
            res.t_done = time.monotonic()
            with self._lock:
                self._results[req.id] = res
                self._in_use -= fp
                self._running -= 1
                self._idle.add(w)
                self._admit()
                self._lock.notify_all()


def summarize(results: List[Result], wall_s: float) -> dict:
    lat = np.array([r.latency for r in results])
    q = np.array([r.queued for r in results])
    ok = sum(1 for r in results if r.status == 0)
    return {"requests": len(results), "converged": ok, "solves_per_s": len(results) / wall_s,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "queue_p50_ms": float(np.percentile(q, 50) * 1e3),
            "queue_p99_ms": float(np.percentile(q, 99) * 1e3),
            "max_iterations": int(max(r.iterations for r in results))}
