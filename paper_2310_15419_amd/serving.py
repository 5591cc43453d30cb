"""Continuous-batching server for sketch-and-precondition least-squares solves
(paper Sec. V-E) on one GPU.

Requests min ||Ax - b|| arrive over time (A and b already resident in device
memory, as a client that uploaded them).  The server admits them in arrival
order whenever a slot (a HIP stream) is free and the request's device
footprint fits the HBM budget.  Each admitted request runs its whole pipeline
-- sketch, FP64 QR, R^{-1}, row-major copy of A, LSQR -- on its own stream, so
the work of several requests overlaps on the device.  LSQR is enqueued in
chunks of iterations; after each chunk a small asynchronous copy brings the
solver info to pinned host memory, and an event tells the server when to read
it and either enqueue the next chunk or the final x = R^{-1} y.  With one slot
the same loop is the plain per-request path (one solve at a time).

Every request's kernels depend only on its own data and tuning, so a result is
the same alone and in the mix.

A request that cannot be served fails alone: one whose arguments the library
refuses, or whose footprint exceeds the whole budget, is rejected at arrival;
one whose A fails the sketch's device validation stops before its first LSQR
iteration (stop code 8).  Its ``error`` says why and its ``x`` stays None; the
others are served as if it were not there.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import binding as B


@dataclasses.dataclass
class Request:
    rid: int
    A: "B.DeviceCsc"
    b: object                 # device FP64 tensor (m)
    params: "B.SapParams"
    arrival: float = 0.0      # seconds after the start of the run
    # filled by the server
    ws_bytes: int = 0
    admitted: float = math.nan
    done: float = math.nan
    x: object = None
    info: dict | None = None
    error: str | None = None  # set when the request failed alone (x is None)

    @property
    def footprint(self) -> int:
        """Device bytes the request holds while admitted: workspace + A + b + x."""
        a = (self.A.colptr.numel() * 8 + self.A.rowidx.numel() * 4 +
             self.A.vals.numel() * self.A.vals.element_size())
        return self.ws_bytes + a + self.b.numel() * 8 + self.A.n * 8

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Slot:
    def __init__(self, torch):
        self.stream = torch.cuda.Stream()  # default priority
        self.info_host = torch.empty(B.SapSolve.INFO_BYTES, dtype=torch.uint8, pin_memory=True)
        self.event = torch.cuda.Event()
        self.req: Request | None = None
        self.solve: B.SapSolve | None = None
        self.phase = ""


class Server:
    """hbm_budget: bytes of device memory the admitted requests may hold
    together; slots: requests in flight at most; chunk: LSQR iterations per
    enqueue."""

    def __init__(self, hbm_budget: int, slots: int, chunk: int = 16):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.slots = [_Slot(torch) for _ in range(int(slots))]
        self.peak_used = 0
        self.peak_inflight = 0

    def _enqueue_chunk(self, s: _Slot):
        torch = self.torch
        s.solve.iterate(self.chunk, s.stream)
        with torch.cuda.stream(s.stream):
            s.info_host.copy_(s.solve.ws[:B.SapSolve.INFO_BYTES], non_blocking=True)
        s.event.record(s.stream)

    def run(self, requests: list[Request], idle_sleep: float = 2e-5) -> list[Request]:
        """Serve the requests (sorted by arrival); returns them with timings."""
        torch = self.torch
        servable = []
        for r in requests:
            try:
                r.ws_bytes = B.SapSolve.workspace_bytes(r.A, r.params)
            except B.SketchError as e:
                self._reject(r, f"refused by the library: {e}")
                continue
            if r.footprint > self.budget:
                self._reject(r, f"needs {r.footprint} B of device memory, more than the "
                                f"whole budget of {self.budget} B")
                continue
            servable.append(r)
        pending = sorted(servable, key=lambda r: r.arrival)
        head = 0
        used = 0
        t0 = time.perf_counter()
        active = 0
        while head < len(pending) or active:
            progressed = False
            for s in self.slots:
                if s.req is None or not s.event.query():
                    continue
                progressed = True
                if s.phase == "iterate":
                    info = B.SapSolve.parse_info(bytes(s.info_host.numpy()))
                    if info["done"] and info["istop"] == ISTOP_INPUT:
                        # A failed the device validation: no x to compute
                        s.req.info = info
                        s.req.error = "A failed the sketch's device validation"
                        s.phase = "failed"
                    elif info["done"]:
                        s.req.info = info
                        s.solve.finish(s.stream)
                        s.event.record(s.stream)
                        s.phase = "finish"
                    else:
                        self._enqueue_chunk(s)
                if s.phase in ("finish", "failed") and s.event.query():
                    r = s.req
                    r.done = time.perf_counter() - t0
                    r.x = s.solve.x if s.phase == "finish" else None
                    used -= r.footprint
                    s.req, s.solve, s.phase = None, None, ""
                    active -= 1
            now = time.perf_counter() - t0
            while head < len(pending) and pending[head].arrival <= now:
                r = pending[head]
                free = next((s for s in self.slots if s.req is None), None)
                if free is None or used + r.footprint > self.budget:
                    break  # in arrival order: the head waits for room
                head += 1
                progressed = True
                used += r.footprint
                self.peak_used = max(self.peak_used, used)
                r.admitted = now
                with torch.cuda.stream(free.stream):
                    ws = B.alloc_workspace(r.ws_bytes, r.A.colptr.device)
                    free.solve = B.SapSolve(r.A, r.b, r.params, ws)
                free.req = r
                free.phase = "iterate"
                free.solve.begin(free.stream)
                self._enqueue_chunk(free)
                active += 1
                self.peak_inflight = max(self.peak_inflight, active)
            if not progressed:
                if head < len(pending) and not active:
                    wait = pending[head].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(idle_sleep)
        torch.cuda.synchronize()
        return requests

    @staticmethod
    def _reject(r: Request, why: str):
        r.error = why
        r.admitted = r.done = r.arrival


# LSQR stop code of a request whose A failed the sketch's device validation
ISTOP_INPUT = 8


def latency_stats(reqs: list[Request]) -> dict:
    """Latency and throughput over the served requests (failed ones counted
    apart)."""
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok])
    t_first = min(r.arrival for r in ok)
    t_last = max(r.done for r in ok)
    return {"requests": len(ok), "failed": len(reqs) - len(ok),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "solves_per_s": len(ok) / max(t_last - t_first, 1e-9),
            "iterations_mean": float(np.mean([r.info["iterations"] for r in ok]))}


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson stream with the given rate (requests/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
