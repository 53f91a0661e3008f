"""Continuous-batching serving loop for Burgers solves on one GPU.

Requests (a problem, its initial state, a step count and a precision) arrive over time.  The loop

  * queues them in arrival order;
  * admits queued requests, strictly first-come first-served, while the HBM budget and the number of
    cohorts in flight allow, gathering the requests that arrive within one batching window into a
    cohort (one library context per precision, scheme and step count, so a cohort is one batched launch
    sequence over all its instances);
  * runs every cohort on its own HIP stream, so cohorts admitted while others are still on the GPU
    overlap with them on the device;
  * retires a cohort as soon as its completion event has fired: its states come back through pinned
    host memory, each request gets its completion time, and the cohort's memory returns to the budget.

Latency of a request = completion time - arrival time.  Every instance of a cohort is advanced by the
same kernels it would get alone (the kernel path of an instance depends only on its own size and
scheme), so a request's result does not depend on which other requests share its cohort.

The GPU work sits behind a small backend interface (``GpuBackend``); the admission and retirement logic
is plain Python and can run against any backend with the same three calls.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence

import numpy as np

ALIGN = 64


@dataclasses.dataclass
class Request:
    rid: int
    problem: object            # n, length, nu, dt, bc, scheme, left, right
    u0: np.ndarray             # initial state (n values)
    nsteps: int
    dtype: str = "f64"         # "f64" or "f32"
    arrival: float = 0.0
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[np.ndarray] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival

    def updates(self) -> int:
        n = int(self.problem.n)
        return (n if self.problem.bc == 0 else n - 2) * self.nsteps


def footprint(req: Request) -> int:
    """Device bytes a request holds while in flight: its state and the context's second buffer, the
    binary64 reduced-system arrays a BTCS instance may need, and a fixed allowance for tables."""
    n = int(req.problem.n)
    word = 8 if req.dtype == "f64" else 4
    padded = (n + ALIGN - 1) // ALIGN * ALIGN
    total = 2 * padded * word + 4096
    if n >= 32:
        total += (n // 8 + 64) * 4 * 8
    return total


class GpuBackend:
    """Runs cohorts through the library on a pool of HIP streams (default priority)."""

    def __init__(self, streams: int = 4):
        import torch
        import paper_2601_12204_amd as B
        self.torch = torch
        self.B = B
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.next = 0

    def launch(self, reqs: Sequence[Request]):
        torch = self.torch
        stream = self.streams[self.next % len(self.streams)]
        self.next += 1
        td = torch.float64 if reqs[0].dtype == "f64" else torch.float32
        with torch.cuda.stream(stream):
            solver = self.B.Solver([r.problem for r in reqs], dtype=td, stream=stream.cuda_stream)
            host = torch.zeros(solver.elems, dtype=td, pin_memory=True)
            hv = host.numpy()
            for b, r in enumerate(reqs):
                hv[solver.offsets[b]:solver.offsets[b] + len(r.u0)] = r.u0
            u = host.to("cuda", non_blocking=True)
            solver.run(u, reqs[0].nsteps)
            out = torch.empty(solver.elems, dtype=td, pin_memory=True)
            out.copy_(u, non_blocking=True)
            event = torch.cuda.Event()
            event.record(stream)
        return {"solver": solver, "u": u, "host_in": host, "out": out, "event": event}

    def ready(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, handle, reqs: Sequence[Request]) -> List[np.ndarray]:
        handle["event"].synchronize()
        solver = handle["solver"]
        out = handle["out"].numpy()
        res = [out[solver.offsets[b]:solver.offsets[b] + int(r.problem.n)].astype(np.float64) for b, r in enumerate(reqs)]
        solver.close()
        return res


class Server:
    def __init__(self, backend=None, hbm_budget: int = 8 << 30, max_in_flight: int = 64,
                 batch_window: float = 0.001, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter):
        self.backend = backend if backend is not None else GpuBackend()
        self.budget = hbm_budget
        self.max_in_flight = max_in_flight
        self.window = batch_window
        self.max_batch = max_batch
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.in_flight: List[tuple] = []      # (handle, requests, bytes)
        self.used = 0
        self.peak_used = 0
        self.finished: List[Request] = []
        self.cohorts = 0

    # -- requests --------------------------------------------------------------------------------------
    def submit(self, req: Request) -> None:
        if footprint(req) > self.budget:
            raise ValueError(f"request {req.rid} needs {footprint(req)} bytes, above the whole budget")
        self.queue.append(req)

    # -- one pass of the loop --------------------------------------------------------------------------
    def poll(self) -> bool:
        """Retire finished cohorts, then admit what fits.  Returns True if anything happened."""
        progressed = self._retire()
        return self._admit() or progressed

    def _retire(self) -> bool:
        done_any = False
        keep = []
        for handle, reqs, nbytes in self.in_flight:
            if self.backend.ready(handle):
                results = self.backend.collect(handle, reqs)
                now = self.clock()
                for r, res in zip(reqs, results):
                    r.result = res
                    r.done = now
                    self.finished.append(r)
                self.used -= nbytes
                done_any = True
            else:
                keep.append((handle, reqs, nbytes))
        self.in_flight = keep
        return done_any

    def _admit(self) -> bool:
        if not self.queue:
            return False
        now = self.clock()
        if now - self.queue[0].arrival < self.window and len(self.queue) < self.max_batch:
            return False                       # let the batching window fill
        admitted: List[Request] = []
        free = self.budget - self.used
        while self.queue and len(admitted) < self.max_batch:
            need = footprint(self.queue[0])
            if need > free:
                break                          # first come, first served: no overtaking
            r = self.queue.popleft()
            r.admitted = now
            free -= need
            admitted.append(r)
        if not admitted:
            return False
        groups: Dict[tuple, List[Request]] = collections.OrderedDict()
        for r in admitted:
            groups.setdefault((r.dtype, int(r.problem.scheme), r.nsteps), []).append(r)
        launched = False
        leftover: List[Request] = []
        for key, reqs in groups.items():
            if len(self.in_flight) >= self.max_in_flight:
                leftover.extend(reqs)
                continue
            nbytes = sum(footprint(r) for r in reqs)
            handle = self.backend.launch(reqs)
            self.in_flight.append((handle, reqs, nbytes))
            self.used += nbytes
            self.peak_used = max(self.peak_used, self.used)
            self.cohorts += 1
            launched = True
        for r in reversed(leftover):           # back to the head of the queue, order kept
            r.admitted = None
            self.queue.appendleft(r)
        return launched

    def drain(self, idle_sleep: float = 0.0001) -> None:
        while self.queue or self.in_flight:
            if not self.poll():
                time.sleep(idle_sleep)

    # -- real-time driver ------------------------------------------------------------------------------
    def run(self, requests: Sequence[Request], offsets: Sequence[float], idle_sleep: float = 0.00005) -> dict:
        """Feed `requests` at wall-clock offsets (seconds from now), serve until all are done, and return
        latency percentiles and throughput."""
        order = np.argsort(np.asarray(offsets), kind="stable")
        t0 = self.clock()
        k = 0
        while k < len(order) or self.queue or self.in_flight:
            now = self.clock()
            while k < len(order) and t0 + offsets[order[k]] <= now:
                req = requests[order[k]]
                req.arrival = t0 + offsets[order[k]]
                self.submit(req)
                k += 1
            if not self.poll():
                time.sleep(idle_sleep)
        wall = self.clock() - t0
        lat = np.array([r.latency for r in requests])
        updates = sum(r.updates() for r in requests)
        return {"requests": len(requests), "wall_s": wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "glups": updates / wall / 1e9, "cohorts": self.cohorts, "peak_bytes": self.peak_used,
                "budget_bytes": self.budget}
