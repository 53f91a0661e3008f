"""Continuous-batching serving loop for Burgers solves on one GPU.

Requests (a problem, its initial state, a step count and a precision) arrive over time.  The loop keeps
them in resident slot pools of the library (``burgers_pool_*``): one pool per precision and scheme,
each a fixed set of device slots with a device slot table, created once, on its own HIP stream.

  * Admission: queued requests are admitted in arrival order into free slots while the HBM budget
    allows (the sum of the admitted requests' footprints stays within it).  A request that does not fit
    the budget stops admission (no overtaking on memory); a request whose pool has no free slot waits
    while later requests of other pools go ahead.
  * Ticks: whenever a pool's previous tick has finished, the loop retires its finished slots, admits
    into it, and enqueues the next tick, which advances every occupied slot by up to the pool's tick
    steps in one graph-replayed launch sequence.  Requests that arrive while others run join at the next
    tick boundary, and their work shares the launches of the slots already in flight.
  * Retirement: a finished slot's state is copied to pinned host memory on the pool's stream; the
    request completes when that copy has landed.

Latency of a request = completion time - arrival time.  A slot runs the kernels a context would run for
its problem alone, so a request's result does not depend on what else is in flight.  Requests a pool
cannot hold (other schemes, grids beyond the pools' slot size) run as one-off cohorts on a context;
so does a BTCS request whose truncated-window bound failed in the pool (the context redoes those steps
exactly).

The GPU work sits behind a backend interface; the admission and retirement logic is plain Python and
runs against any backend with the same calls (the tests use a fake one without a GPU).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np

ALIGN = 64
EXPLICIT = 0
BTCS = 1


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
    path: str = ""             # "pool" or "cohort"

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival

    def updates(self) -> int:
        n = int(self.problem.n)
        return (n if self.problem.bc == 0 else n - 2) * self.nsteps


def footprint(req: Request) -> int:
    """Device bytes a request holds while in flight: its state and a second state buffer, the binary64
    reduced-system arrays a BTCS instance may need, and a fixed allowance for tables."""
    n = int(req.problem.n)
    word = 8 if req.dtype == "f64" else 4
    padded = (n + ALIGN - 1) // ALIGN * ALIGN
    total = 2 * padded * word + 4096
    if n >= 32:
        total += (n // 8 + 64) * 4 * 8
    return total


class GpuBackend:
    """Resident pools through the library, plus one-off cohort contexts for requests no pool holds.

    Each pool has pinned host staging of its own, one region per slot for initial states and one for
    results, allocated with the pool: admitting or retiring a request allocates nothing.  A slot returns
    to the free list only once its result has been copied out of the staging."""

    def __init__(self, slots: int = 128, max_nodes: int = 65536, tick_steps: Optional[Dict[int, int]] = None,
                 cohort_streams: int = 2):
        import torch
        import paper_2601_12204_amd as B
        self.torch = torch
        self.B = B
        self.slots = slots
        self.max_nodes = max_nodes
        self.cap = (max_nodes + ALIGN - 1) // ALIGN * ALIGN
        self.tick_steps = tick_steps or {EXPLICIT: 1000, BTCS: 100}
        self.pools: Dict[tuple, object] = {}
        self.streams: Dict[tuple, object] = {}
        self.occupant: Dict[tuple, Dict[int, Request]] = {}     # key -> slot -> request being advanced
        self.free: Dict[tuple, List[int]] = {}
        self.stage_in: Dict[tuple, object] = {}
        self.stage_out: Dict[tuple, object] = {}
        self.cohort_streams = [torch.cuda.Stream() for _ in range(cohort_streams)]
        self.next_cohort = 0

    # -- pools ---------------------------------------------------------------------------------------
    def key(self, req: Request):
        if int(req.problem.scheme) not in (EXPLICIT, BTCS) or int(req.problem.n) > self.max_nodes:
            return None
        return (req.dtype, int(req.problem.scheme))

    def _pool(self, key):
        if key not in self.pools:
            torch = self.torch
            dtype, scheme = key
            td = torch.float64 if dtype == "f64" else torch.float32
            stream = torch.cuda.Stream()
            self.streams[key] = stream
            self.pools[key] = self.B.Pool(td, scheme, self.slots, self.max_nodes, self.tick_steps[scheme],
                                          stream=stream.cuda_stream)
            self.stage_in[key] = torch.empty(self.slots * self.cap, dtype=td, pin_memory=True)
            self.stage_out[key] = torch.empty(self.slots * self.cap, dtype=td, pin_memory=True)
            self.occupant[key] = {}
            self.free[key] = list(range(self.slots))
        return self.pools[key]

    def keys(self):
        return list(self.pools.keys())

    def free_slots(self, key) -> int:
        self._pool(key)
        return len(self.free[key])

    def admit(self, key, req: Request) -> bool:
        pool = self._pool(key)
        if not self.free[key]:
            return False
        slot = min(self.free[key])
        stage = self.stage_in[key]
        n = int(req.problem.n)
        stage.numpy()[slot * self.cap:slot * self.cap + n] = req.u0
        ptr = stage.data_ptr() + slot * self.cap * stage.element_size()
        got = pool.admit(req.problem, ptr, req.nsteps, slot)
        if got != slot:
            raise RuntimeError(f"pool admitted into slot {got}, expected {slot}")
        self.free[key].remove(slot)
        self.occupant[key][slot] = req
        return True

    def occupied(self, key) -> int:
        return len(self.occupant.get(key, {}))

    def idle(self, key) -> bool:
        return not self._pool(key).busy()

    def active(self, key) -> bool:
        pool = self._pool(key)
        return any(pool.remaining(s) > 0 for s in self.occupant[key])

    def tick(self, key) -> None:
        self._pool(key).tick()

    def finished(self, key) -> List[int]:
        pool = self._pool(key)
        return [s for s in self.occupant[key] if pool.remaining(s) == 0]

    def retire(self, key, slots: Sequence[int]):
        pool = self._pool(key)
        stage = self.stage_out[key]
        items = []
        for s in slots:
            req = self.occupant[key].pop(s)
            status = pool.retire(s, stage.data_ptr() + s * self.cap * stage.element_size())
            items.append((req, s, status))
        event = self.torch.cuda.Event()
        event.record(self.streams[key])
        return {"event": event, "items": items, "key": key}

    # -- one-off cohorts -----------------------------------------------------------------------------
    def launch(self, reqs: Sequence[Request]):
        torch = self.torch
        stream = self.cohort_streams[self.next_cohort % len(self.cohort_streams)]
        self.next_cohort += 1
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
        items = [(r, None, 0) for r in reqs]
        return {"event": event, "items": items, "solver": solver, "u": u, "host_in": host, "out": out}

    # -- results -------------------------------------------------------------------------------------
    def ready(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, handle) -> List[Tuple[Request, np.ndarray, int]]:
        handle["event"].synchronize()
        if "solver" in handle:
            solver = handle["solver"]
            out = handle["out"].numpy()
            res = [(r, out[solver.offsets[b]:solver.offsets[b] + int(r.problem.n)].astype(np.float64), 0)
                   for b, (r, _, _) in enumerate(handle["items"])]
            solver.close()
            return res
        key = handle["key"]
        out = self.stage_out[key].numpy()
        res = []
        for r, s, st in handle["items"]:
            res.append((r, out[s * self.cap:s * self.cap + int(r.problem.n)].astype(np.float64), st))
            self.free[key].append(s)           # the staging region is read: the slot can take a request
        return res


class Server:
    def __init__(self, backend=None, hbm_budget: int = 8 << 30, clock: Callable[[], float] = time.perf_counter):
        self.backend = backend if backend is not None else GpuBackend()
        self.budget = hbm_budget
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.pending: List[dict] = []          # result handles (retired slots, cohorts) not yet landed
        self.used = 0
        self.peak_used = 0
        self.finished: List[Request] = []
        self.ticks = 0
        self.cohorts = 0
        self.redone = 0

    # -- requests --------------------------------------------------------------------------------------
    def submit(self, req: Request) -> None:
        if footprint(req) > self.budget:
            raise ValueError(f"request {req.rid} needs {footprint(req)} bytes, above the whole budget")
        self.queue.append(req)

    # -- one pass of the loop --------------------------------------------------------------------------
    def poll(self) -> bool:
        """Collect landed results, then for every pool whose tick has finished: retire, admit, tick.
        Returns True if anything happened."""
        progressed = self._collect()
        progressed = self._admit() or progressed
        for key in self.backend.keys():
            if not self.backend.idle(key):
                continue
            done = self.backend.finished(key)
            if done:
                self.pending.append(self.backend.retire(key, done))
                progressed = True
            if self.backend.active(key):
                self.backend.tick(key)
                self.ticks += 1
                progressed = True
        return progressed

    def _collect(self) -> bool:
        done_any = False
        keep = []
        for h in self.pending:
            if not self.backend.ready(h):
                keep.append(h)
                continue
            now = self.clock()
            for r, res, status in self.backend.collect(h):
                if status != 0:                # failed window bound in the pool: redo exactly on a context
                    self.redone += 1
                    r.path = "cohort"
                    keep.append(self.backend.launch([r]))
                    self.cohorts += 1
                    continue
                r.result = res
                r.done = now
                self.used -= footprint(r)
                self.finished.append(r)
            done_any = True
        self.pending = keep
        return done_any

    def _admit(self) -> bool:
        admitted = False
        now = self.clock()
        waiting: List[Request] = []
        while self.queue:
            r = self.queue.popleft()
            need = footprint(r)
            if need > self.budget - self.used:
                self.queue.appendleft(r)       # first come, first served on memory: no overtaking
                break
            key = self.backend.key(r)
            if key is None:                    # no pool holds it: a one-off cohort
                r.admitted, r.path = now, "cohort"
                self.pending.append(self.backend.launch([r]))
                self.cohorts += 1
            elif self.backend.free_slots(key) > 0 and self.backend.admit(key, r):
                r.admitted, r.path = now, "pool"
            else:
                waiting.append(r)              # its pool is full; later requests of other pools go on
                continue
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            admitted = True
        for r in reversed(waiting):            # back to the head of the queue, order kept
            self.queue.appendleft(r)
        return admitted

    def drain(self, idle_sleep: float = 0.0001) -> None:
        while self.queue or self.pending or self._busy():
            if not self.poll():
                time.sleep(idle_sleep)

    def _busy(self) -> bool:
        return any(self.backend.occupied(k) for k in self.backend.keys())

    # -- real-time driver ------------------------------------------------------------------------------
    def run(self, requests: Sequence[Request], offsets: Sequence[float], idle_sleep: float = 0.00005) -> dict:
        """Feed `requests` at wall-clock offsets (seconds from now), serve until all are done, and return
        latency percentiles and throughput."""
        order = np.argsort(np.asarray(offsets), kind="stable")
        t0 = self.clock()
        k = 0
        while k < len(order) or self.queue or self.pending or self._busy():
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
                "glups": updates / wall / 1e9, "ticks": self.ticks, "cohorts": self.cohorts,
                "redone": self.redone, "peak_bytes": self.peak_used, "budget_bytes": self.budget}
