"""Admission, tick and retirement logic of the serving loop, against a fake backend (no GPU): resident
pools with a fixed slot count that advance their occupied slots tick by tick."""
import numpy as np
import pytest

import workloads as W
from paper_2601_12204_amd.serve import Request, Server, footprint


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Pools keyed by (dtype, scheme) of `slots` slots; a tick advances every occupied slot by `tick`
    steps and stays busy for `delay` polls; results are the initial states.  Records admissions, ticks
    and the slot occupancy seen at each tick."""

    def __init__(self, slots=4, tick=10, delay=2, max_nodes=1 << 30):
        self.slots, self.tick_steps, self.delay, self.max_nodes = slots, tick, delay, max_nodes
        self.occupant, self.left, self.busy_for = {}, {}, {}
        self.admitted, self.tick_log, self.cohorts = [], [], []

    def key(self, req):
        if int(req.problem.scheme) not in (0, 1) or int(req.problem.n) > self.max_nodes:
            return None
        return (req.dtype, int(req.problem.scheme))

    def _pool(self, key):
        self.occupant.setdefault(key, {})
        self.busy_for.setdefault(key, 0)

    def keys(self):
        return list(self.occupant)

    def free_slots(self, key):
        self._pool(key)
        return self.slots - len(self.occupant[key])

    def admit(self, key, req):
        self._pool(key)
        free = [s for s in range(self.slots) if s not in self.occupant[key]]
        if not free:
            return False
        self.occupant[key][free[0]] = req
        self.left[(key, free[0])] = req.nsteps
        self.admitted.append(req.rid)
        return True

    def occupied(self, key):
        return len(self.occupant.get(key, {}))

    def idle(self, key):
        self._pool(key)
        if self.busy_for[key] > 0:
            self.busy_for[key] -= 1
            return False
        return True

    def active(self, key):
        return any(self.left[(key, s)] > 0 for s in self.occupant[key])

    def tick(self, key):
        assert self.busy_for[key] == 0
        self.tick_log.append((key, sorted(r.rid for s, r in self.occupant[key].items() if self.left[(key, s)] > 0)))
        for s in self.occupant[key]:
            self.left[(key, s)] -= min(self.tick_steps, self.left[(key, s)])
        self.busy_for[key] = self.delay

    def finished(self, key):
        return [s for s in self.occupant[key] if self.left[(key, s)] == 0]

    def retire(self, key, slots):
        items = [(self.occupant[key].pop(s), None, 0) for s in slots]
        return {"left": 1, "items": items}

    def launch(self, reqs):
        self.cohorts.append([r.rid for r in reqs])
        return {"left": 1, "items": [(r, None, 0) for r in reqs]}

    def ready(self, h):
        h["left"] -= 1
        return h["left"] < 0

    def collect(self, h):
        return [(r, r.u0.copy(), st) for r, _, st in h["items"]]


def _requests(k, seed=0, n_hi=5000, steps=(50, 10)):
    b = W.random_batch(seed, k, 3, n_hi, amplitude=1.0)
    return [Request(rid=i, problem=p, u0=b.instance(i).copy(), nsteps=steps[0] if p.scheme == W.EXPLICIT else steps[1],
                    dtype="f64" if i % 2 else "f32") for i, p in enumerate(b.problems)]


def _serve(srv, clock, reqs, polls=5000):
    for step in range(polls):
        clock.t = step * 1e-3
        srv.poll()
        if not srv.queue and not srv.pending and not srv._busy():
            break
    return srv


def test_all_requests_complete_and_ticks_run_only_their_pool():
    clock = FakeClock()
    be = FakeBackend(slots=3, tick=10)
    srv = Server(backend=be, hbm_budget=1 << 40, clock=clock)
    reqs = _requests(30)
    for r in reqs:
        srv.submit(r)
    _serve(srv, clock, reqs)
    assert len(srv.finished) == 30 and all(r.result is not None for r in reqs)
    assert sorted(be.admitted) == list(range(30))
    for key, rids in be.tick_log:          # a tick advances only requests of its own pool
        assert all(be.key(reqs[i]) == key for i in rids)
        assert len(rids) <= be.slots
    # an explicit request (50 steps) takes 5 ticks of 10 steps, a BTCS one (10 steps) one
    for r in reqs:
        n_ticks = sum(r.rid in rids for _, rids in be.tick_log)
        assert n_ticks == (5 if r.problem.scheme == W.EXPLICIT else 1), r.rid


def test_requests_join_between_ticks():
    """A request arriving while a pool's slots are mid-run is admitted into a free slot and advances in
    the same ticks as the ones already in flight."""
    clock = FakeClock()
    be = FakeBackend(slots=4, tick=10, delay=1)
    srv = Server(backend=be, hbm_budget=1 << 40, clock=clock)
    reqs = [r for r in _requests(20, seed=5) if r.problem.scheme == W.EXPLICIT and r.dtype == "f64"][:3]
    srv.submit(reqs[0])
    for step in range(4):
        clock.t = step * 1e-3
        srv.poll()
    srv.submit(reqs[1])
    srv.submit(reqs[2])
    _serve(srv, clock, reqs)
    shared = [rids for _, rids in be.tick_log if reqs[0].rid in rids and reqs[1].rid in rids]
    assert shared, be.tick_log
    assert all(r.result is not None for r in reqs)


def test_budget_is_never_exceeded_and_queue_waits():
    clock = FakeClock()
    be = FakeBackend(slots=64, delay=3)
    reqs = _requests(40, seed=1)
    budget = 3 * max(footprint(r) for r in reqs)
    srv = Server(backend=be, hbm_budget=budget, clock=clock)
    for r in reqs:
        srv.submit(r)
    peak_queue = 0
    for step in range(5000):
        clock.t = step * 1e-3
        srv.poll()
        assert srv.used <= budget
        peak_queue = max(peak_queue, len(srv.queue))
        if not srv.queue and not srv.pending and not srv._busy():
            break
    assert len(srv.finished) == 40
    assert srv.peak_used <= budget and peak_queue > 10


def test_first_come_first_served_on_memory():
    """No request is admitted ahead of an earlier one that is waiting for memory."""
    clock = FakeClock()
    be = FakeBackend(slots=64, delay=1)
    reqs = _requests(12, seed=2)
    big = max(reqs, key=footprint)
    budget = footprint(big) + min(footprint(r) for r in reqs) - 1
    srv = Server(backend=be, hbm_budget=budget, clock=clock)
    order = [big] + [r for r in reqs if r is not big]
    for r in order:
        srv.submit(r)
    _serve(srv, clock, order)
    admitted = [r.admitted for r in order]
    assert all(a is not None for a in admitted)
    assert all(admitted[i] <= admitted[i + 1] for i in range(len(admitted) - 1))


def test_full_pool_lets_other_pools_go_ahead():
    clock = FakeClock()
    be = FakeBackend(slots=1, tick=10, delay=5)
    reqs = _requests(40, seed=4)
    f64x = [r for r in reqs if r.dtype == "f64" and r.problem.scheme == W.EXPLICIT][:3]
    f32b = [r for r in reqs if r.dtype == "f32" and r.problem.scheme == W.BTCS][:1]
    srv = Server(backend=be, hbm_budget=1 << 40, clock=clock)
    for r in f64x + f32b:
        srv.submit(r)
    clock.t = 0.0
    srv.poll()
    assert f64x[0].admitted is not None and f64x[1].admitted is None
    assert f32b[0].admitted is not None           # another pool's request is not held up
    _serve(srv, clock, f64x + f32b)
    assert all(r.result is not None for r in f64x + f32b)


def test_unpooled_requests_run_as_cohorts():
    clock = FakeClock()
    be = FakeBackend(max_nodes=1000)
    reqs = _requests(10, seed=6, n_hi=3000)
    srv = Server(backend=be, hbm_budget=1 << 40, clock=clock)
    for r in reqs:
        srv.submit(r)
    _serve(srv, clock, reqs)
    long_ids = sorted(r.rid for r in reqs if r.problem.n > 1000)
    assert sorted(i for c in be.cohorts for i in c) == long_ids
    assert all(r.path == ("cohort" if r.problem.n > 1000 else "pool") for r in reqs)
    assert all(r.result is not None for r in reqs)


def test_oversized_request_is_rejected():
    srv = Server(backend=FakeBackend(), hbm_budget=1000)
    r = _requests(1)[0]
    with pytest.raises(ValueError):
        srv.submit(r)
