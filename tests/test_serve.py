"""Admission, batching and retirement logic of the serving loop, against a fake backend (no GPU)."""
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
    """Completes a cohort after `delay` polls and returns its initial states; records what it saw."""

    def __init__(self, delay=2):
        self.delay = delay
        self.launched = []

    def launch(self, reqs):
        self.launched.append([r.rid for r in reqs])
        return {"left": self.delay}

    def ready(self, h):
        h["left"] -= 1
        return h["left"] < 0

    def collect(self, h, reqs):
        return [r.u0.copy() for r in reqs]


def _requests(k, seed=0, n_hi=5000):
    b = W.random_batch(seed, k, 3, n_hi, amplitude=1.0)
    return [Request(rid=i, problem=p, u0=b.instance(i).copy(), nsteps=10 if p.scheme == W.BTCS else 50,
                    dtype="f64" if i % 2 else "f32") for i, p in enumerate(b.problems)]


def test_all_requests_complete_in_fifo_order_with_grouping():
    clock = FakeClock()
    be = FakeBackend()
    srv = Server(backend=be, hbm_budget=1 << 40, batch_window=0.001, clock=clock)
    reqs = _requests(30)
    for i, r in enumerate(reqs):
        r.arrival = 0.0
        srv.submit(r)
    clock.t = 0.01
    for _ in range(50):
        srv.poll()
    assert len(srv.finished) == 30 and all(r.result is not None for r in reqs)
    # every cohort is homogeneous in (dtype, scheme, steps)
    for cohort in be.launched:
        keys = {(reqs[i].dtype, reqs[i].problem.scheme, reqs[i].nsteps) for i in cohort}
        assert len(keys) == 1
    flat = [i for c in be.launched for i in c]
    assert sorted(flat) == list(range(30))


def test_budget_is_never_exceeded_and_queue_waits():
    clock = FakeClock()
    be = FakeBackend(delay=3)
    reqs = _requests(40, seed=1)
    budget = 3 * max(footprint(r) for r in reqs)
    srv = Server(backend=be, hbm_budget=budget, batch_window=0.0, clock=clock)
    for r in reqs:
        srv.submit(r)
    peak_queue = 0
    for step in range(2000):
        clock.t = step * 1e-3
        srv.poll()
        assert srv.used <= budget
        peak_queue = max(peak_queue, len(srv.queue))
        if not srv.queue and not srv.in_flight:
            break
    assert len(srv.finished) == 40
    assert srv.peak_used <= budget and peak_queue > 10


def test_first_come_first_served_no_overtaking():
    clock = FakeClock()
    be = FakeBackend(delay=1)
    reqs = _requests(12, seed=2)
    big = max(reqs, key=footprint)
    budget = footprint(big) + min(footprint(r) for r in reqs) - 1
    srv = Server(backend=be, hbm_budget=budget, batch_window=0.0, clock=clock)
    order = [big] + [r for r in reqs if r is not big]
    for r in order:
        srv.submit(r)
    for step in range(500):
        clock.t = step
        srv.poll()
    admitted = [r.admitted for r in order]
    assert all(a is not None for a in admitted)
    assert all(admitted[i] <= admitted[i + 1] for i in range(len(admitted) - 1))


def test_batching_window_and_in_flight_limit():
    clock = FakeClock()
    be = FakeBackend(delay=100)
    srv = Server(backend=be, hbm_budget=1 << 40, batch_window=0.005, max_in_flight=2, clock=clock)
    reqs = _requests(20, seed=3)
    for r in reqs:
        r.arrival = 0.0
        srv.submit(r)
    clock.t = 0.001
    srv.poll()
    assert not be.launched                    # window still open
    clock.t = 0.006
    srv.poll()
    assert len(srv.in_flight) <= 2


def test_oversized_request_is_rejected():
    srv = Server(backend=FakeBackend(), hbm_budget=1000)
    r = _requests(1)[0]
    with pytest.raises(ValueError):
        srv.submit(r)
