"""Serving loop on the GPU: results alone equal results in the mix; the budget is respected."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, set_cfl_steps

pytestmark = pytest.mark.gpu


def _mix(seed, k):
    b = set_cfl_steps(W.random_batch(seed, k, 3, 20000, amplitude=2.0))
    from paper_2601_12204_amd.serve import Request
    rng = np.random.default_rng(seed)
    reqs = [Request(rid=i, problem=p, u0=b.instance(i).copy(), nsteps=40 if p.scheme == W.EXPLICIT else 8,
                    dtype="f64" if rng.integers(0, 2) else "f32") for i, p in enumerate(b.problems)]
    return reqs, rng.uniform(0, 0.03, size=k)


def _alone(r):
    import torch
    import paper_2601_12204_amd as B
    s = B.Solver([r.problem], dtype=torch.float64 if r.dtype == "f64" else torch.float32)
    u = s.pack([r.u0])
    s.run(u, r.nsteps)
    s.sync()
    out = s.unpack(u)[0].astype(np.float64)
    s.close()
    return out


@pytest.mark.parametrize("budget_mb", [8192, 2])
def test_served_results_equal_solo_results(budget_mb):
    from paper_2601_12204_amd.serve import Server
    reqs, offsets = _mix(90 + budget_mb % 7, 60)
    announce(f"serve 60 mixed requests, budget {budget_mb} MiB")
    srv = Server(hbm_budget=budget_mb << 20, batch_window=0.002)
    stats = srv.run(reqs, offsets)
    assert stats["requests"] == 60 and all(r.result is not None for r in reqs)
    assert srv.peak_used <= srv.budget
    if budget_mb == 2:
        assert stats["cohorts"] > 10          # the small budget forced many small cohorts
    for r in reqs:
        assert np.array_equal(r.result, _alone(r)), r.rid
