"""Serving loop on the GPU: every served result matches the oracle, results alone equal results in the
mix, and the budget is respected."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, check_batch, set_cfl_steps

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


def check_served_against_oracle(reqs):
    """Served results against the oracle with the parity bars of the solvers: FP64 within 1e-12
    (relative max-abs per instance), FP32 explicit bitwise equal to the FP32 oracle, FP32 BTCS within 1e-5
    of the exact discrete solution (binary64 solve of a binary32 state)."""
    groups = {}
    for r in reqs:
        groups.setdefault((r.dtype, r.nsteps), []).append(r)
    worst = {}
    for (dtype, nsteps), rs in sorted(groups.items()):
        batch = W._pack([r.problem for r in rs], [np.asarray(r.u0, dtype=np.float64) for r in rs])
        got = np.concatenate([np.asarray(r.result, dtype=np.float64) for r in rs])
        if dtype == "f32":
            got = got.astype(np.float32)
        w = check_batch(batch, got, nsteps, dtype)
        worst[(dtype, nsteps)] = w
    return worst


@pytest.mark.parametrize("budget_mb", [8192, 2])
def test_served_results_match_oracle_and_solo_runs(budget_mb):
    from paper_2601_12204_amd.serve import Server
    reqs, offsets = _mix(90 + budget_mb % 7, 60)
    announce(f"serve 60 mixed requests, budget {budget_mb} MiB")
    srv = Server(hbm_budget=budget_mb << 20, batch_window=0.002)
    stats = srv.run(reqs, offsets)
    assert stats["requests"] == 60 and all(r.result is not None for r in reqs)
    assert srv.peak_used <= srv.budget
    if budget_mb == 2:
        assert stats["cohorts"] > 10          # the small budget forced many small cohorts
    worst = check_served_against_oracle(reqs)
    announce(f"served vs oracle, worst per (dtype, steps): {worst}")
    for r in reqs:
        assert np.array_equal(r.result, _alone(r)), r.rid
