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
    """Requests of mixed size, BC, scheme and precision arriving over 30 ms, served from resident pools
    (ticks of 16 explicit / 4 BTCS steps, so requests span several ticks and join mid-run): every result
    matches the oracle and equals the request's solo run bitwise; the budget holds."""
    from paper_2601_12204_amd.serve import GpuBackend, Server
    reqs, offsets = _mix(90 + budget_mb % 7, 60)
    announce(f"serve 60 mixed requests, budget {budget_mb} MiB")
    backend = GpuBackend(slots=16, max_nodes=20000, tick_steps={W.EXPLICIT: 16, W.BTCS: 4})
    srv = Server(backend=backend, hbm_budget=budget_mb << 20)
    stats = srv.run(reqs, offsets)
    assert stats["requests"] == 60 and all(r.result is not None for r in reqs)
    assert srv.peak_used <= srv.budget
    assert all(r.path == "pool" for r in reqs) and stats["ticks"] > 10
    worst = check_served_against_oracle(reqs)
    announce(f"served vs oracle, worst per (dtype, steps): {worst}")
    for r in reqs:
        assert np.array_equal(r.result, _alone(r)), r.rid


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme", [W.EXPLICIT, W.BTCS])
def test_pool_slots_equal_context_runs(dtype, scheme):
    """The pool through the C ABI: problems on and beyond the on-chip limit (whole instances of every
    width class, explicit windows, truncated BTCS windows), admitted between ticks, with step counts that
    are not multiples of the tick, each retired state bitwise equal to a context's run of the problem."""
    import torch
    import paper_2601_12204_amd as B
    sizes = [3, 40, 700, 1500, 3000, 8192, 8194, 9000, 20000, 33333]
    b = W.random_batch(701 + scheme, len(sizes), 3, 3, amplitude=2.0)
    probs, states = [], []
    for k, n in enumerate(sizes):
        one = W.random_batch(711 + 3 * k + scheme, 1, n, n, scheme=scheme, amplitude=2.0)
        probs.append(one.problems[0])
        states.append(one.instance(0))
    batch = set_cfl_steps(W._pack(probs, states), scheme=scheme)
    td = torch.float64 if dtype == "f64" else torch.float32
    npd = np.float64 if dtype == "f64" else np.float32
    tick = 7 if scheme == W.EXPLICIT else 3
    steps = [5 + 3 * k for k in range(len(sizes))]
    announce(f"pool {dtype} scheme={scheme} {len(sizes)} problems, tick {tick}")
    stream = torch.cuda.current_stream()
    pool = B.Pool(td, scheme, 4, 40000, tick)
    inputs = [torch.from_numpy(np.ascontiguousarray(batch.instance(k), dtype=npd)).to("cuda") for k in range(len(sizes))]
    outputs = [torch.empty_like(x) for x in inputs]
    waiting = list(range(len(sizes)))
    slot_of = {}
    done = set()
    for _ in range(1000):
        for s, k in list(slot_of.items()):
            if pool.remaining(s) == 0:
                assert pool.retire(s, outputs[k].data_ptr()) == 0
                del slot_of[s]
                done.add(k)
        while waiting:
            s = pool.admit(batch.problems[waiting[0]], inputs[waiting[0]].data_ptr(), steps[waiting[0]])
            if s < 0:
                break
            slot_of[s] = waiting.pop(0)
        if not slot_of and not waiting:
            break
        pool.tick()
    stream.synchronize()
    assert len(done) == len(sizes)
    pool.close()
    for k in range(len(sizes)):
        s = B.Solver([batch.problems[k]], dtype=td)
        u = s.pack([batch.instance(k)])
        s.run(u, steps[k])
        s.sync()
        ref = s.unpack(u)[0]
        s.close()
        assert np.array_equal(outputs[k].cpu().numpy(), ref), (k, sizes[k])
