"""The allocation-free entry point burgers_run_static against burgers_run on a context: the same kernels,
so bitwise the same states (and both within the parity bars of the oracle), on two calls in a row that
reuse the static scratch, the second with a smaller input; inputs beyond the scratch are rejected with the
state untouched."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, check_batch, set_cfl_steps

pytestmark = pytest.mark.gpu


def _batch(seed, count, n_hi):
    b = W.random_batch(seed, count, 3, n_hi, amplitude=2.0)
    for k, p in enumerate(b.problems):
        p.scheme = (W.EXPLICIT, W.BTCS, W.RK4, W.CN)[k % 4]
    return set_cfl_steps(b, btcs_factor=10.0)


def _static_run(batch, dtype, nsteps):
    import torch
    import paper_2601_12204_amd as B
    td = torch.float64 if dtype == "f64" else torch.float32
    off = B.packed_offsets(batch.problems)
    host = np.zeros(int(off[-1]), dtype=np.float64 if dtype == "f64" else np.float32)
    for b in range(len(batch.problems)):
        s = batch.instance(b)
        host[off[b]:off[b] + len(s)] = s
    u = torch.from_numpy(host).to("cuda")
    B.burgers_run_static(batch.problems, u, nsteps)
    return u, off


def _dense(u, off, problems):
    host = u.detach().cpu().numpy()
    return np.concatenate([host[off[b]:off[b] + int(p.n)] for b, p in enumerate(problems)])


def _context_run(batch, dtype, nsteps):
    import torch
    import paper_2601_12204_amd as B
    s = B.Solver(batch.problems, dtype=torch.float64 if dtype == "f64" else torch.float32)
    try:
        u = s.pack_flat(batch.u0, batch.offsets)
        s.run(u, nsteps)
        s.sync()
        return s.unpack_flat(u)
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_run_static_matches_run_on_two_calls(dtype):
    import torch
    # the first batch has windowed explicit instances and partitioned BTCS systems (second state buffer
    # and reduced systems in the scratch); the second is smaller and reuses the same scratch
    big = _batch(601, 24, 60000)
    small = _batch(602, 9, 3000)
    nsteps = 7
    announce(f"run_static {dtype}: {len(big.problems)} then {len(small.problems)} instances")
    u1, off1 = _static_run(big, dtype, nsteps)
    u2, off2 = _static_run(small, dtype, nsteps)
    torch.cuda.synchronize()
    got1 = _dense(u1, off1, big.problems)
    got2 = _dense(u2, off2, small.problems)
    ref1 = _context_run(big, dtype, nsteps)
    ref2 = _context_run(small, dtype, nsteps)
    assert np.array_equal(got1, ref1)
    assert np.array_equal(got2, ref2)
    check_batch(big, got1, nsteps, dtype)
    check_batch(small, got2, nsteps, dtype)


def test_run_static_rejects_beyond_the_scratch():
    import torch
    import paper_2601_12204_amd as B
    n = B.STATIC_SCRATCH_BYTES // 8 + 64          # the second FP64 state buffer alone exceeds the scratch
    p = W.Problem(n=n, length=1.0, nu=1e-3, dt=1e-9, bc=W.BC_PERIODIC, scheme=W.EXPLICIT)
    u = torch.linspace(0.0, 1.0, n, dtype=torch.float64, device="cuda")
    before = u.clone()
    announce("run_static beyond the scratch")
    with pytest.raises(B.BurgersError) as err:
        B.burgers_run_static([p], u, 3)
    assert err.value.status == -6
    torch.cuda.synchronize()
    assert torch.equal(u, before)
