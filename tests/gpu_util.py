"""Shared helpers of the GPU parity tests: time steps, oracle runs and device runs on the same inputs."""
import math
import sys

import numpy as np

import oracle
import workloads as W

TOL_F64 = 1e-12     # relative max-abs, FP64 device vs FP64 oracle
TOL_F32 = 1e-5      # relative max-abs, FP32 device vs FP32 oracle


def announce(msg: str) -> None:
    """Name the case on the real stderr before a device step (survives output capture and crashes)."""
    sys.__stderr__.write(f"[gpu case] {msg}\n")
    sys.__stderr__.flush()


def set_cfl_steps(batch, sigma=0.5, explicit_factor=1.0, btcs_factor=10.0, scheme=None):
    """dt = factor * sigma * min(dx/max|u0|, dx^2/(2 nu)); the library's and the oracle's CFL step agree
    bitwise (checked), and the oracle's value is used."""
    import paper_2601_12204_amd as B
    for i, p in enumerate(batch.problems):
        s = p.scheme if scheme is None else scheme
        f = btcs_factor if s == W.BTCS else explicit_factor
        d0 = oracle.cfl_dt(p.n, p.length, p.nu, p.bc, float(batch.umax[i]), sigma)
        d1 = B.burgers_cfl_dt(p, float(batch.umax[i]), sigma)
        assert d0 == d1
        p.dt = f * d0
    return batch


def oracle_run(batch, nsteps, dtype, scheme=None, threads=0):
    u = batch.u0.astype(np.float32) if dtype == "f32" else batch.u0
    return oracle.run(batch.problems, u, batch.offsets, nsteps, scheme=scheme, threads=threads)


def device_run(batch, nsteps, dtype, how="run", plan=None, reps=1):
    """Run on the device through the C ABI; returns the dense concatenation of the instances."""
    import torch
    import paper_2601_12204_amd as B
    td = torch.float64 if dtype == "f64" else torch.float32
    solver = B.Solver(batch.problems, dtype=td)
    try:
        if plan:
            solver.set_plan(**plan)
        u = solver.pack_flat(batch.u0, batch.offsets)
        for _ in range(reps):
            getattr(solver, how)(u, nsteps)
        solver.sync()
        torch.cuda.synchronize()
        return solver.unpack_flat(u)
    finally:
        solver.close()


def rel_err(a, ref):
    return oracle.rel_max_abs(a, ref)


def assert_explicit_parity(batch, got, ref, dtype):
    """Explicit-scheme instances against the oracle of the same precision: FP64 within TOL_F64 per
    instance, FP32 bitwise."""
    if dtype == "f32":
        assert np.array_equal(got, ref)
        return
    errs = per_instance_rel(batch, got, ref)
    assert errs.max() <= TOL_F64, errs


def per_instance_rel(batch, a, ref):
    out = []
    for b in range(batch.count):
        s, e = batch.offsets[b], batch.offsets[b + 1]
        out.append(oracle.rel_max_abs(a[s:e], ref[s:e]))
    return np.array(out)


def check_batch(batch, got, nsteps, dtype, scheme=None, threads=0):
    """Apply the parity bars per instance and return the worst relative errors.

    FP64: every instance within TOL_F64 of the FP64 oracle (the binary64 explicit update is a fused
    convex combination, which rounds differently from the oracle's association).
    FP32: explicit instances bitwise equal to the FP32 oracle (the binary32 update keeps its association).  Implicit (BTCS and Crank-Nicolson)
    instances (solved in binary64 with a binary32 state) within TOL_F32 of the exact discrete solution,
    i.e. the FP64 oracle run from the same binary32-rounded initial state, and within TOL_F32 plus the
    FP32 oracle's own distance from that solution of the FP32 oracle.
    """
    explicit_kind = (W.EXPLICIT, W.RK4)
    worst = {"explicit": 0.0, "btcs": 0.0, "btcs_vs_f32_oracle": 0.0}
    schemes = [p.scheme if scheme is None else scheme for p in batch.problems]
    if dtype == "f64":
        ref = oracle_run(batch, nsteps, "f64", scheme=scheme, threads=threads)
        for b, s in enumerate(schemes):
            lo, hi = batch.offsets[b], batch.offsets[b + 1]
            e = rel_err(got[lo:hi], ref[lo:hi])
            key = "explicit" if s in explicit_kind else "btcs"
            worst[key] = max(worst[key], e)
            assert e <= TOL_F64, (b, batch.problems[b], e)
        return worst
    ref32 = oracle_run(batch, nsteps, "f32", scheme=scheme, threads=threads)
    exact = None
    if any(s not in explicit_kind for s in schemes):
        u0 = batch.u0.astype(np.float32).astype(np.float64)
        exact = oracle.run(batch.problems, u0, batch.offsets, nsteps, scheme=scheme, threads=threads)
    for b, s in enumerate(schemes):
        lo, hi = batch.offsets[b], batch.offsets[b + 1]
        if s in explicit_kind:
            assert np.array_equal(got[lo:hi], ref32[lo:hi]), b
            continue
        e = rel_err(got[lo:hi], exact[lo:hi])
        own = rel_err(ref32[lo:hi], exact[lo:hi])
        e32 = rel_err(got[lo:hi], ref32[lo:hi])
        worst["btcs"] = max(worst["btcs"], e)
        worst["btcs_vs_f32_oracle"] = max(worst["btcs_vs_f32_oracle"], e32)
        assert e <= TOL_F32, (b, batch.problems[b], e)
        assert e32 <= own + TOL_F32, (b, e32, own)
    return worst
