"""Benchmark of the viscous-Burgers hot path on one MI355X.

One step = the whole hot path over one batch: the 4096-instance periodic batch (N = 8192 each, FP64,
nu ~ U[0.005, 0.1], eight-mode sine initial states) advanced 10^4 explicit steps at CFL 0.5 and then
10^3 BTCS steps at ten times that dt.  value = grid-point updates per second over the step (GLUPS,
inputs resident in HBM).  Per-kernel durations come from HIP events on the stream the kernels run on;
the FP32 batch, the single-instance latency case and the long Dirichlet grid are reported beside it, as
is the CPU oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK = 78.6e12     # flop/s, counting a fused multiply-add as two flops
# binary64 vector issue rate: 256 CUs x 4 SIMDs x 16 binary64 lanes x 2.4 GHz = 39.3e12 instructions/s
FP64_ISSUE_RATE = 256 * 4 * 16 * 2.4e9
METRIC = "grid-point updates/sec (GLUPS) + % HBM roofline; served p50/p99 latency"


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def cfl_batch(B, batch, factor):
    for i, p in enumerate(batch.problems):
        p.dt = factor * B.burgers_cfl_dt(p, float(batch.umax[i]), 0.5)


class PhaseTimer:
    """HIP events recorded on the current torch stream, which is the stream the contexts launch on."""

    def __init__(self):
        import torch
        self.torch = torch
        self.marks = []

    def mark(self, name):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        self.marks.append((name, ev))

    def spans(self):
        self.torch.cuda.synchronize()
        out = {}
        for (n0, e0), (n1, e1) in zip(self.marks[:-1], self.marks[1:]):
            out.setdefault(n0, []).append(e0.elapsed_time(e1))
        return out


def bench_c2(B, torch, dtype, steps, warmup, n_exp=10_000, n_btcs=1_000, explicit_path=0, btcs_path=0,
             btcs_block=0, btcs_pipeline=0):
    """Time `steps` passes (after `warmup`) of the explicit and BTCS runs over the 4096 x 8192 batch."""
    import workloads as W
    batch = W.c2_batch()
    exp_batch = W.c2_batch()
    cfl_batch(B, exp_batch, 1.0)
    btcs_batch = W.c2_batch()
    cfl_batch(B, btcs_batch, 10.0)
    s_exp = B.Solver(exp_batch.problems, dtype=dtype)
    s_btcs = B.Solver(btcs_batch.problems, dtype=dtype)
    s_exp.set_plan(explicit_path=explicit_path)
    s_btcs.set_plan(btcs_path=btcs_path, btcs_block=btcs_block, btcs_pipeline=btcs_pipeline)
    u_init = s_exp.pack_flat(batch.u0, batch.offsets)
    u = torch.empty_like(u_init)
    timer = PhaseTimer()
    for it in range(warmup + steps):
        u.copy_(u_init)
        if it == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        if it >= warmup:
            timer.mark("explicit")
        s_exp.step_explicit(u, n_exp)
        if it >= warmup:
            timer.mark("btcs")
        s_btcs.step_btcs(u, n_btcs)
        if it >= warmup:
            timer.mark("copy")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s_exp.sync()
    s_btcs.sync()
    spans = timer.spans()
    nodes = 4096 * 8192
    exp_ms = float(np.mean(spans["explicit"]))
    n_exp, n_btcs = max(n_exp, 1), max(n_btcs, 1)
    btcs_ms = float(np.mean(spans["btcs"]))
    step_ms = exp_ms + btcs_ms
    res = {
        "explicit_ms": exp_ms, "btcs_ms": btcs_ms, "n_exp": n_exp, "n_btcs": n_btcs,
        "explicit_launches": 1 if s_exp.get_plan()["explicit_path"] in (0, 2) else n_exp,
        "btcs_launches": 1 if s_btcs.get_plan()["btcs_path"] in (0, 2) else n_btcs,
        "updates_per_step": nodes * (n_exp + n_btcs),
        "step_ms": step_ms,
        "wall_ms_per_step": wall * 1e3 / steps,
        "glups": nodes * (n_exp + n_btcs) / (step_ms * 1e-3) / 1e9,
        "explicit_glups": nodes * n_exp / (exp_ms * 1e-3) / 1e9,
        "btcs_glups": nodes * n_btcs / (btcs_ms * 1e-3) / 1e9,
        "explicit_launch_ms": exp_ms / n_exp,
        "btcs_step_ms": btcs_ms / n_btcs,
        "plan_explicit": s_exp.get_plan(),
        "plan_btcs": s_btcs.get_plan(),
    }
    s_exp.close()
    s_btcs.close()
    return res


def bench_c2_plain(B, torch, n_exp=200, n_btcs=50):
    """The plain steppers on the C2 batch, one HBM pass per step: the streaming explicit kernel
    (plan path 1) and the per-step whole-system BTCS kernel (plan path 1), each moving the state in and
    out once per step (2 words per node).  Reports their HBM rate against the 8 TB/s peak."""
    out = {}
    nodes = 4096 * 8192
    for name, dtype, word in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        r = bench_c2(B, torch, dtype, 1, 1, n_exp=n_exp, n_btcs=n_btcs, explicit_path=1, btcs_path=1)
        variants = {}
        for tag, block, pipe in (("pipelined", 512, 1), ("1024x8", 1024, 2), ("1024x8_pipelined", 1024, 1)):
            v = bench_c2(B, torch, dtype, 1, 1, n_exp=0, n_btcs=n_btcs, explicit_path=1, btcs_path=1,
                         btcs_block=block, btcs_pipeline=pipe)
            variants[f"btcs_per_step_{tag}"] = v["btcs_step_ms"]
        for leg, ms in (("explicit_stream", r["explicit_launch_ms"]), ("btcs_per_step", r["btcs_step_ms"]),
                        *variants.items()):
            gbs = 2 * word * nodes / (ms * 1e-3) / 1e9
            out[f"{leg}_{name}"] = {"ms_per_step": ms, "glups": nodes / (ms * 1e-3) / 1e9,
                                    "algorithmic_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    return out


def bench_c2_rk4(B, torch, nsteps=2500, reps=2):
    """The C2 batch (4096 x 8192 periodic, FP64) advanced by classical RK4 (eq. 22) at the CFL dt:
    four explicit stages per step, all steps of an instance in one on-chip launch."""
    import workloads as W
    batch = W.c2_batch()
    cfl_batch(B, batch, 1.0)
    for p in batch.problems:
        p.scheme = W.RK4
    s = B.Solver(batch.problems, dtype=torch.float64)
    u0 = s.pack_flat(batch.u0, batch.offsets)
    u = torch.empty_like(u0)
    u.copy_(u0)
    s.run(u, 8)                                  # warm-up (plans)
    timer = PhaseTimer()
    for _ in range(reps):
        u.copy_(u0)
        timer.mark("run")
        s.run(u, nsteps)
        timer.mark("copy")
    ms = float(np.mean(timer.spans()["run"]))
    s.close()
    nodes = 4096 * 8192
    return {"ms": ms, "steps": nsteps, "glups": nodes * nsteps / (ms * 1e-3) / 1e9,
            "stage_glups": 4 * nodes * nsteps / (ms * 1e-3) / 1e9}


def bench_c2_cn(B, torch, nsteps=1000, reps=2):
    """The C2 batch advanced by Crank-Nicolson at 10x the explicit dt: each step one half-dt BTCS solve
    through HBM (the whole-system workgroup solver) and the combination u' = 2y - u."""
    import workloads as W
    batch = W.c2_batch()
    cfl_batch(B, batch, 10.0)
    for p in batch.problems:
        p.scheme = W.CN
    s = B.Solver(batch.problems, dtype=torch.float64)
    u0 = s.pack_flat(batch.u0, batch.offsets)
    u = torch.empty_like(u0)
    u.copy_(u0)
    s.run(u, 2)                                  # warm-up (plans)
    timer = PhaseTimer()
    for _ in range(reps):
        u.copy_(u0)
        timer.mark("run")
        s.run(u, nsteps)
        timer.mark("copy")
    ms = float(np.mean(timer.spans()["run"]))
    s.close()
    nodes = 4096 * 8192
    return {"ms": ms, "steps": nsteps, "glups": nodes * nsteps / (ms * 1e-3) / 1e9}


def bench_c2_newton(B, torch, nsteps=100, reps=2):
    """The C2 batch advanced by the fully implicit central-convection step at twice the CFL dt: four
    Newton iterations per step, each an assembly, a Jacobian solve (array path) and an update."""
    import workloads as W
    batch = W.c2_batch()
    cfl_batch(B, batch, 2.0)
    for p in batch.problems:
        p.scheme = W.NEWTON
    s = B.Solver(batch.problems, dtype=torch.float64)
    u0 = s.pack_flat(batch.u0, batch.offsets)
    u = torch.empty_like(u0)
    u.copy_(u0)
    s.run(u, 2)                                  # warm-up (plans)
    timer = PhaseTimer()
    for _ in range(reps):
        u.copy_(u0)
        timer.mark("run")
        s.run(u, nsteps)
        timer.mark("copy")
    ms = float(np.mean(timer.spans()["run"]))
    s.close()
    nodes = 4096 * 8192
    return {"ms": ms, "steps": nsteps, "newton_iters": 4, "glups": nodes * nsteps / (ms * 1e-3) / 1e9}


def bench_c1_latency(B, torch, solves=200):
    """Single periodic N=101 sawtooth to t=0.5: latency of one whole solve (explicit 113 steps, BTCS 12)."""
    import workloads as W
    out = {}
    for scheme, name, factor in ((W.EXPLICIT, "explicit", 1.0), (W.BTCS, "btcs", 10.0)):
        b = W.c1_problem(scheme)
        p = b.problems[0]
        dtmax = factor * B.burgers_cfl_dt(p, float(b.umax[0]), 0.5)
        nsteps = int(math.ceil(W.C1_T / dtmax))
        p.dt = W.C1_T / nsteps
        s = B.Solver([p], dtype=torch.float64)
        u0 = s.pack_flat(b.u0, b.offsets)
        u = torch.empty_like(u0)
        lat = []
        for i in range(solves + 5):
            u.copy_(u0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            s.run(u, nsteps)
            torch.cuda.synchronize()
            if i >= 5:
                lat.append((time.perf_counter() - t) * 1e3)
        s.close()
        out[name] = {"steps": nsteps, "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99))}
    return out


def bench_c3(B, torch, n_exp=1024, n_btcs=128):
    import workloads as W
    b = W.c3_problem()
    p = b.problems[0]
    p.dt = B.burgers_cfl_dt(p, float(b.umax[0]), 0.5)
    s = B.Solver([p], dtype=torch.float64)
    u = s.pack_flat(b.u0, b.offsets)
    timer = PhaseTimer()
    s.step_explicit(u, 8)
    timer.mark("explicit")
    s.step_explicit(u, n_exp)
    timer.mark("end")
    s.close()
    q = W.c3_problem(scheme=W.BTCS).problems[0]
    q.dt = 10 * p.dt
    s2 = B.Solver([q], dtype=torch.float64)
    s2.step_btcs(u, 2)
    timer.mark("btcs")
    s2.step_btcs(u, n_btcs)
    timer.mark("end2")
    spans = timer.spans()
    upd = p.n - 2
    out = {"explicit_glups": upd * n_exp / (spans["explicit"][0] * 1e-3) / 1e9,
           "btcs_glups": upd * n_btcs / (spans["btcs"][0] * 1e-3) / 1e9,
           "explicit_steps": n_exp, "btcs_steps": n_btcs}
    # the long-system solvers side by side (same state, same step count), eager and graph-replayed
    for name, plan in (("btcs_windows_graph", dict(use_graph=1)),
                       ("btcs_windows8192", dict(btcs_long=2)),
                       ("btcs_partition", dict(btcs_long=1))):
        s2.set_plan(**plan)
        s2.step_btcs(u, n_btcs)
        t = PhaseTimer()
        t.mark("x")
        s2.step_btcs(u, n_btcs)
        t.mark("end")
        ms = t.spans()["x"][0]
        out[name] = {"glups": upd * n_btcs / (ms * 1e-3) / 1e9, "us_per_step": 1e3 * ms / n_btcs}
    s2.close()
    return out


# r*u; (u - u_m), (u_p - u); the two clipped products and the two subtractions; (u_p + u_m), 2u and
# their difference; D*lap and the final add.  The two clips (max, min) are not counted.
EXPLICIT_FLOPS_PER_UPDATE = 12
# binary64 instructions of the update as the kernels evaluate it, u + alpha (u_p - u) - beta (u - u_m):
# beta = max(r*u + D, D) (a fused multiply-add and a max), alpha = beta - r*u (one fused multiply-add),
# one one-sided difference (the other is the neighbour's), two fused multiply-adds.  Issue-bound ceiling
# of its flop rate = issue rate x 12 / 6, which equals the published FMA-counted binary64 vector peak.
EXPLICIT_INSTS_PER_UPDATE = 6
EXPLICIT_ALU_PEAK = FP64_ISSUE_RATE * EXPLICIT_FLOPS_PER_UPDATE / EXPLICIT_INSTS_PER_UPDATE


def profiled_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if the kernel's sources are
    unchanged since the counters were taken; else None."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                rec = json.loads(line.split(":", 1)[1])
                if rec.get("kernel") != kernel or rec.get("workload") != workload:
                    continue
                for src, digest in rec["sources"].items():
                    with open(os.path.join(ROOT, src), "rb") as g:
                        if hashlib.sha256(g.read()).hexdigest() != digest:
                            return None
                return rec["traffic_bytes_per_launch"]
    return None


def dominant_roofline(c2):
    """Roofline of the kernel that takes most of the C2 step (per-launch figures from HIP events)."""
    nodes = 4096 * 8192
    word = 8
    exp_ms, btcs_ms = c2["explicit_ms"], c2["btcs_ms"]
    if exp_ms >= btcs_ms:
        # explicit: all steps of an instance in one on-chip launch -> bound by vector ALU
        flops = EXPLICIT_FLOPS_PER_UPDATE * nodes * c2["n_exp"]
        achieved = flops / (exp_ms * 1e-3) / 1e12
        peak = EXPLICIT_ALU_PEAK / 1e12
        traffic = profiled_traffic("explicit_block_kernel<double, false, 512>", "c2_f64")
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic,
                "kernel": "explicit_block_kernel<double, false, 512>", "launches": c2["explicit_launches"],
                "algorithmic_flops_per_launch": flops / c2["explicit_launches"],
                "algorithmic_bytes_per_launch": 2 * word * nodes,
                "peak_basis": "binary64 issue 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 inst/s, "
                              "x 12 flops per 6 instructions of the update",
                "frac_of_fma_peak": achieved / (FP64_VECTOR_PEAK / 1e12)}
    per_launch = btcs_ms / c2["btcs_launches"]
    if c2["btcs_launches"] == 1:
        # resident BTCS: state on chip for all steps; the HBM traffic is one read and one write per launch
        bytes_ = 2 * word * nodes
        achieved = bytes_ * c2["n_btcs"] / (btcs_ms * 1e-3) / 1e9
        return {"bound": "alu", "achieved_equiv_GBs": achieved, "kernel": "btcs_resident_kernel<double>",
                "launches": 1, "note": "equivalent per-step HBM rate; the kernel moves the state once"}
    bytes_ = 2 * word * nodes
    achieved = bytes_ / (per_launch * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "btcs_wg_kernel<double, true>",
            "launches": c2["btcs_launches"], "algorithmic_bytes_per_launch": bytes_}


def bench_c4(B, torch, dtype, graph, batch, n_exp=1_000, n_btcs=100, plan=None, tune=False):
    """Ragged batch: 10^4 instances, N log-uniform in [64, 65536], half periodic / half Dirichlet, half
    explicit / half BTCS; explicit instances 10^3 steps at CFL 0.5, BTCS 10^2 steps at 10x, in one call.
    `plan`: knobs to force; `tune`: run the autotuner first and time its choice."""
    import workloads as W
    count = batch.count
    for i, p in enumerate(batch.problems):
        f = 1.0 if p.scheme == W.EXPLICIT else 10.0
        p.dt = f * B.burgers_cfl_dt(p, float(batch.umax[i]), 0.5)
    s = B.Solver(batch.problems, dtype=dtype)
    s.set_plan(use_graph=1 if graph else 0, **(plan or {}))
    u0 = s.pack_flat(batch.u0, batch.offsets)
    u = torch.empty_like(u0)
    u.copy_(u0)
    tuned = None
    if tune:
        tuned, tuned_ms, _ = s.autotune(u0, n_exp, n_btcs)
    s.run_mixed(u, n_exp, n_btcs)                # warm-up (plans, graph capture)
    s.sync()
    timer = PhaseTimer()
    reps = 2
    for _ in range(reps):
        u.copy_(u0)
        timer.mark("run")
        s.run_mixed(u, n_exp, n_btcs)
        timer.mark("copy")
    spans = timer.spans()
    s.close()
    ms = float(np.mean(spans["run"]))
    upd_exp = sum((p.n if p.bc == W.BC_PERIODIC else p.n - 2) for p in batch.problems if p.scheme == W.EXPLICIT)
    upd_btcs = sum((p.n if p.bc == W.BC_PERIODIC else p.n - 2) for p in batch.problems if p.scheme == W.BTCS)
    updates = upd_exp * n_exp + upd_btcs * n_btcs
    out = {"ms": ms, "glups": updates / (ms * 1e-3) / 1e9, "instances": count,
           "nodes": int(batch.offsets[-1]), "updates": int(updates), "graph": bool(graph)}
    if plan:
        out["plan"] = plan
    if tuned is not None:
        out["tuned_plan"] = tuned
        out["tuned_ms_in_autotune"] = tuned_ms
    return out


def bench_c5_adjoint(B, torch, scheme, count=256, n=16384, nsteps=2000, ckpt=100):
    """Gradient of 1/2 |u_T - target|^2 w.r.t. u0 and nu for 256 periodic instances of N=16384 (FP64),
    2000 steps, checkpoints every 100 steps: forward, checkpointed recompute and reverse sweep."""
    import workloads as W
    first, second = W.adjoint_batch(count, n, scheme=scheme)
    f = 1.0 if scheme == W.EXPLICIT else 10.0
    for i, (p, q) in enumerate(zip(first.problems, second.problems)):
        p.dt = f * B.burgers_cfl_dt(p, float(first.umax[i]), 0.5)
        q.dt = p.dt
    s = B.Solver(first.problems, dtype=torch.float64)
    u0 = s.pack_flat(first.u0, first.offsets)
    target = s.pack_flat(second.u0, second.offsets)
    s2 = B.Solver(second.problems, dtype=torch.float64)
    s2.run(target, nsteps)
    uT = u0.clone()
    s.run(uT, nsteps)
    lam = uT - target
    g = torch.zeros_like(u0)
    gn = torch.zeros(count, dtype=torch.float64, device="cuda")
    B.adjoint_into(s, u0, lam, nsteps, ckpt, g, gn)   # warm-up (buffers)
    s.sync()
    timer = PhaseTimer()
    timer.mark("adjoint")
    B.adjoint_into(s, u0, lam, nsteps, ckpt, g, gn)
    timer.mark("end")
    ms = timer.spans()["adjoint"][0]
    s.close()
    s2.close()
    return {"ms": ms, "point_steps_per_s": count * n * nsteps / (ms * 1e-3),
            "steps": nsteps, "ckpt_every": ckpt, "instances": count, "n": n}


def bench_serve(B, torch, duration=10.0, rate=2000.0, pool=800, budget=8 << 30, runs=1):
    """Poisson request stream (rate 2000/s for `duration` s) over the ragged mix (N log-uniform in
    [64, 65536], half periodic / half Dirichlet, half explicit (10^3 steps) / half BTCS (10^2 steps), half
    FP32 / half FP64), admitted by HBM budget into resident slot pools (one per precision and scheme,
    ticks of 1000 explicit / 100 BTCS steps); latency = completion - arrival.  `runs` streams are served
    in turn by the same pools (warm), each with its own arrivals."""
    import workloads as W
    from paper_2601_12204_amd.serve import GpuBackend, Request, Server
    batch, dtypes = W.ragged_batch(pool, seed=W.SEED_BASE + 4, dtype_mix=True)
    for i, p in enumerate(batch.problems):
        f = 1.0 if p.scheme == W.EXPLICIT else 10.0
        p.dt = f * B.burgers_cfl_dt(p, float(batch.umax[i]), 0.5)

    def make(k, rid):
        p = batch.problems[k]
        return Request(rid=rid, problem=p, u0=batch.instance(k), dtype="f64" if dtypes[k] else "f32",
                       nsteps=1000 if p.scheme == W.EXPLICIT else 100)

    backend = GpuBackend(slots=128, max_nodes=65536)
    warm = [make(k, k) for k in range(min(pool, 256))]
    Server(backend=backend, hbm_budget=budget).run(warm, np.linspace(0.0, 0.1, len(warm)))
    out = []
    for run in range(runs):
        arrivals = W.poisson_arrivals(rate, duration, seed=W.SEED_BASE + 40 + run)
        reqs = [make(k % pool, k) for k in range(len(arrivals))]
        srv = Server(backend=backend, hbm_budget=budget)
        stats = srv.run(reqs, arrivals)
        stats.update({"rate_per_s": rate, "duration_s": duration, "pool": pool,
                      "pooled": sum(r.path == "pool" for r in reqs)})
        out.append(stats)
    res = dict(out[0])
    if runs > 1:
        res["runs"] = [{k: o[k] for k in ("p50_ms", "p99_ms", "glups", "requests")} for o in out]
        p99 = [o["p99_ms"] for o in out]
        res["p99_spread"] = max(p99) / min(p99)
    return res


def cpu_baseline(target_s=15.0):
    """The oracle as it stands on the host cores, on a bounded sample of the same workload."""
    import oracle
    import workloads as W
    threads = oracle.max_threads()
    batch = W.c2_batch()
    sub = W.subset(batch, range(min(4096, 4 * threads)))
    for i, p in enumerate(sub.problems):
        p.dt = oracle.cfl_dt(p.n, p.length, p.nu, p.bc, float(sub.umax[i]), 0.5)
    # calibrate both legs on short runs, then size the sample (10:1 step mix) to about target_s
    t = time.perf_counter()
    oracle.run(sub.problems, sub.u0, sub.offsets, 20, scheme=W.EXPLICIT, threads=threads)
    per_exp = (time.perf_counter() - t) / 20
    for i, p in enumerate(sub.problems):
        p.dt *= 10
    t = time.perf_counter()
    oracle.run(sub.problems, sub.u0, sub.offsets, 2, scheme=W.BTCS, threads=threads)
    per_btcs = (time.perf_counter() - t) / 2
    for i, p in enumerate(sub.problems):
        p.dt /= 10
    n_exp = max(20, int(target_s / (per_exp + per_btcs / 10) / 10) * 10)

    def timed(n_exp):
        n_btcs = max(2, n_exp // 10)
        t = time.perf_counter()
        oracle.run(sub.problems, sub.u0, sub.offsets, n_exp, scheme=W.EXPLICIT, threads=threads)
        t_exp = time.perf_counter() - t
        for p in sub.problems:
            p.dt *= 10
        t = time.perf_counter()
        oracle.run(sub.problems, sub.u0, sub.offsets, n_btcs, scheme=W.BTCS, threads=threads)
        t_btcs = time.perf_counter() - t
        for p in sub.problems:
            p.dt /= 10
        return n_btcs, t_exp, t_btcs

    n_btcs, t_exp, t_btcs = timed(n_exp)
    if t_exp + t_btcs < 0.6 * target_s:        # short calibration runs overstate the per-step cost
        n_exp = int(n_exp * target_s / (t_exp + t_btcs) / 10) * 10
        n_btcs, t_exp, t_btcs = timed(n_exp)
    nodes = sub.count * 8192
    glups = nodes * (n_exp + n_btcs) / (t_exp + t_btcs) / 1e9
    # one thread on one instance, the same step mix, about a fifth of the time
    one = W.subset(sub, [0])
    n1 = max(20, int(n_exp * sub.count / threads / 5 / 10) * 10)
    t = time.perf_counter()
    oracle.run(one.problems, one.u0, one.offsets, n1, scheme=W.EXPLICIT, threads=1)
    t1_exp = time.perf_counter() - t
    for p in one.problems:
        p.dt *= 10
    t = time.perf_counter()
    oracle.run(one.problems, one.u0, one.offsets, max(2, n1 // 10), scheme=W.BTCS, threads=1)
    t1_btcs = time.perf_counter() - t
    for p in one.problems:
        p.dt /= 10
    single = 8192 * (n1 + max(2, n1 // 10)) / (t1_exp + t1_btcs) / 1e9
    return {"value": glups, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{sub.count} of the 4096 instances (N=8192, FP64), {n_exp} explicit + {n_btcs} BTCS "
                      f"steps (same 10:1 step mix as the GPU step), {t_exp + t_btcs:.1f} s",
            "explicit_glups": nodes * n_exp / t_exp / 1e9, "btcs_glups": nodes * n_btcs / t_btcs / 1e9,
            "single_thread": {"value": single, "unit": "GLUPS", "cores": 1,
                              "sample": f"1 instance, {n1} explicit + {max(2, n1 // 10)} BTCS steps, "
                                        f"{t1_exp + t1_btcs:.1f} s"},
            "cpu_model": cpu_model(), "host_threads": os.cpu_count()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--quick", action="store_true", help="skip the side measurements")
    ap.add_argument("--legs", default="c2,c2f32,c2plain,c2rk4,c2cn,c2newton,c1,c3,c4,c5,serve",
                    help="comma-separated side measurements to run (profiling runs select one; c5seg, "
                         "one 100-step checkpoint segment of the C5 gradients, only when named)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--exp-steps", type=int, default=10_000, help="explicit steps per step (profiling runs)")
    ap.add_argument("--btcs-steps", type=int, default=1_000, help="BTCS steps per step (profiling runs)")
    ap.add_argument("--explicit-path", type=int, default=0, help="force an explicit kernel path (0 auto)")
    ap.add_argument("--btcs-path", type=int, default=0, help="force a BTCS kernel path (0 auto)")
    ap.add_argument("--btcs-block", type=int, default=0, help="lanes per system of the BTCS solver (0 auto)")
    ap.add_argument("--serve-runs", type=int, default=1, help="serving streams of 10 s each")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="length of each serving stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the instances are "
              "independent, so a batch would shard across GPUs by instance without communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2601_12204_amd as B
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)

    import workloads as W
    legs = set() if args.quick else set(args.legs.split(","))
    extra = {}
    c2 = None
    if "c2" in legs or args.quick:
        log("C2 FP64")
        c2 = bench_c2(B, torch, torch.float64, args.steps, args.warmup, args.exp_steps, args.btcs_steps,
                      args.explicit_path, args.btcs_path, args.btcs_block)
        extra["c2_f64"] = c2
    if "c2f32" in legs:
        log("C2 FP32")
        extra["c2_f32"] = bench_c2(B, torch, torch.float32, 1, 1)
    if "c2plain" in legs:
        log("C2 plain steppers")
        extra["c2_plain_hbm"] = bench_c2_plain(B, torch)
    if "c2rk4" in legs:
        log("C2 RK4")
        extra["c2_rk4_f64"] = bench_c2_rk4(B, torch)
    if "c2cn" in legs:
        log("C2 Crank-Nicolson")
        extra["c2_cn_f64"] = bench_c2_cn(B, torch)
    if "c2newton" in legs:
        log("C2 Newton")
        extra["c2_newton_f64"] = bench_c2_newton(B, torch)
    if "c1" in legs:
        log("C1 latency")
        extra["c1_latency"] = bench_c1_latency(B, torch)
    if "c3" in legs:
        log("C3")
        extra["c3_f64"] = bench_c3(B, torch)
    if "c4" in legs:
        log("C4 ragged")
        c4 = W.ragged_batch(10_000)
        extra["c4_f64_graph"] = bench_c4(B, torch, torch.float64, True, c4)
        extra["c4_f64_eager"] = bench_c4(B, torch, torch.float64, False, c4)
        extra["c4_f64_graph_serial"] = bench_c4(B, torch, torch.float64, True, c4, plan={"serial": 1})
        extra["c4_f64_tuned"] = bench_c4(B, torch, torch.float64, True, c4, tune=True)
        extra["c4_f32_graph"] = bench_c4(B, torch, torch.float32, True, c4)
    if "c5" in legs:
        log("C5 adjoint")
        extra["c5_adjoint_explicit"] = bench_c5_adjoint(B, torch, W.EXPLICIT)
        extra["c5_adjoint_btcs"] = bench_c5_adjoint(B, torch, W.BTCS)
    if "c5seg" in legs:   # not a default leg: one checkpoint segment on one stream, for counter runs
        log("C5 adjoint, one segment")
        extra["c5seg_adjoint_explicit"] = bench_c5_adjoint(B, torch, W.EXPLICIT, nsteps=100, ckpt=100)
        extra["c5seg_adjoint_btcs"] = bench_c5_adjoint(B, torch, W.BTCS, nsteps=100, ckpt=100)
    if "serve" in legs:
        log("serving")
        extra["serve"] = bench_serve(B, torch, duration=args.serve_seconds, runs=args.serve_runs)
    if c2 is None:
        print(json.dumps({"metric": METRIC, "partial": True, "extra": extra}), flush=True)
        return

    roofline = dominant_roofline(c2)
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline()
    if "serve" in extra:
        line_latency = {"p50_ms": extra["serve"]["p50_ms"], "p99_ms": extra["serve"]["p99_ms"]}
    else:
        line_latency = None
    line = {
        "metric": METRIC, "value": c2["glups"], "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": c2["step_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4096 periodic instances x N=8192 on [0,2pi], nu~U[0.005,0.1], 8-mode sine "
                               "IC + 1; 1e4 explicit steps at CFL 0.5 then 1e3 BTCS steps at 10x dt",
                   "instances": 4096, "n": 8192, "explicit_steps": args.exp_steps,
                   "btcs_steps": args.btcs_steps,
                   "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "served_latency": line_latency, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
