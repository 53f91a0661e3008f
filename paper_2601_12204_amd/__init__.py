"""Python binding of libburgers.so, the gfx950 viscous-Burgers steppers (explicit FE and BTCS).

Argument marshalling only: every step of the solvers runs in the library's HIP kernels.  PyTorch supplies
device memory (tensors) and the HIP stream.  The functions keep the C names of include/burgers.h;
``Solver`` wraps a context for convenience.  There is no fallback: if the library is missing or cannot
be loaded, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

from .build import library_path

BC_PERIODIC = 0
BC_DIRICHLET = 1
EXPLICIT = 0
BTCS = 1
RK4 = 2
CN = 3
NEWTON = 4
F32 = 0
F64 = 1
ALIGN = 64

STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported request", -3: "out of device memory",
          -4: "device error", -5: "non-finite value", -6: "memory budget exceeded",
          -7: "Newton step not converged or Jacobian not diagonally dominant",
          -8: "truncated-window step outside its accuracy bound"}


class BurgersError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, 'unknown')} ({status})")
        self.status = status


class CProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("length", ctypes.c_double), ("nu", ctypes.c_double),
                ("dt", ctypes.c_double), ("bc", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("left", ctypes.c_double), ("right", ctypes.c_double)]


class CPlan(ctypes.Structure):
    _fields_ = [("explicit_path", ctypes.c_int32), ("tblock_depth", ctypes.c_int32),
                ("btcs_path", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("btcs_block", ctypes.c_int32), ("btcs_long", ctypes.c_int32), ("serial", ctypes.c_int32),
                ("btcs_pipeline", ctypes.c_int32)]


_lib = None
EXPORTS = ["burgers_create", "burgers_destroy", "burgers_offsets", "burgers_state_elems",
           "burgers_step_explicit", "burgers_step_btcs", "burgers_run", "burgers_run_mixed",
           "burgers_adjoint", "burgers_sync",
           "burgers_get_plan", "burgers_set_plan", "burgers_status_string", "burgers_cfl_dt",
           "burgers_ratios", "burgers_abi_version", "burgers_autotune", "burgers_run_static",
           "burgers_pool_create", "burgers_pool_destroy", "burgers_pool_admit", "burgers_pool_tick",
           "burgers_pool_busy", "burgers_pool_remaining", "burgers_pool_retire"]

# workspace of burgers_run_static (BURGERS_STATIC_SCRATCH_BYTES in include/burgers.h)
STATIC_SCRATCH_BYTES = 64 << 20


def load() -> ctypes.CDLL:
    """Load libburgers.so (built in-tree by build.py).  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"libburgers.so not built ({path}); run paper_2601_12204_amd/build.py")
    # One HIP runtime per process: torch's bundled runtime must be loaded first so that libburgers.so
    # (which needs libamdhip64.so.7) binds to it by soname instead of loading a second copy whose
    # streams and allocations torch's would not recognise.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    lib.burgers_create.argtypes = [P(CProblem), i64, ctypes.c_int, vp, P(vp)]
    lib.burgers_create.restype = ctypes.c_int
    lib.burgers_destroy.argtypes = [vp]
    lib.burgers_destroy.restype = None
    lib.burgers_offsets.argtypes = [vp, P(i64)]
    lib.burgers_offsets.restype = ctypes.c_int
    lib.burgers_state_elems.argtypes = [vp]
    lib.burgers_state_elems.restype = i64
    for name in ("burgers_step_explicit", "burgers_step_btcs", "burgers_run"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i64]
        f.restype = ctypes.c_int
    lib.burgers_run_mixed.argtypes = [vp, vp, i64, i64]
    lib.burgers_run_mixed.restype = ctypes.c_int
    lib.burgers_adjoint.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    lib.burgers_adjoint.restype = ctypes.c_int
    lib.burgers_sync.argtypes = [vp]
    lib.burgers_sync.restype = ctypes.c_int
    lib.burgers_get_plan.argtypes = [vp, P(CPlan)]
    lib.burgers_get_plan.restype = ctypes.c_int
    lib.burgers_set_plan.argtypes = [vp, P(CPlan)]
    lib.burgers_set_plan.restype = ctypes.c_int
    lib.burgers_status_string.argtypes = [ctypes.c_int]
    lib.burgers_status_string.restype = ctypes.c_char_p
    lib.burgers_cfl_dt.argtypes = [P(CProblem), dbl, dbl]
    lib.burgers_cfl_dt.restype = dbl
    lib.burgers_ratios.argtypes = [P(CProblem), P(dbl), P(dbl)]
    lib.burgers_ratios.restype = ctypes.c_int
    lib.burgers_autotune.argtypes = [vp, vp, i64, i64, P(CPlan), P(dbl)]
    lib.burgers_autotune.restype = ctypes.c_int
    lib.burgers_run_static.argtypes = [P(CProblem), i64, ctypes.c_int, vp, vp, i64]
    lib.burgers_run_static.restype = ctypes.c_int
    lib.burgers_pool_create.argtypes = [ctypes.c_int, i32, i64, i64, i64, vp, P(vp)]
    lib.burgers_pool_create.restype = ctypes.c_int
    lib.burgers_pool_destroy.argtypes = [vp]
    lib.burgers_pool_destroy.restype = None
    lib.burgers_pool_admit.argtypes = [vp, P(CProblem), vp, i64, P(i64)]
    lib.burgers_pool_admit.restype = ctypes.c_int
    lib.burgers_pool_tick.argtypes = [vp]
    lib.burgers_pool_tick.restype = ctypes.c_int
    lib.burgers_pool_busy.argtypes = [vp]
    lib.burgers_pool_busy.restype = i32
    lib.burgers_pool_remaining.argtypes = [vp, i64]
    lib.burgers_pool_remaining.restype = i64
    lib.burgers_pool_retire.argtypes = [vp, i64, vp]
    lib.burgers_pool_retire.restype = ctypes.c_int
    lib.burgers_abi_version.argtypes = []
    lib.burgers_abi_version.restype = i32
    _lib = lib
    return lib


def _check(status: int, where: str) -> None:
    if status != 0:
        raise BurgersError(status, where)


def to_cproblem(p) -> CProblem:
    return CProblem(int(p.n), float(p.length), float(p.nu), float(p.dt), int(p.bc), int(p.scheme),
                    float(getattr(p, "left", 0.0)), float(getattr(p, "right", 0.0)))


# ---------------------------------------------------------------------------------- C-named calls
def burgers_cfl_dt(p, umax: float, sigma: float = 0.5) -> float:
    return float(load().burgers_cfl_dt(ctypes.byref(to_cproblem(p)), float(umax), float(sigma)))


def burgers_ratios(p):
    r, D = ctypes.c_double(), ctypes.c_double()
    _check(load().burgers_ratios(ctypes.byref(to_cproblem(p)), ctypes.byref(r), ctypes.byref(D)),
           "burgers_ratios")
    return r.value, D.value


def burgers_autotune(ctx, u, explicit_steps: int, btcs_steps: int):
    """Time candidate plans on a scratch copy of u; the context keeps the fastest. Returns (plan, ms)."""
    plan = CPlan()
    ms = ctypes.c_double()
    _check(load().burgers_autotune(ctx, _ptr(u), int(explicit_steps), int(btcs_steps), ctypes.byref(plan),
                                   ctypes.byref(ms)), "burgers_autotune")
    return ({"explicit_path": plan.explicit_path, "tblock_depth": plan.tblock_depth, "btcs_path": plan.btcs_path,
             "use_graph": plan.use_graph, "btcs_block": plan.btcs_block, "btcs_long": plan.btcs_long,
             "serial": plan.serial, "btcs_pipeline": plan.btcs_pipeline}, ms.value)


def burgers_status_string(status: int) -> str:
    return load().burgers_status_string(int(status)).decode()


def burgers_abi_version() -> int:
    return int(load().burgers_abi_version())


def _dtype_code(dtype) -> int:
    import torch
    if dtype in (torch.float64, np.float64, "f64", F64):
        return F64
    if dtype in (torch.float32, np.float32, "f32", F32):
        return F32
    raise ValueError(f"unsupported dtype {dtype}")


def burgers_create(problems: Sequence, dtype=F64, stream=None) -> ctypes.c_void_p:
    arr = (CProblem * len(problems))(*[to_cproblem(p) for p in problems])
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    handle = ctypes.c_void_p()
    _check(load().burgers_create(arr, len(problems), _dtype_code(dtype), ctypes.c_void_p(stream),
                                 ctypes.byref(handle)), "burgers_create")
    return handle


def burgers_destroy(ctx) -> None:
    load().burgers_destroy(ctx)


def burgers_offsets(ctx, count: int) -> np.ndarray:
    out = np.zeros(count + 1, dtype=np.int64)
    _check(load().burgers_offsets(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "burgers_offsets")
    return out


def burgers_state_elems(ctx) -> int:
    return int(load().burgers_state_elems(ctx))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def burgers_step_explicit(ctx, u, nsteps: int) -> None:
    _check(load().burgers_step_explicit(ctx, _ptr(u), int(nsteps)), "burgers_step_explicit")


def burgers_step_btcs(ctx, u, nsteps: int) -> None:
    _check(load().burgers_step_btcs(ctx, _ptr(u), int(nsteps)), "burgers_step_btcs")


def burgers_run(ctx, u, nsteps: int) -> None:
    _check(load().burgers_run(ctx, _ptr(u), int(nsteps)), "burgers_run")


def burgers_run_mixed(ctx, u, explicit_steps: int, btcs_steps: int) -> None:
    _check(load().burgers_run_mixed(ctx, _ptr(u), int(explicit_steps), int(btcs_steps)), "burgers_run_mixed")


def burgers_adjoint(ctx, u0, lambda_T, nsteps: int, ckpt_every: int, grad_u0, grad_nu) -> None:
    _check(load().burgers_adjoint(ctx, _ptr(u0), _ptr(lambda_T), int(nsteps), int(ckpt_every),
                                  _ptr(grad_u0), _ptr(grad_nu)), "burgers_adjoint")


def burgers_run_static(problems: Sequence, u, nsteps: int, dtype=None, stream=None) -> None:
    """burgers_run over a batch without a context; allocates no device memory (the library's static
    scratch holds the workspace).  u: device tensor in the packed layout (``packed_offsets``)."""
    import torch
    arr = (CProblem * len(problems))(*[to_cproblem(p) for p in problems])
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    code = _dtype_code(u.dtype if dtype is None else dtype)
    want = torch.float64 if code == F64 else torch.float32
    need = int(packed_offsets(problems)[-1])
    if not (u.is_cuda and u.dtype == want and u.is_contiguous() and u.numel() >= need):
        raise ValueError(f"state must be a contiguous device tensor of {want} with >= {need} elements")
    _check(load().burgers_run_static(arr, len(problems), code, ctypes.c_void_p(stream), _ptr(u), int(nsteps)),
           "burgers_run_static")


class Pool:
    """A resident slot pool (burgers_pool_*): `slots` device slots of one precision and scheme for problems
    of up to max_nodes nodes, advanced tick by tick.  States cross through caller-owned buffers (host
    arrays or device tensors) whose addresses the library reads or writes on the pool's stream."""

    def __init__(self, dtype, scheme: int, slots: int, max_nodes: int, tick_steps: int, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.code = _dtype_code(dtype)
        self.word = 8 if self.code == F64 else 4
        self.scheme = int(scheme)
        self.slots = int(slots)
        self.handle = ctypes.c_void_p()
        _check(load().burgers_pool_create(self.code, self.scheme, self.slots, int(max_nodes), int(tick_steps),
                                          ctypes.c_void_p(stream), ctypes.byref(self.handle)), "burgers_pool_create")

    def admit(self, problem, u0_ptr: int, nsteps: int, slot: int = -1) -> int:
        """Place a problem whose initial state is at address u0_ptr into `slot` (-1: the lowest free one);
        returns the slot used, or -1 if it (or every slot) is taken."""
        slot = ctypes.c_int64(int(slot))
        st = load().burgers_pool_admit(self.handle, ctypes.byref(to_cproblem(problem)), ctypes.c_void_p(u0_ptr),
                                       int(nsteps), ctypes.byref(slot))
        if st == -6:
            return -1
        _check(st, "burgers_pool_admit")
        return int(slot.value)

    def tick(self) -> None:
        _check(load().burgers_pool_tick(self.handle), "burgers_pool_tick")

    def busy(self) -> bool:
        return bool(load().burgers_pool_busy(self.handle))

    def remaining(self, slot: int) -> int:
        return int(load().burgers_pool_remaining(self.handle, int(slot)))

    def retire(self, slot: int, dst_ptr: int) -> int:
        """Copy a finished slot's state to address dst_ptr (enqueued) and free the slot.  Returns 0, or -8
        when a truncated-window step of the slot failed its accuracy bound."""
        st = load().burgers_pool_retire(self.handle, int(slot), ctypes.c_void_p(dst_ptr))
        if st == -8:
            return st
        _check(st, "burgers_pool_retire")
        return 0

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().burgers_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def packed_offsets(problems: Sequence) -> np.ndarray:
    """The packed layout's count+1 offsets (instance starts aligned to ALIGN elements), as
    burgers_offsets gives them for a context over the same problems."""
    n = np.array([int(p.n) for p in problems], dtype=np.int64)
    off = np.zeros(len(n) + 1, dtype=np.int64)
    off[1:] = np.cumsum((n + ALIGN - 1) // ALIGN * ALIGN)
    return off


def burgers_sync(ctx) -> None:
    _check(load().burgers_sync(ctx), "burgers_sync")


def burgers_get_plan(ctx) -> dict:
    plan = CPlan()
    _check(load().burgers_get_plan(ctx, ctypes.byref(plan)), "burgers_get_plan")
    return {"explicit_path": plan.explicit_path, "tblock_depth": plan.tblock_depth,
            "btcs_path": plan.btcs_path, "use_graph": plan.use_graph, "btcs_block": plan.btcs_block,
            "btcs_long": plan.btcs_long, "serial": plan.serial, "btcs_pipeline": plan.btcs_pipeline}


def burgers_set_plan(ctx, explicit_path=0, tblock_depth=0, btcs_path=0, use_graph=-1, btcs_block=0,
                     btcs_long=0, serial=0, btcs_pipeline=0) -> None:
    plan = CPlan(int(explicit_path), int(tblock_depth), int(btcs_path), int(use_graph), int(btcs_block),
                 int(btcs_long), int(serial), int(btcs_pipeline))
    _check(load().burgers_set_plan(ctx, ctypes.byref(plan)), "burgers_set_plan")


# ---------------------------------------------------------------------------------- convenience
class Solver:
    """A context over a batch of problems, with packing helpers for torch device tensors."""

    def __init__(self, problems: Sequence, dtype=None, stream=None):
        import torch
        self.torch_dtype = torch.float64 if dtype is None else dtype
        if _dtype_code(self.torch_dtype) == F64:
            self.torch_dtype = torch.float64
        else:
            self.torch_dtype = torch.float32
        self.problems = list(problems)
        self.count = len(self.problems)
        self.ctx = burgers_create(self.problems, self.torch_dtype, stream)
        self.offsets = burgers_offsets(self.ctx, self.count)
        self.elems = burgers_state_elems(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            burgers_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # layout --------------------------------------------------------------------------------------
    def empty(self):
        import torch
        return torch.zeros(self.elems, dtype=self.torch_dtype, device="cuda")

    def pack(self, states: Iterable[np.ndarray]):
        """Host arrays (one per instance) -> device tensor in the library's packed layout."""
        import torch
        host = np.zeros(self.elems, dtype=np.float64 if self.torch_dtype == torch.float64 else np.float32)
        for b, s in enumerate(states):
            host[self.offsets[b]:self.offsets[b] + len(s)] = s
        return torch.from_numpy(host).to("cuda")

    def pack_flat(self, u: np.ndarray, offsets: np.ndarray):
        """Re-pack a dense concatenation (instance b at offsets[b]..offsets[b+1]) into the layout."""
        return self.pack([u[offsets[b]:offsets[b + 1]] for b in range(self.count)])

    def unpack(self, u) -> List[np.ndarray]:
        host = u.detach().cpu().numpy()
        return [host[self.offsets[b]:self.offsets[b] + int(p.n)].copy() for b, p in enumerate(self.problems)]

    def unpack_flat(self, u) -> np.ndarray:
        return np.concatenate(self.unpack(u))

    def _check_state(self, u) -> None:
        if not (u.is_cuda and u.dtype == self.torch_dtype and u.is_contiguous() and u.numel() >= self.elems):
            raise ValueError("state must be a contiguous device tensor of the context dtype with "
                             f">= {self.elems} elements")

    # stepping ------------------------------------------------------------------------------------
    def step_explicit(self, u, nsteps: int) -> None:
        self._check_state(u)
        burgers_step_explicit(self.ctx, u, nsteps)

    def step_btcs(self, u, nsteps: int) -> None:
        self._check_state(u)
        burgers_step_btcs(self.ctx, u, nsteps)

    def run(self, u, nsteps: int) -> None:
        self._check_state(u)
        burgers_run(self.ctx, u, nsteps)

    def run_mixed(self, u, explicit_steps: int, btcs_steps: int) -> None:
        self._check_state(u)
        burgers_run_mixed(self.ctx, u, explicit_steps, btcs_steps)

    def sync(self) -> None:
        burgers_sync(self.ctx)

    def tuning_key(self, explicit_steps: int, btcs_steps: int) -> str:
        """Cache key of a tuned plan: the precision, the step counts and how many instances fall in each
        (size class, boundary type, scheme), size classes being powers of two of n.  Batches drawn from
        the same mix share it, so a plan tuned once serves them all."""
        import hashlib
        import json
        classes = {}
        for p in self.problems:
            c = (int(np.ceil(np.log2(max(int(p.n), 2)))), int(p.bc), int(p.scheme))
            classes[c] = classes.get(c, 0) + 1
        # counts rounded to two significant figures, so that draws of one mix agree
        hist = sorted((list(c), int(float(f"{k:.2g}"))) for c, k in classes.items())
        sig = [self.torch_dtype == __import__("torch").float64, int(explicit_steps), int(btcs_steps), hist]
        return hashlib.sha1(json.dumps(sig).encode()).hexdigest()

    def autotune(self, u, explicit_steps: int, btcs_steps: int, cache: Optional[str] = None):
        """Pick the fastest plan for this workload (burgers_autotune); with `cache`, a JSON file keyed by
        tuning_key stores and reuses the choice."""
        import json
        key = self.tuning_key(explicit_steps, btcs_steps)
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
            if key in store:
                self.set_plan(**store[key]["plan"])
                return store[key]["plan"], store[key]["ms"], True
        plan, ms = burgers_autotune(self.ctx, u, explicit_steps, btcs_steps)
        if cache:
            store[key] = {"plan": plan, "ms": ms}
            with open(cache, "w") as f:
                json.dump(store, f, indent=1)
        return plan, ms, False

    def set_plan(self, **kw) -> None:
        burgers_set_plan(self.ctx, **kw)

    def get_plan(self) -> dict:
        return burgers_get_plan(self.ctx)


def adjoint_into(solver: "Solver", u0, lam_T, nsteps: int, ckpt_every: int, grad_u0, grad_nu) -> None:
    """burgers_adjoint through a Solver (FP64 contexts): device buffers in the packed layout."""
    solver._check_state(u0)
    solver._check_state(lam_T)
    solver._check_state(grad_u0)
    if not (grad_nu.is_cuda and grad_nu.dtype == solver.torch_dtype and grad_nu.numel() >= solver.count):
        raise ValueError("grad_nu must be a device tensor of the context dtype with >= count elements")
    burgers_adjoint(solver.ctx, u0, lam_T, nsteps, ckpt_every, grad_u0, grad_nu)


class BurgersSolve:
    """torch.autograd.Function over burgers_run / burgers_adjoint.

    ``u_T = BurgersSolve.apply(u0, nu, problems, nsteps, ckpt_every)`` advances the packed FP64 state u0
    (layout of a Solver over ``problems``) nsteps steps of each instance's scheme, with the viscosities
    taken from the tensor ``nu`` (one per instance).  Backward returns dJ/du0 and dJ/dnu from the
    library's discrete adjoint, recomputing forward states from checkpoints every ckpt_every steps.
    """

    @staticmethod
    def _function():
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, u0, nu, problems, nsteps, ckpt_every):
                import dataclasses
                nus = nu.detach().cpu().double().tolist()
                probs = [dataclasses.replace(p, nu=float(v)) for p, v in zip(problems, nus)]
                solver = Solver(probs, dtype=torch.float64)
                u = u0.detach().clone()
                solver.run(u, nsteps)
                ctx.save_for_backward(u0.detach())
                ctx.solver, ctx.nsteps, ctx.ckpt, ctx.nu_dtype = solver, nsteps, ckpt_every, nu.dtype
                return u

            @staticmethod
            def backward(ctx, grad_uT):
                (u0,) = ctx.saved_tensors
                solver = ctx.solver
                grad_u0 = torch.zeros_like(u0)
                grad_nu = torch.zeros(solver.count, dtype=torch.float64, device=u0.device)
                adjoint_into(solver, u0, grad_uT.contiguous(), ctx.nsteps, ctx.ckpt, grad_u0, grad_nu)
                return grad_u0, grad_nu.to(ctx.nu_dtype), None, None, None

        return _Fn

    @staticmethod
    def apply(u0, nu, problems, nsteps: int, ckpt_every: int = 100):
        return BurgersSolve._function().apply(u0, nu, problems, nsteps, ckpt_every)
