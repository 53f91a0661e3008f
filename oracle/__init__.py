"""CPU oracle for the viscous-Burgers steppers (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this package.  The
device library never loads it and shares no code with it.  The arithmetic lives in
``burgers_oracle.cpp`` (plain loops, FP64 reference and an FP32 instantiation); this module only loads
the compiled library and marshals numpy arrays.

Functions and the passages they follow (Potluri et al., arXiv 2601.12204):
  ratios, dx        Sec. 2.2 grid, r = dt/dx, D = nu dt/dx^2
  cfl_dt            eqs. 7-8
  explicit_step     eq. 21, upwind direction by sign of u_i (text after eq. 3)
  rk4_step          eq. 22: classical RK4 over eq. 21's spatial operator
  cn_step           Crank-Nicolson (Sec. 2.2) with the BTCS lagged operator
  newton_step       fully implicit central-convection step by Newton-Raphson (eqs. 10-14)
  btcs_assemble     Sec. 2.4 / eq. 23 with the convective coefficient lagged at u^n
  thomas, cyclic    tridiagonal and cyclic (Sherman-Morrison) solves of eq. 23
  btcs_step         assemble + solve
  run               n fixed-dt steps of a packed batch, OpenMP over instances
  cole_hopf         closed-form sawtooth solution (Sec. 2.6 verification by Cole-Hopf)
  adjoint, tangent  discrete adjoint and tangent-linear sweeps of run (gradients, Sec. 2.7.1 / 2.7.3)
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.library_path()
    if not os.path.exists(path):
        _build.build()
    _lib = configure(ctypes.CDLL(path))
    return _lib


def configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    i64, c_int, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.oracle_dx.restype = dbl
    lib.oracle_dx.argtypes = [i64, dbl, c_int]
    lib.oracle_ratios.restype = None
    lib.oracle_ratios.argtypes = [i64, dbl, dbl, dbl, c_int, _dp, _dp]
    lib.oracle_cfl_dt.restype = dbl
    lib.oracle_cfl_dt.argtypes = [i64, dbl, dbl, c_int, dbl, dbl]
    for name, ptr in (("f64", _dp), ("f32", _fp)):
        for fn in ("rk4", "cn"):
            f = getattr(lib, f"oracle_{fn}_step_{name}")
            f.restype = None
            f.argtypes = [i64, c_int, dbl, dbl, dbl, dbl, ptr, ptr]
        f = getattr(lib, f"oracle_newton_step_{name}")
        f.restype = None
        f.argtypes = [i64, c_int, dbl, dbl, dbl, dbl, ptr, ptr, c_int]
        f = getattr(lib, f"oracle_explicit_step_{name}")
        f.restype = None
        f.argtypes = [i64, c_int, dbl, dbl, dbl, dbl, ptr, ptr]
        f = getattr(lib, f"oracle_btcs_step_{name}")
        f.restype = None
        f.argtypes = [i64, c_int, dbl, dbl, dbl, dbl, ptr, ptr]
        f = getattr(lib, f"oracle_run_{name}")
        f.restype = None
        f.argtypes = [i64, _i64p, _i32p, _i32p, _dp, _dp, _dp, _dp, ptr, i64, c_int]
    lib.oracle_newton_iters.restype = c_int
    lib.oracle_newton_iters.argtypes = []
    lib.oracle_btcs_assemble_f64.restype = i64
    lib.oracle_btcs_assemble_f64.argtypes = [i64, c_int, dbl, dbl, dbl, dbl, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_thomas_f64.restype = None
    lib.oracle_thomas_f64.argtypes = [i64, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_cyclic_f64.restype = None
    lib.oracle_cyclic_f64.argtypes = [i64, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_run_explicit_large_f64.restype = None
    lib.oracle_run_explicit_large_f64.argtypes = [i64, c_int, dbl, dbl, dbl, dbl, _dp, i64, c_int]
    lib.oracle_cole_hopf.restype = None
    lib.oracle_cole_hopf.argtypes = [i64, _dp, dbl, dbl, _dp]
    lib.oracle_max_threads.restype = c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_adjoint_run.restype = None
    lib.oracle_adjoint_run.argtypes = [i64, _i64p, _i32p, _i32p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, i64,
                                       _dp, _dp, c_int]
    lib.oracle_tangent_run.restype = None
    lib.oracle_tangent_run.argtypes = [i64, _i64p, _i32p, _i32p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                       i64, _dp, c_int]
    return lib


def _ptr(a: np.ndarray):
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.float32:
        return a.ctypes.data_as(_fp)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_i64p)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_i32p)
    raise TypeError(a.dtype)


def _tag(dtype) -> str:
    return "f64" if np.dtype(dtype) == np.float64 else "f32"


def max_threads() -> int:
    return int(_load().oracle_max_threads())


# ------------------------------------------------------------------------------------------------ H1
def dx(n: int, length: float, bc: int) -> float:
    return float(_load().oracle_dx(n, length, bc))


def ratios(p) -> tuple:
    """(r, D) = (dt/dx, nu dt/dx^2) in FP64 for a problem-like object."""
    r = ctypes.c_double()
    D = ctypes.c_double()
    _load().oracle_ratios(p.n, p.length, p.nu, p.dt, p.bc, ctypes.byref(r), ctypes.byref(D))
    return r.value, D.value


def cfl_dt(n: int, length: float, nu: float, bc: int, umax: float, sigma: float = 0.5) -> float:
    return float(_load().oracle_cfl_dt(n, length, nu, bc, umax, sigma))


# ------------------------------------------------------------------------------------------ steppers
def rk4_step(p, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u)
    out = np.empty_like(u)
    r, D = ratios(p)
    getattr(_load(), f"oracle_rk4_step_{_tag(u.dtype)}")(p.n, p.bc, p.left, p.right, r, D, _ptr(u), _ptr(out))
    return out


def newton_step(p, u: np.ndarray, iters: Optional[int] = None) -> np.ndarray:
    u = np.ascontiguousarray(u)
    out = np.empty_like(u)
    r, D = ratios(p)
    it = _load().oracle_newton_iters() if iters is None else iters
    getattr(_load(), f"oracle_newton_step_{_tag(u.dtype)}")(p.n, p.bc, p.left, p.right, r, D, _ptr(u), _ptr(out),
                                                          it)
    return out


def newton_iters() -> int:
    return _load().oracle_newton_iters()


def cn_step(p, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u)
    out = np.empty_like(u)
    r, D = ratios(p)
    getattr(_load(), f"oracle_cn_step_{_tag(u.dtype)}")(p.n, p.bc, p.left, p.right, r, D, _ptr(u), _ptr(out))
    return out


def explicit_step(p, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u)
    out = np.empty_like(u)
    r, D = ratios(p)
    getattr(_load(), f"oracle_explicit_step_{_tag(u.dtype)}")(p.n, p.bc, p.left, p.right, r, D,
                                                               _ptr(u), _ptr(out))
    return out


def btcs_step(p, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u)
    out = np.empty_like(u)
    r, D = ratios(p)
    getattr(_load(), f"oracle_btcs_step_{_tag(u.dtype)}")(p.n, p.bc, p.left, p.right, r, D,
                                                           _ptr(u), _ptr(out))
    return out


def btcs_assemble(p, u: np.ndarray):
    """Tridiagonal rows (l, d, p, rhs) of the BTCS step from state u (FP64)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    bufs = [np.zeros(p.n) for _ in range(4)]
    r, D = ratios(p)
    m = _load().oracle_btcs_assemble_f64(p.n, p.bc, p.left, p.right, r, D, _ptr(u),
                                         *[_ptr(b) for b in bufs])
    return tuple(b[:m].copy() for b in bufs)


def thomas(l, d, p, rhs) -> np.ndarray:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (l, d, p, rhs)]
    x = np.zeros(len(arrs[1]))
    _load().oracle_thomas_f64(len(x), *[_ptr(a) for a in arrs], _ptr(x))
    return x


def cyclic(l, d, p, rhs) -> np.ndarray:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (l, d, p, rhs)]
    x = np.zeros(len(arrs[1]))
    _load().oracle_cyclic_f64(len(x), *[_ptr(a) for a in arrs], _ptr(x))
    return x


def run(problems: Sequence, u: np.ndarray, offsets: np.ndarray, nsteps: int,
        scheme: Optional[int] = None, threads: int = 0) -> np.ndarray:
    """Advance a packed batch nsteps; scheme None takes each problem's own scheme.

    The dtype of u (float64 or float32) selects the instantiation; the result is a new array.
    """
    out = np.array(u, copy=True, order="C")
    count = len(problems)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    bc = np.array([q.bc for q in problems], dtype=np.int32)
    sch = np.array([q.scheme if scheme is None else scheme for q in problems], dtype=np.int32)
    rd = np.array([ratios(q) for q in problems], dtype=np.float64).reshape(count, 2)
    r = np.ascontiguousarray(rd[:, 0])
    D = np.ascontiguousarray(rd[:, 1])
    a = np.array([q.left for q in problems], dtype=np.float64)
    b = np.array([q.right for q in problems], dtype=np.float64)
    getattr(_load(), f"oracle_run_{_tag(out.dtype)}")(count, _ptr(offs), _ptr(bc), _ptr(sch), _ptr(r),
                                                      _ptr(D), _ptr(a), _ptr(b), _ptr(out), nsteps,
                                                      threads)
    return out


def run_explicit_large(p, u: np.ndarray, nsteps: int, threads: int = 0) -> np.ndarray:
    """Explicit steps of one large FP64 instance with nodes split across threads."""
    out = np.array(u, dtype=np.float64, copy=True)
    r, D = ratios(p)
    _load().oracle_run_explicit_large_f64(p.n, p.bc, p.left, p.right, r, D, _ptr(out), nsteps, threads)
    return out


# ------------------------------------------------------------------------------------ verification
def cole_hopf(x: np.ndarray, t: float, nu: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    _load().oracle_cole_hopf(len(x), _ptr(x), t, nu, _ptr(out))
    return out


def rel_max_abs(a: np.ndarray, ref: np.ndarray) -> float:
    """max |a - ref| / max |ref|: the parity metric."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = float(np.max(np.abs(ref))) if ref.size else 1.0
    return float(np.max(np.abs(a - ref))) / (scale if scale > 0 else 1.0) if ref.size else 0.0


def rms(a: np.ndarray, ref: np.ndarray) -> float:
    """Root-mean-square error, the paper's L2 norm (Nomenclature)."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.mean(d * d)))


def run_ratios(u: np.ndarray, bc: int, a: float, b: float, r: float, D: float, nsteps: int,
               scheme: int = 0) -> np.ndarray:
    """Advance one instance with given r and D (used to follow the dependency cone of a few nodes of a
    long grid: a window of half-width k + 1 around a node, with its ends held, reproduces that node after
    k explicit steps)."""
    out = np.array(u, copy=True, order="C")
    offs = np.array([0, len(out)], dtype=np.int64)
    one = lambda v, t: np.array([v], dtype=t)
    getattr(_load(), f"oracle_run_{_tag(out.dtype)}")(1, _ptr(offs), _ptr(one(bc, np.int32)),
                                                      _ptr(one(scheme, np.int32)), _ptr(one(r, np.float64)),
                                                      _ptr(one(D, np.float64)), _ptr(one(a, np.float64)),
                                                      _ptr(one(b, np.float64)), _ptr(out), nsteps, 1)
    return out


def _scalars(problems, scheme):
    count = len(problems)
    bc = np.array([q.bc for q in problems], dtype=np.int32)
    sch = np.array([q.scheme if scheme is None else scheme for q in problems], dtype=np.int32)
    rd = np.array([ratios(q) for q in problems], dtype=np.float64).reshape(count, 2)
    r = np.ascontiguousarray(rd[:, 0])
    D = np.ascontiguousarray(rd[:, 1])
    a = np.array([q.left for q in problems], dtype=np.float64)
    b = np.array([q.right for q in problems], dtype=np.float64)
    dtdx2 = np.array([q.dt / dx(q.n, q.length, q.bc) ** 2 for q in problems], dtype=np.float64)
    return bc, sch, r, D, a, b, dtdx2


def adjoint(problems: Sequence, u0: np.ndarray, offsets: np.ndarray, lam_T: np.ndarray, nsteps: int,
            scheme: Optional[int] = None, threads: int = 0):
    """(dJ/du0, dJ/dnu) for dJ/du_T = lam_T after nsteps steps (FP64, all forward states kept)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    lam = np.ascontiguousarray(lam_T, dtype=np.float64)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    bc, sch, r, D, a, b, dtdx2 = _scalars(problems, scheme)
    g_u0 = np.zeros_like(u0)
    g_nu = np.zeros(len(problems))
    _load().oracle_adjoint_run(len(problems), _ptr(offs), _ptr(bc), _ptr(sch), _ptr(r), _ptr(D), _ptr(a),
                               _ptr(b), _ptr(dtdx2), _ptr(u0), _ptr(lam), nsteps, _ptr(g_u0), _ptr(g_nu),
                               threads)
    return g_u0, g_nu


def tangent(problems: Sequence, u0: np.ndarray, offsets: np.ndarray, du0: np.ndarray, dnu: np.ndarray,
            nsteps: int, scheme: Optional[int] = None, threads: int = 0) -> np.ndarray:
    """Directional derivative du_T of the final state for perturbations du0 and dnu (FP64)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    du0 = np.ascontiguousarray(du0, dtype=np.float64)
    dnu = np.ascontiguousarray(dnu, dtype=np.float64)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    bc, sch, r, D, a, b, dtdx2 = _scalars(problems, scheme)
    out = np.zeros_like(u0)
    _load().oracle_tangent_run(len(problems), _ptr(offs), _ptr(bc), _ptr(sch), _ptr(r), _ptr(D), _ptr(a),
                               _ptr(b), _ptr(dtdx2), _ptr(u0), _ptr(du0), _ptr(dnu), nsteps, _ptr(out),
                               threads)
    return out
