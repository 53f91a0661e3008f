"""Seeded synthetic inputs for the viscous-Burgers solvers.

Test and benchmark infrastructure shared by the CPU oracle's tests and by the device path's tests and
benchmark, so that both sides receive identical arrays.  This module holds none of the solvers'
arithmetic: it draws random numbers, samples node coordinates and evaluates initial conditions.  Grid
ratios, time-step selection, stencils and tridiagonal solves are implemented separately on each side.

The paper (Sec. 2.5, eqs. 16-20) fixes the two boundary conditions (Dirichlet u(0)=a, u(L)=b and
periodic u_0 = u_N) and two initial conditions (sin(pi x) and a step); it publishes no data set, so every
workload here is synthetic, seeded, and shaped after the benchmark configurations:

  C1  one periodic instance on [0, 2pi], N=101, nu=0.07, with the sawtooth initial condition obtained by
      the Cole-Hopf transform of a two-image heat kernel (the paper verifies against Cole-Hopf, Sec. 2.6).
  C2  uniform batch: 4096 periodic instances, N=8192, nu ~ U[0.005, 0.1], initial condition
      1 + sum_{k=1..8} (g_k / k) sin(k x) with g_k ~ N(0, 1).
  C3  one Dirichlet grid, N = 2**24 on [0, 1], a=1, b=0, nu=1e-4, tanh-smoothed step (smoothed eq. 20).
  C4  ragged batch of 10**4 instances, N = round(exp(U[ln 64, ln 65536])), half periodic and half
      Dirichlet (on [0, 2pi], a = b = 1), half explicit and half BTCS, same Fourier initial conditions.
  C5  Poisson request stream (rate 2000/s) over the C4 mix, and an adjoint batch of 256 x 16384.

Node convention: N stored nodes.  Periodic nodes sit at x_i = i L / N (node N is node 0 again, eq. 18);
Dirichlet nodes at x_i = i L / (N - 1), both boundary nodes included and held at a and b.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BC_PERIODIC = 0
BC_DIRICHLET = 1
EXPLICIT = 0
BTCS = 1
RK4 = 2
CN = 3
NEWTON = 4

SEED_BASE = 12204
TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Problem:
    """One solve instance: stored nodes n, domain [0, length], viscosity nu, step dt, BC, scheme, a, b."""
    n: int
    length: float
    nu: float
    dt: float = 0.0
    bc: int = BC_PERIODIC
    scheme: int = EXPLICIT
    left: float = 0.0
    right: float = 0.0


@dataclasses.dataclass
class Batch:
    problems: List[Problem]
    u0: np.ndarray            # packed float64 initial states, instance b at [offsets[b], offsets[b+1])
    offsets: np.ndarray       # int64, len(problems) + 1
    umax: np.ndarray          # max |u0| per instance (input to the CFL time step)

    @property
    def count(self) -> int:
        return len(self.problems)

    def instance(self, b: int) -> np.ndarray:
        return self.u0[self.offsets[b]:self.offsets[b + 1]]


def node_coordinates(n: int, length: float, bc: int) -> np.ndarray:
    if bc == BC_PERIODIC:
        return np.arange(n, dtype=np.float64) * (length / n)
    return np.arange(n, dtype=np.float64) * (length / (n - 1))


def _pack(problems: List[Problem], states: List[np.ndarray]) -> Batch:
    offsets = np.zeros(len(problems) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([p.n for p in problems])
    u0 = np.concatenate(states) if states else np.zeros(0)
    umax = np.array([float(np.max(np.abs(s))) for s in states], dtype=np.float64)
    return Batch(problems, u0.astype(np.float64), offsets, umax)


# ----------------------------------------------------------------------------------------------- C1
C1_N = 101
C1_NU = 0.07
C1_T = 0.5


def sawtooth_ic(x: np.ndarray, nu: float) -> np.ndarray:
    """u0 = -2 nu phi_x / phi + 4 with phi = exp(-x^2/4nu) + exp(-(x-2pi)^2/4nu), written out directly."""
    e0 = np.exp(-x * x / (4.0 * nu))
    e1 = np.exp(-(x - TWO_PI) ** 2 / (4.0 * nu))
    phi = e0 + e1
    phi_x = -(x / (2.0 * nu)) * e0 - ((x - TWO_PI) / (2.0 * nu)) * e1
    return -2.0 * nu * phi_x / phi + 4.0


def c1_problem(scheme: int = EXPLICIT, n: int = C1_N, nu: float = C1_NU) -> Batch:
    x = node_coordinates(n, TWO_PI, BC_PERIODIC)
    p = Problem(n=n, length=TWO_PI, nu=nu, bc=BC_PERIODIC, scheme=scheme)
    return _pack([p], [sawtooth_ic(x, nu)])


# ------------------------------------------------------------------------------------ Fourier ICs
N_MODES = 8


def fourier_ic(x: np.ndarray, g: np.ndarray) -> np.ndarray:
    """1 + sum_{k=1..8} (g_k / k) sin(k x)."""
    u = np.ones_like(x)
    for k in range(1, N_MODES + 1):
        u = u + (g[k - 1] / k) * np.sin(k * x)
    return u


def c2_batch(count: int = 4096, n: int = 8192, scheme: int = EXPLICIT,
             seed: int = SEED_BASE + 1) -> Batch:
    """Uniform periodic batch on [0, 2pi]; draw order: nu[count], then g[count, 8]."""
    rng = np.random.default_rng(seed)
    nus = rng.uniform(0.005, 0.1, size=count)
    g = rng.standard_normal(size=(count, N_MODES))
    x = node_coordinates(n, TWO_PI, BC_PERIODIC)
    sines = np.stack([np.sin(k * x) for k in range(1, N_MODES + 1)])        # [8, n]
    coef = g / np.arange(1, N_MODES + 1)[None, :]                              # [count, 8]
    u0 = 1.0 + coef @ sines                                                    # [count, n]
    problems = [Problem(n=n, length=TWO_PI, nu=float(nus[b]), bc=BC_PERIODIC, scheme=scheme)
                for b in range(count)]
    offsets = np.arange(count + 1, dtype=np.int64) * n
    umax = np.max(np.abs(u0), axis=1)
    return Batch(problems, np.ascontiguousarray(u0.reshape(-1)), offsets, umax)


# ---------------------------------------------------------------------------------------------- C3
C3_N = 1 << 24
C3_NU = 1e-4


def tanh_step_ic(x: np.ndarray) -> np.ndarray:
    return 0.5 * (1.0 - np.tanh((x - 0.3) / 0.01))


def c3_problem(n: int = C3_N, scheme: int = EXPLICIT) -> Batch:
    x = node_coordinates(n, 1.0, BC_DIRICHLET)
    u0 = tanh_step_ic(x)
    u0[0] = 1.0
    u0[-1] = 0.0
    p = Problem(n=n, length=1.0, nu=C3_NU, bc=BC_DIRICHLET, scheme=scheme, left=1.0, right=0.0)
    return _pack([p], [u0])


def step_ic(x: np.ndarray, length: float) -> np.ndarray:
    """Eq. 20: 1 for x < L/2, else 0."""
    return np.where(x < 0.5 * length, 1.0, 0.0)


# ---------------------------------------------------------------------------------------------- C4
def ragged_batch(count: int = 10_000, n_min: int = 64, n_max: int = 65536,
                 seed: int = SEED_BASE + 3, dtype_mix: bool = False):
    """Ragged mix; draw order: nu[count], g[count, 8], then N, BC, scheme (and dtype when asked).

    Dirichlet instances live on [0, 2pi] with a = b = 1, which the Fourier initial condition meets
    exactly at both ends (the sines are set to zero there rather than evaluated at 2 pi k).
    """
    rng = np.random.default_rng(seed)
    nus = rng.uniform(0.005, 0.1, size=count)
    g = rng.standard_normal(size=(count, N_MODES))
    ns = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=count))).astype(np.int64)
    bcs = rng.integers(0, 2, size=count)
    schemes = rng.integers(0, 2, size=count)
    dtypes = rng.integers(0, 2, size=count) if dtype_mix else None
    problems, states = [], []
    for b in range(count):
        n = int(ns[b])
        bc = int(bcs[b])
        x = node_coordinates(n, TWO_PI, bc)
        u = fourier_ic(x, g[b])
        if bc == BC_DIRICHLET:
            u[0] = 1.0
            u[-1] = 1.0
        problems.append(Problem(n=n, length=TWO_PI, nu=float(nus[b]), bc=bc, scheme=int(schemes[b]),
                                left=1.0 if bc == BC_DIRICHLET else 0.0,
                                right=1.0 if bc == BC_DIRICHLET else 0.0))
        states.append(u)
    batch = _pack(problems, states)
    if dtype_mix:
        return batch, dtypes
    return batch


def subset(batch: Batch, idx) -> Batch:
    idx = list(idx)
    return _pack([dataclasses.replace(batch.problems[i]) for i in idx], [batch.instance(i).copy() for i in idx])


# ---------------------------------------------------------------------------------------------- C5
def poisson_arrivals(rate: float = 2000.0, duration: float = 10.0, seed: int = SEED_BASE + 4) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential inter-arrival gaps with mean 1/rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.5) + 64)
    t = np.cumsum(gaps)
    return t[t < duration]


def adjoint_batch(count: int = 256, n: int = 16384, scheme: int = EXPLICIT, seed: int = SEED_BASE + 4):
    """Initial states and targets for the gradient workload: targets come from a second draw (seed+1)."""
    first = c2_batch(count=count, n=n, scheme=scheme, seed=seed)
    second = c2_batch(count=count, n=n, scheme=scheme, seed=seed + 1)
    for p, q in zip(first.problems, second.problems):
        q.nu = p.nu
    return first, second


# ------------------------------------------------------------------------------------ small cases
def random_batch(seed: int, count: int, n_lo: int, n_hi: int, bc: Optional[int] = None,
                 scheme: Optional[int] = None, amplitude: float = 1.0, length: float = TWO_PI,
                 nu_lo: float = 0.005, nu_hi: float = 0.1) -> Batch:
    """Small seeded ragged batches for parity tests (mixed sign initial states when amplitude > 1)."""
    rng = np.random.default_rng(seed)
    problems, states = [], []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        b = int(rng.integers(0, 2)) if bc is None else bc
        s = int(rng.integers(0, 2)) if scheme is None else scheme
        nu = float(rng.uniform(nu_lo, nu_hi))
        g = rng.standard_normal(N_MODES) * amplitude
        x = node_coordinates(n, length, b)
        u = fourier_ic(x * (TWO_PI / length), g)
        left = right = 0.0
        if b == BC_DIRICHLET:
            left, right = float(rng.uniform(-1, 2)), float(rng.uniform(-1, 2))
            u[0], u[-1] = left, right
        problems.append(Problem(n=n, length=length, nu=nu, bc=b, scheme=s, left=left, right=right))
        states.append(u)
    return _pack(problems, states)
