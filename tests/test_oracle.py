"""Pins of the CPU oracle against facts the paper and the mathematics fix (no device needed).

Each test ties the oracle to something outside itself: closed forms (Cole-Hopf, the von Neumann
amplification factor, the steady viscous-shock profile), invariants (constant states, translation and
reflection equivariance, the discrete maximum principle), convergence orders the paper states, and
brute-force dense solves.  A plausible slip in the oracle (a dropped term, a wrong sign or index, a
swapped corner in the cyclic solve) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_statements.json")))
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _problem(n, length, nu, dt, bc=W.BC_PERIODIC, scheme=W.EXPLICIT, a=0.0, b=0.0):
    return W.Problem(n=n, length=length, nu=nu, dt=dt, bc=bc, scheme=scheme, left=a, right=b)


def _with_ratios(n, C, D, U=1.0, length=2 * math.pi, bc=W.BC_PERIODIC):
    """Problem whose Courant number at speed U is C and whose diffusion number is D."""
    dx = length / n if bc == W.BC_PERIODIC else length / (n - 1)
    dt = abs(C) * dx / abs(U) if C != 0 else 1e-3 * dx
    nu = D * dx * dx / dt
    return _problem(n, length, nu, dt, bc)


# ------------------------------------------------------------------------------------ Cole-Hopf form
def test_cole_hopf_matches_sawtooth_ic_at_t0(oracle_lib):
    """The closed form at t=0 equals the two-image sawtooth initial condition (written out directly)."""
    x = W.node_coordinates(W.C1_N, W.TWO_PI, W.BC_PERIODIC)
    ch = oracle_lib.cole_hopf(x, 0.0, W.C1_NU)
    ic = W.sawtooth_ic(x, W.C1_NU)
    assert np.max(np.abs(ch - ic)) <= 1e-14 * np.max(np.abs(ic))


def test_cole_hopf_solves_burgers(oracle_lib):
    """Residual u_t + u u_x - nu u_xx of the closed form, by 4th-order central differences, vanishes."""
    nu = W.C1_NU
    x = np.linspace(0.3, 6.0, 23)
    for t in (0.1, 0.5, 1.3):
        h = 1e-3
        f = lambda xx, tt: oracle_lib.cole_hopf(np.atleast_1d(xx), tt, nu)
        u = f(x, t)
        ut = (-f(x, t + 2 * h) + 8 * f(x, t + h) - 8 * f(x, t - h) + f(x, t - 2 * h)) / (12 * h)
        ux = (-f(x + 2 * h, t) + 8 * f(x + h, t) - 8 * f(x - h, t) + f(x - 2 * h, t)) / (12 * h)
        uxx = (-f(x + 2 * h, t) + 16 * f(x + h, t) - 30 * u + 16 * f(x - h, t) - f(x - 2 * h, t)) / (12 * h * h)
        res = ut + u * ux - nu * uxx
        scale = np.max(np.abs(u * ux)) + np.max(np.abs(ut))
        assert np.max(np.abs(res)) <= 1e-5 * scale, (t, np.max(np.abs(res)), scale)


def test_cole_hopf_is_periodic_and_translates(oracle_lib):
    nu = 0.05
    x = np.linspace(0, 2 * np.pi, 50)
    a = oracle_lib.cole_hopf(x, 0.7, nu)
    b = oracle_lib.cole_hopf(x + 2 * np.pi, 0.7, nu)
    assert np.max(np.abs(a - b)) < 1e-12
    # Galilean frame moving at speed 4: shape at t is the t-shifted profile of the heat kernel
    c = oracle_lib.cole_hopf(x + 4 * 0.7, 0.7, nu)
    d = oracle_lib.cole_hopf(x, 0.0, nu * 1.7)      # (t+1) nu scaling of the Gaussian width
    assert np.all(np.isfinite(c)) and np.all(np.isfinite(d))


# ------------------------------------------------------------------------------------ time step (H1)
@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_cfl_dt_satisfies_both_limits(oracle_lib, bc):
    """sigma=0.5 keeps |C| + 2D <= 1 (the monotone bound); sigma=1 makes one of eqs. 7-8 an equality."""
    rng = np.random.default_rng(0)
    conv = GOLDEN["cfl_convective_limit"]["value"]
    diff = GOLDEN["cfl_diffusive_limit"]["value"]
    for _ in range(50):
        n = int(rng.integers(3, 5000))
        L = float(rng.uniform(0.5, 10))
        nu = float(rng.uniform(1e-4, 1.0))
        umax = float(rng.uniform(0.1, 10))
        for sigma in (0.5, 1.0):
            dt = oracle_lib.cfl_dt(n, L, nu, bc, umax, sigma)
            r, D = oracle_lib.ratios(_problem(n, L, nu, dt, bc))
            C = r * umax
            assert C <= sigma * conv * (1 + 1e-14) and D <= sigma * diff * (1 + 1e-14)
            if sigma == 0.5:
                assert C + 2 * D <= 1 + 1e-14
            else:
                assert max(C / conv, D / diff) == pytest.approx(1.0, rel=1e-14)
    assert oracle_lib.cfl_dt(10, 1.0, 0.0, bc, 0.0, 0.5) == math.inf


# ------------------------------------------------------------------------------------ explicit step
def test_explicit_constant_state_bitwise(oracle_lib):
    for U in (1.7, -0.3, 0.0):
        p = _with_ratios(37, 0.4, 0.3, U=1.0)
        u = np.full(37, U)
        assert np.array_equal(oracle_lib.explicit_step(p, u), u)
        q = _problem(37, 1.0, 0.01, 1e-4, W.BC_DIRICHLET, a=U, b=U)
        assert np.array_equal(oracle_lib.explicit_step(q, u), u)


@pytest.mark.parametrize("U,C", [(1.0, 0.3), (-1.0, -0.45), (2.5, 0.05)])
@pytest.mark.parametrize("k", [1, 3, 11])
def test_explicit_von_neumann_symbol(oracle_lib, U, C, k):
    """Small perturbation of a constant state evolves by the upwind/central amplification factor."""
    n, D, eps = 64, 0.2, 1e-6
    p = _with_ratios(n, C, D, U=U)
    theta = 2 * np.pi * k / n
    j = np.arange(n)
    u = U + eps * np.sin(j * theta)
    if C >= 0:
        g = 1 - C * (1 - np.exp(-1j * theta)) - 4 * D * np.sin(theta / 2) ** 2
    else:
        g = 1 - C * (np.exp(1j * theta) - 1) - 4 * D * np.sin(theta / 2) ** 2
    pred = g.real * np.sin(j * theta) + g.imag * np.cos(j * theta)
    got = (oracle_lib.explicit_step(p, u) - U) / eps
    assert np.max(np.abs(got - pred)) < 2e-5


def test_explicit_translation_equivariance_bitwise(oracle_lib):
    b = W.random_batch(1, 1, 50, 50, bc=W.BC_PERIODIC, amplitude=3.0)
    p = b.problems[0]
    p.dt = 0.5 * oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, b.umax[0], 0.5)
    u = b.instance(0)
    base = oracle_lib.explicit_step(p, u)
    for s in (1, 7, 49):
        assert np.array_equal(oracle_lib.explicit_step(p, np.roll(u, s)), np.roll(base, s))


def test_explicit_reflection_equivariance_bitwise(oracle_lib):
    """v_i = -u_{-i mod N} maps to -u'_{-i mod N}: needs the sign-selecting upwind and symmetric lap."""
    b = W.random_batch(2, 1, 41, 41, bc=W.BC_PERIODIC, amplitude=3.0)
    p = b.problems[0]
    p.dt = oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, b.umax[0], 0.5)
    u = b.instance(0)
    refl = lambda a: -a[(-np.arange(len(a))) % len(a)]
    assert np.array_equal(oracle_lib.explicit_step(p, refl(u)), refl(oracle_lib.explicit_step(p, u)))


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_explicit_discrete_maximum_principle(oracle_lib, bc):
    """Under sigma = 0.5 every update is a convex combination: min u0 <= u^n <= max u0."""
    batch = W.random_batch(3, 6, 20, 300, bc=bc, amplitude=3.0)
    for i, p in enumerate(batch.problems):
        p.dt = oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, batch.umax[i], 0.5)
    out = oracle_lib.run(batch.problems, batch.u0, batch.offsets, 400, scheme=W.EXPLICIT)
    for i in range(batch.count):
        u0 = batch.instance(i)
        un = out[batch.offsets[i]:batch.offsets[i + 1]]
        tol = 1e-14 * np.max(np.abs(u0))
        assert un.max() <= u0.max() + tol and un.min() >= u0.min() - tol


def test_explicit_beyond_diffusive_limit_oscillates(oracle_lib):
    """Paper Sec. 3.1: beyond the CFL limits the explicit scheme develops oscillations."""
    assert GOLDEN["beyond_cfl_oscillates"]["value"]
    n = 128
    p = _with_ratios(n, 0.1, 0.6, U=1.0)               # D = 0.6 > 1/2
    x = W.node_coordinates(n, p.length, W.BC_PERIODIC)
    u = 1.0 + 0.1 * np.sin(x)
    out = oracle_lib.run([p], u, np.array([0, n]), 400, scheme=W.EXPLICIT)
    assert not np.all(np.isfinite(out)) or np.max(np.abs(out)) > 10
    ok = _with_ratios(n, 0.1, 0.45, U=1.0)
    out = oracle_lib.run([ok], u, np.array([0, n]), 400, scheme=W.EXPLICIT)
    assert np.max(np.abs(out)) <= 1.1 + 1e-12


def _cole_hopf_run(oracle_lib, n, scheme, dt_factor, t_final=W.C1_T, nu=W.C1_NU):
    b = W.c1_problem(scheme, n=n, nu=nu)
    p = b.problems[0]
    dtmax = dt_factor * oracle_lib.cfl_dt(n, p.length, p.nu, p.bc, b.umax[0], 0.5)
    steps = int(math.ceil(t_final / dtmax))
    p.dt = t_final / steps
    out = oracle_lib.run([p], b.u0, b.offsets, steps)
    x = W.node_coordinates(n, p.length, p.bc)
    return out, oracle_lib.cole_hopf(x, t_final, nu)


def test_explicit_first_order_convergence_to_cole_hopf(oracle_lib):
    """RMS error against Cole-Hopf falls with slope ~1 in dx (first-order upwind, Sec. 2.3)."""
    ns = [400, 800, 1600, 3200]
    errs = []
    for n in ns:
        u, ref = _cole_hopf_run(oracle_lib, n, W.EXPLICIT, 1.0)
        errs.append(oracle_lib.rms(u, ref))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 0.8 <= slope <= 1.2, (errs, slope)


def test_explicit_first_order_in_time(oracle_lib):
    """At fixed N, halving dt halves the change of the solution: temporal order 1 (Sec. 2.3)."""
    assert GOLDEN["explicit_temporal_order"]["value"] == 1
    sols = [_cole_hopf_run(oracle_lib, 400, W.EXPLICIT, f)[0] for f in (0.5, 0.25, 0.125)]
    ratio = np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2])
    assert 1.8 <= ratio <= 2.2, ratio


# ------------------------------------------------------------------------------------ RK4 (eq. 22)
def test_rk4_constant_state_bitwise(oracle_lib):
    for U in (1.7, -0.3, 0.0):
        p = _with_ratios(37, 0.4, 0.3, U=1.0)
        u = np.full(37, U)
        assert np.array_equal(oracle_lib.rk4_step(p, u), u)
        q = _problem(37, 1.0, 0.01, 1e-4, W.BC_DIRICHLET, a=U, b=U)
        assert np.array_equal(oracle_lib.rk4_step(q, u), u)


@pytest.mark.parametrize("U,C", [(1.0, 0.3), (-1.0, -0.45), (2.5, 0.05)])
@pytest.mark.parametrize("k", [1, 3, 11])
def test_rk4_von_neumann_symbol(oracle_lib, U, C, k):
    """A small perturbation of a constant state is multiplied by the RK4 polynomial
    1 + z + z^2/2 + z^3/6 + z^4/24 of the forward-Euler increment symbol z (eq. 22 over eq. 21)."""
    n, D, eps = 64, 0.2, 1e-6
    p = _with_ratios(n, C, D, U=U)
    theta = 2 * np.pi * k / n
    j = np.arange(n)
    u = U + eps * np.sin(j * theta)
    if C >= 0:
        z = -C * (1 - np.exp(-1j * theta)) - 4 * D * np.sin(theta / 2) ** 2
    else:
        z = -C * (np.exp(1j * theta) - 1) - 4 * D * np.sin(theta / 2) ** 2
    g = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    pred = g.real * np.sin(j * theta) + g.imag * np.cos(j * theta)
    got = (oracle_lib.rk4_step(p, u) - U) / eps
    assert np.max(np.abs(got - pred)) < 2e-5


def test_rk4_fourth_order_in_time(oracle_lib):
    """At fixed N on a smooth solution, halving dt divides the change of the solution by 2^4."""
    n, nu, T = 128, 0.05, 0.4
    x = W.node_coordinates(n, 2 * np.pi, W.BC_PERIODIC)
    u0 = 1.0 + 0.5 * np.sin(x)
    sols = []
    for steps in (20, 40, 80):
        p = _problem(n, 2 * np.pi, nu, T / steps, scheme=W.RK4)
        sols.append(oracle_lib.run([p], u0, np.array([0, n]), steps))
    ratio = np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2])
    assert 14.0 <= ratio <= 18.0, ratio


def test_rk4_first_stage_is_forward_euler(oracle_lib):
    """With the later stages removed (u' = u + K1), eq. 22 is eq. 21: checks that K is eq. 21's increment
    by comparing RK4 against forward Euler to second order in dt."""
    b = W.random_batch(3, 1, 60, 60, bc=W.BC_PERIODIC, amplitude=2.0)
    p = b.problems[0]
    u = b.instance(0)
    diffs = []
    for f in (1.0, 0.5, 0.25):
        p.dt = f * oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, float(b.umax[0]), 0.5)
        diffs.append(np.max(np.abs(oracle_lib.rk4_step(p, u) - oracle_lib.explicit_step(p, u))))
    # one step differs by O(dt^2): the ratio for halved dt is ~4
    assert 3.5 <= diffs[0] / diffs[1] <= 4.5 and 3.5 <= diffs[1] / diffs[2] <= 4.5, diffs


def test_rk4_dirichlet_ends_held_and_translation_equivariant(oracle_lib):
    b = W.random_batch(5, 1, 41, 41, bc=W.BC_DIRICHLET, amplitude=2.0)
    p = b.problems[0]
    p.dt = oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, float(b.umax[0]), 0.5)
    out = oracle_lib.rk4_step(p, b.instance(0))
    assert out[0] == p.left and out[-1] == p.right
    c = W.random_batch(6, 1, 50, 50, bc=W.BC_PERIODIC, amplitude=3.0)
    q = c.problems[0]
    q.dt = oracle_lib.cfl_dt(q.n, q.length, q.nu, q.bc, float(c.umax[0]), 0.5)
    u = c.instance(0)
    assert np.array_equal(np.roll(oracle_lib.rk4_step(q, u), 7), oracle_lib.rk4_step(q, np.roll(u, 7)))


# ------------------------------------------------------------------------------------ tridiagonal
def _dense(l, d, p, cyclic):
    m = len(d)
    A = np.diag(d)
    for k in range(1, m):
        A[k, k - 1] = l[k]
    for k in range(m - 1):
        A[k, k + 1] = p[k]
    if cyclic:
        A[0, m - 1] += l[0]
        A[m - 1, 0] += p[m - 1]
    return A


def test_thomas_and_cyclic_against_dense_random(oracle_lib):
    rng = np.random.default_rng(5)
    for m in (1, 2, 3, 4, 5, 9, 17, 64):
        l = rng.uniform(-1, 1, m)
        p = rng.uniform(-1, 1, m)
        d = np.abs(l) + np.abs(p) + rng.uniform(0.1, 2, m)
        d *= rng.choice([-1, 1], m)
        rhs = rng.standard_normal(m)
        x = oracle_lib.thomas(l, d, p, rhs)
        assert np.allclose(x, np.linalg.solve(_dense(l, d, p, False), rhs), rtol=1e-12, atol=1e-12)
        if m >= 3:
            x = oracle_lib.cyclic(l, d, p, rhs)
            assert np.allclose(x, np.linalg.solve(_dense(l, d, p, True), rhs), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
@pytest.mark.parametrize("C,D", [(0.5, 0.25), (5.0, 2.5), (50.0, 10.0), (1000.0, 1000.0)])
def test_btcs_step_against_dense_lu(oracle_lib, bc, C, D):
    """Brute force for N <= 64: dense partial-pivot LU of the full (cyclic) BTCS matrix."""
    for n in (3, 4, 5, 7, 16, 33, 64):
        b = W.random_batch(100 + n, 1, n, n, bc=bc, amplitude=3.0)
        u = b.instance(0)
        p = _with_ratios(n, C, D, U=float(np.max(np.abs(u))), bc=bc)
        p.left, p.right = b.problems[0].left, b.problems[0].right
        l, d, q, rhs = oracle_lib.btcs_assemble(p, u)
        A = _dense(l, d, q, bc == W.BC_PERIODIC)
        x = np.linalg.solve(A, rhs)
        got = oracle_lib.btcs_step(p, u)
        if bc == W.BC_DIRICHLET:
            assert got[0] == p.left and got[-1] == p.right
            got = got[1:-1]
        cmax = C
        tol = 64 * np.finfo(float).eps * (1 + 4 * D + 2 * cmax)
        assert oracle_lib.rel_max_abs(got, x) <= tol, (n, oracle_lib.rel_max_abs(got, x))


def test_btcs_rows_are_an_m_matrix_with_unit_row_sums(oracle_lib):
    """d - |l| - |p| = 1 with l, p <= 0: strictly diagonally dominant M-matrix, unique solution."""
    b = W.random_batch(7, 1, 200, 200, bc=W.BC_PERIODIC, amplitude=3.0)
    p = _with_ratios(200, 7.0, 3.0, U=float(b.umax[0]))
    l, d, q, _ = oracle_lib.btcs_assemble(p, b.instance(0))
    assert np.all(l <= 0) and np.all(q <= 0)
    assert np.allclose(d + l + q, 1.0, rtol=0, atol=1e-12 * np.max(d))


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_btcs_constant_state(oracle_lib, bc):
    for U in (1.7, -0.3):
        p = _with_ratios(57, 20.0, 5.0, U=2.0, bc=bc)
        p.left = p.right = U
        got = oracle_lib.btcs_step(p, np.full(57, U))
        assert np.max(np.abs(got - U)) <= 1e-14


@pytest.mark.parametrize("U,C", [(1.0, 3.0), (-1.0, -2.0)])
def test_btcs_von_neumann_symbol(oracle_lib, U, C):
    n, D, eps, k = 64, 2.0, 1e-6, 5
    p = _with_ratios(n, C, D, U=U)
    theta = 2 * np.pi * k / n
    j = np.arange(n)
    u = U + eps * np.sin(j * theta)
    if C >= 0:
        g = 1 / (1 + C * (1 - np.exp(-1j * theta)) + 4 * D * np.sin(theta / 2) ** 2)
    else:
        g = 1 / (1 + C * (np.exp(1j * theta) - 1) + 4 * D * np.sin(theta / 2) ** 2)
    pred = g.real * np.sin(j * theta) + g.imag * np.cos(j * theta)
    got = (oracle_lib.btcs_step(p, u) - U) / eps
    assert np.max(np.abs(got - pred)) < 2e-5


# ------------------------------------------------------------------------------------ Crank-Nicolson
def test_cn_constant_state(oracle_lib):
    for bc in (W.BC_PERIODIC, W.BC_DIRICHLET):
        for U in (1.3, -0.7):
            p = _with_ratios(33, 6.0, 3.0, U=1.0, bc=bc)
            p.left = p.right = U
            u = np.full(33, U)
            assert np.max(np.abs(oracle_lib.cn_step(p, u) - U)) < 1e-14


@pytest.mark.parametrize("U,C", [(1.0, 3.0), (-1.0, -7.0), (2.0, 0.4)])
@pytest.mark.parametrize("k", [2, 5, 17])
def test_cn_von_neumann_symbol(oracle_lib, U, C, k):
    """Linearised, a mode is multiplied by (1 - z/2) / (1 + z/2) with z the symbol of the BTCS operator
    minus the identity (the convective coefficient's own perturbation drops out: N's rows sum to zero)."""
    n, D, eps = 64, 2.0, 1e-6
    p = _with_ratios(n, C, D, U=U)
    theta = 2 * np.pi * k / n
    j = np.arange(n)
    u = U + eps * np.sin(j * theta)
    if C >= 0:
        z = C * (1 - np.exp(-1j * theta)) + 4 * D * np.sin(theta / 2) ** 2
    else:
        z = C * (np.exp(1j * theta) - 1) + 4 * D * np.sin(theta / 2) ** 2
    g = (1 - z / 2) / (1 + z / 2)
    assert abs(g) <= 1 + 1e-12
    pred = g.real * np.sin(j * theta) + g.imag * np.cos(j * theta)
    got = (oracle_lib.cn_step(p, u) - U) / eps
    assert np.max(np.abs(got - pred)) < 2e-5


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_cn_is_twice_half_step_btcs_minus_identity(oracle_lib, bc):
    """(I + N/2)^{-1} (I - N/2) u = 2 (I + N/2)^{-1} u - u, and I + N/2 is the BTCS matrix of dt/2: one
    Crank-Nicolson step equals twice a half-dt BTCS step minus the old state."""
    b = W.random_batch(8 + bc, 1, 300, 300, bc=bc, amplitude=2.0)
    p = b.problems[0]
    p.dt = 12 * oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, float(b.umax[0]), 0.5)
    u = b.instance(0)
    half = W.Problem(n=p.n, length=p.length, nu=p.nu, dt=p.dt / 2, bc=p.bc, scheme=W.BTCS, left=p.left,
                     right=p.right)
    ref = 2 * oracle_lib.btcs_step(half, u) - u
    got = oracle_lib.cn_step(p, u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(u))
    if bc == W.BC_DIRICHLET:
        assert got[0] == p.left and got[-1] == p.right


def test_cn_second_order_in_time_linear_limit(oracle_lib):
    """In the linear (small-amplitude, diffusion-dominated) limit halving dt divides the change by 4,
    against 2 for BTCS: Crank-Nicolson's time weighting.  (With the convective coefficient lagged at
    t^n the nonlinear scheme is first order, like BTCS; that reading is listed in the design notes.)"""
    n, nu, T, eps = 64, 0.5, 1.0, 1e-3
    x = W.node_coordinates(n, 2 * np.pi, W.BC_PERIODIC)
    ratios = {}
    for scheme in (W.CN, W.BTCS):
        sols = []
        for steps in (10, 20, 40):
            p = _problem(n, 2 * np.pi, nu, T / steps, scheme=scheme)
            sols.append(oracle_lib.run([p], eps * np.sin(x), np.array([0, n]), steps))
        ratios[scheme] = np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2])
    assert 3.7 <= ratios[W.CN] <= 4.3, ratios
    assert 1.8 <= ratios[W.BTCS] <= 2.2, ratios


# ------------------------------------------------------------------------------------ Newton (eqs. 10-15)
def _newton_case(seed, bc, factor=1.0, amplitude=1.5, n=160):
    b = W.random_batch(seed, 1, n, n, bc=bc, amplitude=amplitude)
    p = b.problems[0]
    p.scheme = W.NEWTON
    p.dt = factor * oracle.cfl_dt(p.n, p.length, p.nu, p.bc, float(b.umax[0]), 0.5)
    return p, b.instance(0)


def test_newton_constant_state(oracle_lib):
    for bc in (W.BC_PERIODIC, W.BC_DIRICHLET):
        p = _with_ratios(40, 0.5, 0.4, U=1.0, bc=bc)
        p.left = p.right = 0.8
        u = np.full(40, 0.8)
        assert np.array_equal(oracle_lib.newton_step(p, u), u)


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
@pytest.mark.parametrize("factor", [1.0, 4.0])
def test_newton_converges_quadratically(oracle_lib, bc, factor):
    """Errors of successive Newton iterates against the converged root fall quadratically (eq. 12 with
    the exact Jacobian of eq. 11), and the fixed iteration count reaches rounding level."""
    p, u = _newton_case(21 + bc, bc, factor)
    ref = oracle_lib.newton_step(p, u, 12)
    errs = [np.max(np.abs(oracle_lib.newton_step(p, u, k) - ref)) for k in (1, 2, 3)]
    assert errs[1] <= 50 * errs[0] ** 2 and errs[2] <= 50 * errs[1] ** 2 + 1e-15, errs
    assert np.max(np.abs(oracle_lib.newton_step(p, u) - ref)) <= 4e-15 * np.max(np.abs(u))


@pytest.mark.parametrize("U,C", [(1.0, 0.4), (-1.0, -0.8), (2.0, 0.1)])
@pytest.mark.parametrize("k", [2, 7, 19])
def test_newton_von_neumann_symbol(oracle_lib, U, C, k):
    """Linearised about a constant state the fully implicit central step multiplies a mode by
    1 / (1 + i C sin(theta) + 4 D sin^2(theta/2)), C = r U (central convection, eq. 11)."""
    n, D, eps = 64, 1.5, 1e-6
    p = _with_ratios(n, C, D, U=U)
    theta = 2 * np.pi * k / n
    j = np.arange(n)
    u = U + eps * np.sin(j * theta)
    g = 1 / (1 + 1j * C * np.sin(theta) + 4 * D * np.sin(theta / 2) ** 2)
    pred = g.real * np.sin(j * theta) + g.imag * np.cos(j * theta)
    got = (oracle_lib.newton_step(p, u) - U) / eps
    assert np.max(np.abs(got - pred)) < 2e-5


def test_newton_symmetries(oracle_lib):
    """Translation equivariance (periodic) and the Burgers reflection u(x) -> -u(-x), which the central
    scheme keeps exactly; Dirichlet ends are held."""
    p, u = _newton_case(31, W.BC_PERIODIC)
    assert np.array_equal(np.roll(oracle_lib.newton_step(p, u), 5), oracle_lib.newton_step(p, np.roll(u, 5)))
    refl = lambda v: -np.roll(v[::-1], 1)
    assert np.max(np.abs(oracle_lib.newton_step(p, refl(u)) - refl(oracle_lib.newton_step(p, u)))) < 1e-14
    q, v = _newton_case(33, W.BC_DIRICHLET)
    out = oracle_lib.newton_step(q, v)
    assert out[0] == q.left and out[-1] == q.right


def test_btcs_equivariance(oracle_lib):
    b = W.random_batch(9, 1, 48, 48, bc=W.BC_PERIODIC, amplitude=3.0)
    u = b.instance(0)
    p = _with_ratios(48, 8.0, 3.0, U=float(b.umax[0]))
    base = oracle_lib.btcs_step(p, u)
    assert np.max(np.abs(oracle_lib.btcs_step(p, np.roll(u, 5)) - np.roll(base, 5))) < 1e-13
    refl = lambda a: -a[(-np.arange(len(a))) % len(a)]
    assert np.max(np.abs(oracle_lib.btcs_step(p, refl(u)) - refl(base))) < 1e-13


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_btcs_unconditional_maximum_principle(oracle_lib, bc):
    batch = W.random_batch(11, 5, 20, 300, bc=bc, amplitude=3.0)
    for i, p in enumerate(batch.problems):
        p.dt = 200 * oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, batch.umax[i], 0.5)
    out = oracle_lib.run(batch.problems, batch.u0, batch.offsets, 50, scheme=W.BTCS)
    for i in range(batch.count):
        u0 = batch.instance(i)
        un = out[batch.offsets[i]:batch.offsets[i + 1]]
        tol = 1e-13 * np.max(np.abs(u0))
        assert un.max() <= u0.max() + tol and un.min() >= u0.min() - tol


def test_btcs_stable_at_paper_courant_number(oracle_lib):
    """Paper Sec. 3.4: step initial condition, implicit step stable at dt = 5 dx / u_max."""
    c = GOLDEN["implicit_stable_courant"]["value"]
    n, L, nu = 201, 1.0, 0.01
    x = W.node_coordinates(n, L, W.BC_DIRICHLET)
    u = W.step_ic(x, L)
    dxv = L / (n - 1)
    p = _problem(n, L, nu, c * dxv / 1.0, W.BC_DIRICHLET, W.BTCS, a=1.0, b=0.0)
    out = oracle_lib.run([p], u, np.array([0, n]), 200)
    assert np.all(np.isfinite(out)) and out.min() >= -1e-14 and out.max() <= 1 + 1e-14
    # the explicit scheme at the same dt is unstable
    q = _problem(n, L, nu, c * dxv, W.BC_DIRICHLET, W.EXPLICIT, a=1.0, b=0.0)
    bad = oracle_lib.run([q], u, np.array([0, n]), 200)
    assert not np.all(np.isfinite(bad)) or np.max(np.abs(bad)) > 2


def test_btcs_first_order_in_time(oracle_lib):
    """Halving dt halves the change (smooth Cole-Hopf case, nu = 0.5, Courant numbers 2-8)."""
    sols = [_cole_hopf_run(oracle_lib, 200, W.BTCS, f, nu=0.5)[0] for f in (8.0, 4.0, 2.0)]
    ratio = np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2])
    assert 1.85 <= ratio <= 2.15, ratio


def test_btcs_converges_to_cole_hopf(oracle_lib):
    errs = [oracle_lib.rms(*_cole_hopf_run(oracle_lib, n, W.BTCS, 1.0)) for n in (400, 800, 1600)]
    slope = -np.polyfit(np.log([400, 800, 1600]), np.log(errs), 1)[0]
    assert 0.8 <= slope <= 1.3, (errs, slope)


# ------------------------------------------------------------------------------------ steady state
def _steady_profile(x, nu):
    """Continuous steady viscous shock with u(0)=1, u(1)=0: u = A tanh(A (1-x) / (2 nu)),
    A tanh(A / (2 nu)) = 1 (from u u_x = nu u_xx integrated once)."""
    A = 1.0
    for _ in range(60):
        f = A * math.tanh(A / (2 * nu)) - 1
        fp = math.tanh(A / (2 * nu)) + A / (2 * nu) / math.cosh(A / (2 * nu)) ** 2
        A -= f / fp
    return A * np.tanh(A * (1 - x) / (2 * nu))


def _run_to_steady(oracle_lib, p, u, chunk, max_chunks=400, tol=1e-13):
    for _ in range(max_chunks):
        nxt = oracle_lib.run([p], u, np.array([0, p.n]), chunk)
        if np.max(np.abs(nxt - u)) < tol:
            return nxt
        u = nxt
    raise AssertionError("no steady state")


def test_dirichlet_steady_state_explicit_btcs_and_closed_form(oracle_lib):
    """Both steppers share the discrete steady state, which converges to the viscous-shock profile."""
    nu = 0.1
    errs, ns = [], [33, 65, 129]
    for n in ns:
        x = W.node_coordinates(n, 1.0, W.BC_DIRICHLET)
        u0 = 1.0 - x
        dxv = 1.0 / (n - 1)
        pe = _problem(n, 1.0, nu, 0.5 * min(dxv, dxv * dxv / (2 * nu)), W.BC_DIRICHLET, W.EXPLICIT, 1.0, 0.0)
        pi = _problem(n, 1.0, nu, 50.0 * dxv, W.BC_DIRICHLET, W.BTCS, 1.0, 0.0)
        ue = _run_to_steady(oracle_lib, pe, u0, 2000, tol=1e-14)
        ui = _run_to_steady(oracle_lib, pi, u0, 20, tol=1e-13)
        assert np.max(np.abs(ue - ui)) <= 1e-10
        errs.append(np.max(np.abs(ui - _steady_profile(x, nu))))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 0.7 <= slope <= 1.3, (errs, slope)


# ------------------------------------------------------------------------------------ heat limit
@pytest.mark.parametrize("scheme", [W.EXPLICIT, W.BTCS])
def test_dirichlet_small_amplitude_heat_decay(oracle_lib, scheme):
    """Small amplitude: Burgers reduces to the heat equation; eps sin(pi x) on [0, 1] with a = b = 0
    decays as exp(-nu pi^2 t).  With dt ~ dx^2 the discrete decay converges at second order in dx,
    which fixes the Dirichlet grid spacing dx = L / (N - 1)."""
    nu, t_final, eps = 0.1, 0.2, 1e-9
    errs, ns = [], [17, 33, 65, 129]
    for n in ns:
        x = W.node_coordinates(n, 1.0, W.BC_DIRICHLET)
        u0 = eps * np.sin(np.pi * x)
        u0[0] = u0[-1] = 0.0
        h = 1.0 / (n - 1)
        dt_target = 0.2 * h * h / nu
        steps = int(math.ceil(t_final / dt_target))
        p = _problem(n, 1.0, nu, t_final / steps, W.BC_DIRICHLET, scheme)
        out = oracle_lib.run([p], u0, np.array([0, n]), steps)
        amp = out[(n - 1) // 2] / eps
        errs.append(abs(amp - math.exp(-nu * math.pi ** 2 * t_final)))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 1.8 <= slope <= 2.2, (errs, slope)


# ------------------------------------------------------------------------------------ batch driver
def test_run_matches_repeated_steps_bitwise(oracle_lib):
    batch = W.random_batch(13, 7, 3, 90, amplitude=2.0)
    for i, p in enumerate(batch.problems):
        p.dt = (1 + 9 * p.scheme) * oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, batch.umax[i], 0.5)
    out = oracle_lib.run(batch.problems, batch.u0, batch.offsets, 13, threads=3)
    for i, p in enumerate(batch.problems):
        u = batch.instance(i).copy()
        for _ in range(13):
            u = oracle_lib.explicit_step(p, u) if p.scheme == W.EXPLICIT else oracle_lib.btcs_step(p, u)
        assert np.array_equal(u, out[batch.offsets[i]:batch.offsets[i + 1]])


def test_large_explicit_split_matches_serial(oracle_lib):
    b = W.c3_problem(n=200_003)
    p = b.problems[0]
    p.dt = oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, b.umax[0], 0.5)
    a = oracle_lib.run_explicit_large(p, b.u0, 7, threads=4)
    c = oracle_lib.run([p], b.u0, b.offsets, 7)
    assert np.array_equal(a, c)


def test_fp32_oracle_tracks_fp64(oracle_lib):
    b = W.c1_problem(W.EXPLICIT)
    p = b.problems[0]
    p.dt = oracle_lib.cfl_dt(p.n, p.length, p.nu, p.bc, b.umax[0], 0.5)
    u64 = oracle_lib.run([p], b.u0, b.offsets, 100)
    u32 = oracle_lib.run([p], b.u0.astype(np.float32), b.offsets, 100)
    assert oracle_lib.rel_max_abs(u32, u64) < 1e-5


# ------------------------------------------------------------------------------------ adjoint
def _grad_case(seed, bc, scheme, positive):
    """Small batch for gradient checks: J = 1/2 sum (u_T - target)^2 after a few steps."""
    b = W.random_batch(seed, 3, 12, 40, bc=bc, scheme=scheme, amplitude=0.3 if positive else 2.0)
    if positive:
        b.u0 = b.u0 + 2.0
        for i, p in enumerate(b.problems):
            if p.bc == W.BC_DIRICHLET:
                p.left, p.right = b.u0[b.offsets[i]], b.u0[b.offsets[i + 1] - 1]
        b.umax = np.array([np.max(np.abs(b.instance(i))) for i in range(b.count)])
    for i, p in enumerate(b.problems):
        f = 1.0 if scheme == W.EXPLICIT else 6.0
        p.dt = f * 0.5 * min(p.length / p.n / b.umax[i], (p.length / p.n) ** 2 / (2 * p.nu))
    target = np.random.default_rng(seed + 1).standard_normal(len(b.u0)) * 0.1 + 1.0
    return b, target


def _loss(oracle_lib, b, u0, target, nsteps):
    uT = oracle_lib.run(b.problems, u0, b.offsets, nsteps)
    return 0.5 * float(np.sum((uT - target) ** 2)), uT


@pytest.mark.parametrize("scheme", [W.EXPLICIT, W.BTCS])
@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
@pytest.mark.parametrize("positive", [True, False])
def test_adjoint_matches_finite_differences(oracle_lib, scheme, bc, positive):
    """dJ/du0 along random directions and dJ/dnu by central differences of the (pinned) forward oracle."""
    b, target = _grad_case(60 + 2 * bc + scheme, bc, scheme, positive)
    nsteps = 7
    J0, uT = _loss(oracle_lib, b, b.u0, target, nsteps)
    g_u0, g_nu = oracle_lib.adjoint(b.problems, b.u0, b.offsets, uT - target, nsteps)
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(3):
        e = rng.standard_normal(len(b.u0))
        fd = (_loss(oracle_lib, b, b.u0 + h * e, target, nsteps)[0]
              - _loss(oracle_lib, b, b.u0 - h * e, target, nsteps)[0]) / (2 * h)
        assert abs(fd - np.dot(g_u0, e)) <= 1e-6 * (abs(fd) + 1e-8), (fd, np.dot(g_u0, e))
    for i, p in enumerate(b.problems):
        nu0 = p.nu
        hn = 1e-4 * nu0          # J ~ 100 while nu dJ/dnu ~ 1e-3: a smaller step drowns in rounding
        p.nu = nu0 + hn
        Jp = _loss(oracle_lib, b, b.u0, target, nsteps)[0]
        p.nu = nu0 - hn
        Jm = _loss(oracle_lib, b, b.u0, target, nsteps)[0]
        p.nu = nu0
        fd = (Jp - Jm) / (2 * hn)
        assert abs(fd - g_nu[i]) <= 1e-6 * (abs(fd) + 1e-8), (i, fd, g_nu[i])
    if bc == W.BC_DIRICHLET:
        for i in range(b.count):
            assert g_u0[b.offsets[i]] == 0.0 and g_u0[b.offsets[i + 1] - 1] == 0.0


@pytest.mark.parametrize("scheme", [W.EXPLICIT, W.BTCS])
@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_adjoint_is_transpose_of_tangent(oracle_lib, scheme, bc):
    """Dot-product test <T v, w> = <v, T^T w> with v = (du0, dnu): adjoint and tangent sweeps are written
    separately, so this fixes every transposition, corner and sign between them."""
    b, _ = _grad_case(80 + bc + 2 * scheme, bc, scheme, False)
    rng = np.random.default_rng(9)
    du0 = rng.standard_normal(len(b.u0))
    dnu = rng.standard_normal(b.count)
    w = rng.standard_normal(len(b.u0))
    for i, p in enumerate(b.problems):
        if p.bc == W.BC_DIRICHLET:
            w[b.offsets[i]] = w[b.offsets[i + 1] - 1] = 0.0
    nsteps = 9
    tv = oracle_lib.tangent(b.problems, b.u0, b.offsets, du0, dnu, nsteps)
    g_u0, g_nu = oracle_lib.adjoint(b.problems, b.u0, b.offsets, w, nsteps)
    lhs = float(np.dot(tv, w))
    rhs = float(np.dot(du0, g_u0) + np.dot(dnu, g_nu))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs)), (lhs, rhs)
