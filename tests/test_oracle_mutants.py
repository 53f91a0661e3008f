"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutant edits one expression of burgers_oracle.cpp (a dropped term, a flipped sign, a wrong index,
swapped cyclic corners), compiles it into a temporary library on the CPU, swaps it in for the real one
and runs the pin tests of test_oracle.py against it.  A mutant that passes every pin would mean the pins
do not cover that part of the method.
"""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
from oracle import build as obuild

import test_oracle as T

MUTANTS = {
    "diffusion_sign": ("T lap = (up + um) - two * ui;", "T lap = (up - um) - two * ui;"),
    "diffusion_dropped": ("+ D * lap;", "+ zero * lap;"),
    "upwind_always_backward": ("- cneg * (up - ui))", "- cneg * (ui - um))"),
    "upwind_direction_swapped": ("T cpos = c > zero ? c : zero;      // max(c, 0): backward difference",
                                 "T cpos = c < zero ? c : zero;      // max(c, 0): backward difference"),
    "periodic_wrap_index": ("um = u[i == 0 ? n - 1 : i - 1];", "um = u[i == 0 ? n - 2 : i - 1];"),
    "dirichlet_left_value": ("um = (i == 1) ? a : u[i - 1];", "um = (i == 1) ? b : u[i - 1];"),
    "btcs_diag_missing_D": ("d[k] = (one + two * D) + cabs;", "d[k] = one + cabs;"),
    "btcs_sub_sign": ("l[k] = -(D + cpos);", "l[k] = (D + cpos);"),
    "btcs_super_uses_cpos": ("p[k] = cneg - D;", "p[k] = -cpos - D;"),
    "btcs_dirichlet_rhs": ("rhs[0] = rhs[0] - l[0] * a;", "rhs[0] = rhs[0] + l[0] * a;"),
    "cyclic_corners_swapped": ("const T beta = l[0];\n  const T alpha = p[m - 1];",
                               "const T beta = p[m - 1];\n  const T alpha = l[0];"),
    "cyclic_gamma_sign": ("const T g = -d[0];", "const T g = d[0];"),
    "thomas_back_sub": ("x[k] = yw[k] - cw[k] * x[k + 1];", "x[k] = yw[k] + cw[k] * x[k + 1];"),
    "cfl_diffusive_factor": ("lim = std::min(lim, dx * dx / (2.0 * nu));", "lim = std::min(lim, dx * dx / nu);"),
    "dx_dirichlet": ("length / (double)(n - 1);", "length / (double)n;"),
    "cole_hopf_speed": ("std::fmod(x - 4.0 * t, two_pi)", "std::fmod(x - 3.0 * t, two_pi)"),
    "adj_explicit_self": ("self = 1.0 - r * (ui - um) - r * ui - 2.0 * D;", "self = 1.0 - r * (ui - um) + r * ui - 2.0 * D;"),
    "adj_explicit_left": ("left = r * ui + D;", "left = D;"),
    "adj_explicit_nu": ("gD += li * ((up + um) - 2.0 * ui);", "gD += li * ((up - um) - 2.0 * ui);"),
    "adj_btcs_untransposed": ("btcs_matrix_solve(n, bc, r, D, y, lamp, mu.data(), true);",
                              "btcs_matrix_solve(n, bc, r, D, y, lamp, mu.data(), false);"),
    "adj_btcs_g_sign": ("lam[i] = (1.0 - G[i]) * mu[i];", "lam[i] = (1.0 + G[i]) * mu[i];"),
    "adj_btcs_nu_sign": ("gD -= mu[i] * Lx[i];", "gD += mu[i] * Lx[i];"),
    "adj_transpose_corner": ("tp[k] = bc == PERIODIC ? l[(k + 1) % m]", "tp[k] = bc == PERIODIC ? l[k]"),
    "adj_g_upwind_side": ("G[i] = y[i] >= 0 ? r * (x[i] - xm) : r * (xp - x[i]);",
                          "G[i] = y[i] >= 0 ? r * (xp - x[i]) : r * (x[i] - xm);"),
    "tangent_drops_nu": ("dout[i] = v + D * dlap + dD * lap;", "dout[i] = v + D * dlap;"),
    "newton_convection_sign": ("const T F = (xi - u[i]) + (half_r * xi * (xp - xm) - D * ((xp + xm) - two * xi));",
                               "const T F = (xi - u[i]) + (-half_r * xi * (xp - xm) - D * ((xp + xm) - two * xi));"),
    "newton_jacobian_diag": ("d[k] = (one + two * D) + half_r * (xp - xm);", "d[k] = one + two * D;"),
    "newton_jacobian_sub": ("l[k] = -(half_r * xi) - D;", "l[k] = (half_r * xi) - D;"),
    "newton_upwinded": ("const T F = (xi - u[i]) + (half_r * xi * (xp - xm) - D * ((xp + xm) - two * xi));",
                        "const T F = (xi - u[i]) + (two * half_r * xi * (xi - xm) - D * ((xp + xm) - two * xi));"),
    "newton_diffusion_sign": ("const T F = (xi - u[i]) + (half_r * xi * (xp - xm) - D * ((xp + xm) - two * xi));",
                              "const T F = (xi - u[i]) + (half_r * xi * (xp - xm) + D * ((xp + xm) - two * xi));"),
    "cn_diag_half": ("d[k] = one + half * nd;", "d[k] = one + nd;"),
    "cn_rhs_sign": ("rhs[k] = ui - half * ((nl * um + nd * ui) + np * up);",
                    "rhs[k] = ui + half * ((nl * um + nd * ui) + np * up);"),
    "cn_rhs_neighbours_swapped": ("rhs[k] = ui - half * ((nl * um + nd * ui) + np * up);",
                                  "rhs[k] = ui - half * ((nl * up + nd * ui) + np * um);"),
    "cn_dirichlet_rhs": ("    rhs[0] = rhs[0] - l[0] * a;\n    rhs[m - 1] = rhs[m - 1] - p[m - 1] * b;\n    thomas",
                         "    rhs[0] = rhs[0] + l[0] * a;\n    rhs[m - 1] = rhs[m - 1] - p[m - 1] * b;\n    thomas"),
    "cn_sub_uses_half_twice": ("l[k] = half * nl;", "l[k] = half * half * nl;"),
    "rk4_weights": ("(((K1[i] + two * K2[i]) + two * K3[i]) + K4[i]) / six", "(((K1[i] + K2[i]) + K3[i]) + K4[i]) / six"),
    "rk4_half_stage": ("for (int64_t i = 0; i < n; ++i) v[i] = u[i] + half * K1[i];",
                       "for (int64_t i = 0; i < n; ++i) v[i] = u[i] + K1[i];"),
    "rk4_last_stage": ("for (int64_t i = 0; i < n; ++i) v[i] = u[i] + K3[i];",
                       "for (int64_t i = 0; i < n; ++i) v[i] = u[i] + half * K3[i];"),
    "rk4_increment_sign": ("K[i] = D * lap - (cpos * (vi - um) + cneg * (up - vi));",
                           "K[i] = D * lap + (cpos * (vi - um) + cneg * (up - vi));"),
    "rk4_upwind_side": ("K[i] = D * lap - (cpos * (vi - um) + cneg * (up - vi));",
                        "K[i] = D * lap - (cpos * (up - vi) + cneg * (vi - um));"),
}

PINS = [name for name in dir(T) if name.startswith("test_")]


def _call_pin(fn):
    import inspect
    params = inspect.signature(fn).parameters
    marks = getattr(fn, "pytestmark", [])
    cases = [dict()]
    for m in marks:
        if m.name == "parametrize":
            argnames = [a.strip() for a in m.args[0].split(",")]
            new = []
            for c in cases:
                for vals in m.args[1]:
                    vals = vals if isinstance(vals, tuple) else (vals,)
                    d = dict(c)
                    d.update(zip(argnames, vals))
                    new.append(d)
            cases = new
    for c in cases:
        kwargs = {k: v for k, v in c.items() if k in params}
        fn(oracle, **kwargs)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    src = open(obuild.SOURCE).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation site missing: {old!r}"
    with tempfile.TemporaryDirectory() as tmp:
        cpp = os.path.join(tmp, "mutant.cpp")
        so = os.path.join(tmp, "libmutant.so")
        open(cpp, "w").write(src.replace(old, new))
        subprocess.run(["g++", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c++17", "-shared", "-fPIC",
                        "-o", so, cpp], check=True)
        lib = oracle.configure(ctypes.CDLL(so))
        saved = oracle._load()
        oracle._lib = lib
        failed = []
        try:
            for pin in PINS:
                try:
                    _call_pin(getattr(T, pin))
                except Exception:                    # assertion, overflow or a non-converging loop
                    failed.append(pin)
                    break
        finally:
            oracle._lib = saved
        assert failed, f"mutant {name} passed every pin"
