"""C-ABI checks that need no GPU: the library loads, exports what include/burgers.h declares, validates
arguments before touching the device, and its host-side time-step arithmetic agrees with the oracle."""
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2601_12204_amd as B
    return B.load()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "burgers.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(burgers_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("burgers_create", "burgers_step_explicit", "burgers_step_btcs", "burgers_run",
                 "burgers_adjoint", "burgers_destroy", "burgers_sync", "burgers_offsets",
                 "burgers_cfl_dt", "burgers_status_string"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    import paper_2601_12204_amd as B
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) <= set(B.EXPORTS) | set(declared_symbols())
    assert B.burgers_abi_version() == 1


def test_status_strings(lib):
    import paper_2601_12204_amd as B
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert B.burgers_status_string(code) == B.STATUS[code]


def test_cfl_dt_and_ratios_match_oracle_bitwise(lib, oracle_lib):
    import paper_2601_12204_amd as B
    rng = np.random.default_rng(3)
    for _ in range(200):
        bc = int(rng.integers(0, 2))
        p = W.Problem(n=int(rng.integers(3, 1 << 24)), length=float(rng.uniform(0.1, 10)),
                      nu=float(rng.uniform(0, 1)), bc=bc)
        umax = float(rng.uniform(0, 10))
        dt_lib = B.burgers_cfl_dt(p, umax, 0.5)
        assert dt_lib == oracle_lib.cfl_dt(p.n, p.length, p.nu, bc, umax, 0.5)
        p.dt = dt_lib
        assert B.burgers_ratios(p) == oracle_lib.ratios(p)
    assert math.isnan(B.burgers_cfl_dt(W.Problem(n=2, length=1.0, nu=0.1), 1.0, 0.5))


def test_create_rejects_invalid_problems_without_a_device(lib):
    import ctypes
    import paper_2601_12204_amd as B
    good = W.Problem(n=16, length=1.0, nu=0.01, dt=1e-3)
    bad = [dict(n=2), dict(length=0.0), dict(nu=-1.0), dict(dt=0.0), dict(dt=float("nan")),
           dict(bc=2), dict(scheme=5), dict(scheme=-1), dict(left=float("inf")), dict(n=(1 << 31) - 65535)]
    for change in bad:
        p = W.Problem(**{**good.__dict__, **change})
        arr = (B.CProblem * 1)(B.to_cproblem(p))
        h = ctypes.c_void_p()
        assert lib.burgers_create(arr, 1, B.F64, None, ctypes.byref(h)) == -1, change
        assert not h.value
    arr = (B.CProblem * 1)(B.to_cproblem(good))
    h = ctypes.c_void_p()
    assert lib.burgers_create(arr, 0, B.F64, None, ctypes.byref(h)) == -1
    assert lib.burgers_create(arr, 1, 7, None, ctypes.byref(h)) == -1
    assert lib.burgers_create(None, 1, B.F64, None, ctypes.byref(h)) == -1
    assert lib.burgers_create(arr, 1, B.F64, None, None) == -1
    lib.burgers_destroy(None)


def test_null_context_calls_are_invalid(lib):
    import paper_2601_12204_amd as B
    for name in ("burgers_step_explicit", "burgers_step_btcs", "burgers_run"):
        assert getattr(lib, name)(None, None, 1) == -1
    assert lib.burgers_sync(None) == -1
    assert lib.burgers_adjoint(None, None, None, 1, 1, None, None) == -1
    assert lib.burgers_offsets(None, None) == -1
    assert lib.burgers_state_elems(None) == -1
    plan = B.CPlan()
    assert lib.burgers_get_plan(None, plan) == -1


def test_run_static_rejects_invalid_arguments_without_a_device(lib):
    """The allocation-free entry point validates everything before it touches the device."""
    import ctypes
    import paper_2601_12204_amd as B
    good = W.Problem(n=16, length=1.0, nu=0.01, dt=1e-3)
    arr = (B.CProblem * 1)(B.to_cproblem(good))
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails its checks first
    assert lib.burgers_run_static(None, 1, B.F64, None, dummy, 1) == -1
    assert lib.burgers_run_static(arr, 0, B.F64, None, dummy, 1) == -1
    assert lib.burgers_run_static(arr, 1, 7, None, dummy, 1) == -1
    assert lib.burgers_run_static(arr, 1, B.F64, None, None, 1) == -1
    assert lib.burgers_run_static(arr, 1, B.F64, None, dummy, -1) == -1
    bad = (B.CProblem * 1)(B.to_cproblem(W.Problem(**{**good.__dict__, "n": 2})))
    assert lib.burgers_run_static(bad, 1, B.F64, None, dummy, 1) == -1
    newton = (B.CProblem * 1)(B.to_cproblem(W.Problem(**{**good.__dict__, "scheme": W.NEWTON})))
    assert lib.burgers_run_static(newton, 1, B.F64, None, dummy, 1) == -2
    text = open(os.path.join(ROOT, "include", "burgers.h")).read()
    assert re.search(r"#define BURGERS_STATIC_SCRATCH_BYTES \(64u << 20\)", text)
    assert B.STATIC_SCRATCH_BYTES == 64 << 20


def test_single_hip_runtime_in_process():
    """Loading the binding first and torch afterwards must leave exactly one HIP runtime mapped, so that
    torch's streams and allocations are valid handles in the library."""
    import subprocess
    import sys
    code = ("import paper_2601_12204_amd as B; B.load(); import torch; "
            "maps = open('/proc/self/maps').read().split('\\n'); "
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l}; print(len(libs)); print(libs)")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, check=True)
    assert out.stdout.splitlines()[0] == "1", out.stdout
