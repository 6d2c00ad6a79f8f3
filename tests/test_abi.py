"""CPU checks of the C-ABI boundary and host-side logic (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")
LIB = os.path.join(ROOT, "paper_1806_01422_amd", "libsem.so")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(sem_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def libsem():
    if not os.path.exists(LIB):
        from paper_1806_01422_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = header_functions()
    for f in ("sem_setup", "sem_destroy", "sem_rhs", "sem_jac_vec", "sem_jact_vec", "sem_rk4_forward",
              "sem_rk4_adjoint", "sem_batch_setup", "sem_batch_rk4_forward", "sem_batch_rk4_adjoint",
              "sem_batch_autotune", "sem_last_error"):
        assert f in fns


def test_library_exports_every_declared_symbol(libsem):
    for f in header_functions():
        assert hasattr(libsem, f), f


def test_binding_covers_the_header():
    from paper_1806_01422_amd import sem
    assert sorted(sem.EXPORTED) == header_functions()


def test_last_error_without_gpu(libsem):
    libsem.sem_last_error.restype = ctypes.c_char_p
    libsem.sem_setup.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p()
    # a null descriptor is rejected before any device work
    assert libsem.sem_setup(None, None, ctypes.byref(out)) == -1
    assert b"descriptor" in libsem.sem_last_error()


def test_probe_rejects_bad_arguments_without_gpu(libsem):
    # argument errors are reported before any device call
    fn = libsem.sem_probe_fp64_rates
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    out = (ctypes.c_double * 4)()
    assert fn(None, 0, out) == -1
    assert fn(None, 10, None) == -1
    libsem.sem_last_error.restype = ctypes.c_char_p
    assert b"sem_probe_fp64_rates" in libsem.sem_last_error()


def test_lattice_and_fourier_recipe():
    assert len(wl.lattice(1, 3)) == 6
    assert len(wl.lattice(2, 1)) == 4
    ks = wl.lattice(3, 6)
    assert all(0 < sum(v * v for v in k) <= 36 for k in ks)
    x = np.linspace(0, 1, 17)[:-1]
    f = wl.fourier_field([x, x], [1.0, 1.0], 2, 5)
    assert f.shape == (2, 16, 16) and abs(np.abs(f).max() - 1.0) < 1e-15
    # periodic with zero mean (no k = 0 mode) on a uniform grid
    assert abs(f.mean()) < 1e-12
    # same seed, same field
    np.testing.assert_array_equal(f, wl.fourier_field([x, x], [1.0, 1.0], 2, 5))


def test_batched_problem_recipe():
    a, b = wl.c5_problems(), wl.c5_problems()
    assert len(a) == 128 and a == b
    assert {p.E for p in a} <= set(wl.C5_E) and {p.N for p in a} <= set(wl.C5_N)
    assert all(1e-4 <= p.nu <= 1e-2 and p.dt > 0 for p in a)
    # each step is inside its stability estimate, and the horizon ends at about half the time
    # 1 / (2 pi K) ~ 0.04 in which the initial field's steepest mode (K = 4, max|u0| = 1) forms a shock
    assert all(p.dt <= wl.stable_dt(2, p.N, p.E, 1.0, p.nu) for p in a)
    assert all(p.dt * wl.C5_STEPS <= wl.C5_T_MAX * (1 + 1e-12) for p in a)
    assert wl.C5_T_MAX < 0.6 / (2 * np.pi * wl.C5_K)
    # the 2-D 64x64 N=7 step of the adjoint configuration is inside the estimated stability region
    assert wl.C4_DT < wl.stable_dt(2, 7, 64, 1.0, 1e-3, safety=1.0)
