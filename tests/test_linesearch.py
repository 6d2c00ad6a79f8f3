"""Host-side pins of libsem's More-Thuente line search (the step-length rule of the paper's LMVM
optimiser, Sec. 5; no GPU needed): on smooth one-dimensional functions, from small and large
initial steps and for loose and tight tolerances, every trial step equals the one SciPy's
independent implementation of the same published method (DCSRCH) takes, and the accepted step
satisfies the strong Wolfe conditions."""
import ctypes
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


class LS(ctypes.Structure):
    _fields_ = [("ftol", ctypes.c_double), ("gtol", ctypes.c_double), ("xtol", ctypes.c_double),
                ("stpmin", ctypes.c_double), ("stpmax", ctypes.c_double), ("work", ctypes.c_double * 14),
                ("iwork", ctypes.c_int32 * 4)]


START, FG, CONV, WARN, ERR = 0, 1, 2, 3, 4

FUNCS = {
    # phi(a), phi'(a): shapes with a single interior minimiser, a flat tail, and a steep wall
    "rational": (lambda a: -a / (a * a + 2.0), lambda a: (a * a - 2.0) / (a * a + 2.0) ** 2),
    "quintic": (lambda a: (a + 0.004) ** 5 - 2.0 * (a + 0.004) ** 4,
                lambda a: 5 * (a + 0.004) ** 4 - 8 * (a + 0.004) ** 3),
    "wiggle": (lambda a: (1 - a) ** 2 + 0.01 * math.sin(30 * a), lambda a: -2 * (1 - a) + 0.3 * math.cos(30 * a)),
    "exp": (lambda a: math.exp(-3 * a) + 0.5 * a * a, lambda a: -3 * math.exp(-3 * a) + a),
}


@pytest.fixture(scope="module")
def lib():
    import paper_1806_01422_amd as P
    L = P.lib()
    L.sem_line_search_step.argtypes = [ctypes.POINTER(LS), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double]
    return L


def ours(lib, phi, dphi, stp0, ftol, gtol, xtol, stpmin, stpmax, maxit=60):
    ls = LS(ftol, gtol, xtol, stpmin, stpmax)
    task, stp = ctypes.c_int32(START), ctypes.c_double(stp0)
    assert lib.sem_line_search_step(ctypes.byref(ls), ctypes.byref(task), ctypes.byref(stp), phi(0.0), dphi(0.0)) == 0
    steps = []
    for _ in range(maxit):
        if task.value != FG:
            break
        steps.append(stp.value)
        assert lib.sem_line_search_step(ctypes.byref(ls), ctypes.byref(task), ctypes.byref(stp), phi(stp.value),
                                        dphi(stp.value)) == 0
    return steps, stp.value, task.value


def reference(phi, dphi, stp0, ftol, gtol, xtol, stpmin, stpmax, maxit=60):
    from scipy.optimize._dcsrch import DCSRCH
    steps = []

    def p(a):
        steps.append(float(a))
        return phi(a)
    ds = DCSRCH(p, dphi, ftol, gtol, xtol, stpmin, stpmax)
    stp, _, _, task = ds(stp0, phi(0.0), dphi(0.0), maxiter=maxit)
    return steps, stp, task


@pytest.mark.parametrize("name", sorted(FUNCS))
@pytest.mark.parametrize("stp0", [1e-3, 0.1, 10.0, 1e3])
@pytest.mark.parametrize("ftol,gtol", [(1e-3, 0.1), (0.1, 1e-3), (1e-4, 0.9)])
def test_steps_match_reference(lib, name, stp0, ftol, gtol):
    phi, dphi = FUNCS[name]
    if dphi(0.0) >= 0:
        pytest.skip("not a descent direction")
    a, sa, ta = ours(lib, phi, dphi, stp0, ftol, gtol, 1e-10, 0.0, 1e10)
    b, sb, tb = reference(phi, dphi, stp0, ftol, gtol, 1e-10, 0.0, 1e10)
    assert len(a) == len(b), (a, b)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)
    if ta == CONV:
        assert tb.startswith(b"CONV") if isinstance(tb, bytes) else str(tb).startswith("CONV")
        f0, g0 = phi(0.0), dphi(0.0)
        assert phi(sa) <= f0 + ftol * sa * g0 and abs(dphi(sa)) <= gtol * abs(g0)


def test_invalid_start_is_an_error(lib):
    phi, dphi = FUNCS["rational"]
    ls = LS(1e-3, 0.1, 1e-10, 0.0, 10.0)
    task, stp = ctypes.c_int32(START), ctypes.c_double(1.0)
    lib.sem_line_search_step(ctypes.byref(ls), ctypes.byref(task), ctypes.byref(stp), 0.0, +1.0)  # ascent
    assert task.value == ERR
