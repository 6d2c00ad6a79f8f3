"""Host-side pins of libsem's More-Thuente line search (the step-length rule of the paper's LMVM
optimiser, Sec. 5; no GPU needed), by the properties the method guarantees, on the six test
problems of More and Thuente's paper, from small and large initial steps and several tolerance
pairs:
  - every trial step lies in [stpmin, stpmax];
  - a converged step meets the strong Wolfe conditions;
  - in stage 1 the best step found so far has sufficient decrease (psi <= 0);
  - once a minimiser is bracketed, the bracket holds a point meeting both tests (a local minimiser
    of psi with psi <= 0, when ftol <= gtol);
  - the search ends within a small number of evaluations.
SciPy's implementation of the same published method (DCSRCH) is compared with as a cross-check
that reports agreement but does not gate the tests."""
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
MAX_EVALS = 30


def _gamma(b):
    return math.sqrt(1.0 + b * b) - b


def _yanai(b1, b2):
    # problems 4-6: phi(a) = gamma(b1) sqrt((1 - a)^2 + b2^2) + gamma(b2) sqrt(a^2 + b1^2)
    g1, g2 = _gamma(b1), _gamma(b2)
    return (lambda a: g1 * math.sqrt((1 - a) ** 2 + b2 * b2) + g2 * math.sqrt(a * a + b1 * b1),
            lambda a: g1 * (a - 1) / math.sqrt((1 - a) ** 2 + b2 * b2) + g2 * a / math.sqrt(a * a + b1 * b1))


def _wiggly(b=0.01, l=39):
    # problem 3: a kinked line smoothed over [1 - b, 1 + b] plus a sine of l half-periods
    def base(a):
        if a <= 1 - b:
            return 1 - a, -1.0
        if a >= 1 + b:
            return a - 1, 1.0
        return (a - 1) ** 2 / (2 * b) + b / 2, (a - 1) / b
    amp = 2 * (1 - b) / (l * math.pi)
    return (lambda a: base(a)[0] + amp * math.sin(l * math.pi * a / 2),
            lambda a: base(a)[1] + (1 - b) * math.cos(l * math.pi * a / 2))


FUNCS = {
    "mt1": (lambda a: -a / (a * a + 2.0), lambda a: (a * a - 2.0) / (a * a + 2.0) ** 2),
    "mt2": (lambda a: (a + 0.004) ** 5 - 2.0 * (a + 0.004) ** 4,
            lambda a: 5 * (a + 0.004) ** 4 - 8 * (a + 0.004) ** 3),
    "mt3": _wiggly(),
    "mt4": _yanai(0.001, 0.001),
    "mt5": _yanai(0.01, 0.001),
    "mt6": _yanai(0.001, 0.01),
}
TOLS = [(1e-3, 0.1), (1e-4, 0.9), (1e-3, 1e-3), (0.1, 1e-3)]
STEPS0 = [1e-3, 1e-1, 10.0, 1e3]


@pytest.fixture(scope="module")
def lib():
    import paper_1806_01422_amd as P
    L = P.lib()
    L.sem_line_search_step.argtypes = [ctypes.POINTER(LS), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double]
    return L


def run(lib, phi, dphi, stp0, ftol, gtol, xtol=1e-10, stpmin=0.0, stpmax=1e10, watch=None):
    """Drives the search; watch(ls) sees the state after every call.  Returns trials, step, task."""
    ls = LS(ftol, gtol, xtol, stpmin, stpmax)
    task, stp = ctypes.c_int32(START), ctypes.c_double(stp0)
    assert lib.sem_line_search_step(ctypes.byref(ls), ctypes.byref(task), ctypes.byref(stp), phi(0.0), dphi(0.0)) == 0
    trials = []
    while task.value == FG and len(trials) < 100:
        trials.append(stp.value)
        assert lib.sem_line_search_step(ctypes.byref(ls), ctypes.byref(task), ctypes.byref(stp), phi(stp.value),
                                        dphi(stp.value)) == 0
        if watch:
            watch(ls)
    return trials, stp.value, task.value


def holds_acceptable_point(phi, dphi, lo, hi, f0, g0, ftol, n=4001):
    """True if [lo, hi] contains a local minimiser of psi(t) = phi(t) - f0 - ftol t g0 (or of phi)
    with psi <= 0: psi' (or phi') changes sign from - to + between neighbouring samples, at least
    one of which has psi <= 0."""
    t = np.linspace(lo, hi, n)
    psi = np.array([phi(x) - f0 - ftol * x * g0 for x in t])
    d = np.array([dphi(x) for x in t])
    for slope in (d - ftol * g0, d):
        turn = (slope[:-1] <= 0) & (slope[1:] >= 0) & (np.minimum(psi[:-1], psi[1:]) <= 0)
        if turn.any():
            return True
    return False


CASES = [(n, s, ft, gt) for n in sorted(FUNCS) for s in STEPS0 for ft, gt in TOLS]


@pytest.mark.parametrize("name,stp0,ftol,gtol", CASES)
def test_properties(lib, name, stp0, ftol, gtol):
    phi, dphi = FUNCS[name]
    f0, g0 = phi(0.0), dphi(0.0)
    assert g0 < 0
    seen = []

    def watch(ls):
        lt, ut = ls.work[2], ls.work[5]
        seen.append((ls.iwork[0], ls.iwork[1], lt, ut))
        if ls.iwork[0] == 1:  # stage 1: the best step found so far has sufficient decrease
            assert phi(lt) <= f0 + ftol * lt * g0 + 1e-15 * abs(f0)
        if ls.iwork[1] and ftol <= gtol:
            assert holds_acceptable_point(phi, dphi, min(lt, ut), max(lt, ut), f0, g0, ftol), (lt, ut)

    trials, stp, task = run(lib, phi, dphi, stp0, ftol, gtol, watch=watch)
    assert task in (CONV, WARN), task
    assert len(trials) <= MAX_EVALS, len(trials)
    assert all(0.0 <= t <= 1e10 for t in trials)
    if task == CONV:
        assert phi(stp) <= f0 + ftol * stp * g0
        assert abs(dphi(stp)) <= gtol * abs(g0)
    else:  # a warning ends at the best step found, which has sufficient decrease
        assert phi(stp) <= f0 + ftol * stp * g0


@pytest.mark.parametrize("name", sorted(FUNCS))
def test_converges_for_standard_tolerances(lib, name):
    """With ftol <= gtol the method's guarantee applies: every start converges."""
    phi, dphi = FUNCS[name]
    for stp0 in STEPS0:
        for ftol, gtol in [(1e-3, 0.1), (1e-4, 0.9)]:
            _, _, task = run(lib, phi, dphi, stp0, ftol, gtol)
            assert task == CONV, (stp0, ftol, gtol)


def test_respects_step_bounds(lib):
    phi, dphi = FUNCS["mt1"]  # minimiser at sqrt(2)
    trials, stp, task = run(lib, phi, dphi, 0.1, 1e-3, 0.1, stpmax=0.5)
    assert all(t <= 0.5 for t in trials) and stp == 0.5 and task == WARN
    trials, stp, task = run(lib, phi, dphi, 10.0, 1e-3, 0.1, stpmin=5.0)
    assert all(t >= 5.0 for t in trials) and stp >= 5.0 and task in (CONV, WARN)


def test_invalid_start_is_an_error(lib):
    phi, dphi = FUNCS["mt1"]
    for f, g, stp, lo, hi in [(0.0, +1.0, 1.0, 0.0, 10.0),   # ascent direction
                              (0.0, -1.0, 20.0, 0.0, 10.0),  # initial step above stpmax
                              (0.0, -1.0, 1.0, 2.0, 10.0)]:  # initial step below stpmin
        ls = LS(1e-3, 0.1, 1e-10, lo, hi)
        task, s = ctypes.c_int32(START), ctypes.c_double(stp)
        lib.sem_line_search_step(ctypes.byref(ls), ctypes.byref(task), ctypes.byref(s), f, g)
        assert task.value == ERR


def test_crosscheck_with_scipy(lib):
    """Non-gating: how often SciPy's DCSRCH takes the same trial steps (up to rounding).  The
    methods are the same; SciPy evaluates the best step once more before a warning, which this
    implementation returns directly."""
    try:
        from scipy.optimize._dcsrch import DCSRCH
    except ImportError:
        pytest.skip("SciPy's DCSRCH not available")
    same = 0
    for name, stp0, ftol, gtol in CASES:
        phi, dphi = FUNCS[name]
        a, _, _ = run(lib, phi, dphi, stp0, ftol, gtol)
        b = []

        def p(x, phi=phi):
            b.append(float(x))
            return phi(x)
        DCSRCH(p, dphi, ftol, gtol, 1e-10, 0.0, 1e10)(stp0, phi(0.0), dphi(0.0), maxiter=100)
        n = min(len(a), len(b))
        if n and np.allclose(a[:n], b[:n], rtol=1e-8, atol=0):
            same += 1
    print(f"cross-check: {same} of {len(CASES)} trial sequences agree with SciPy's DCSRCH")
