"""CPU oracle for the matrix-free SEM Burgers operators (test infrastructure only).

A plain FP64 C implementation (``sem_oracle.c``) of F(u), J(u)v, J(u)^T w, classical RK4, its
tangent-linear model and its discrete adjoint with uniform checkpoints, following arXiv 1806.01422
(Sec. 3.2-3.3 for the operators, Sec. 4.1 for the adjoint, Sec. 5.3-5.4 for checkpointing).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use this module.  The
product library never imports it, and it imports nothing from the product.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))


class OrcDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("N", ctypes.c_int32), ("E", ctypes.c_int32 * 3),
                ("L", ctypes.c_double * 3), ("nu", ctypes.c_double), ("batch", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pd = ctypes.POINTER(OrcDesc)
        _lib.orc_gll.argtypes = [ctypes.c_int, dp, dp, dp]
        for name in ("orc_rhs",):
            getattr(_lib, name).argtypes = [pd, dp, dp]
        for name in ("orc_jac_vec", "orc_jact_vec"):
            getattr(_lib, name).argtypes = [pd, dp, dp, dp]
        _lib.orc_rk4_forward.argtypes = [pd, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, dp, dp]
        _lib.orc_rk4_adjoint.argtypes = [pd, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, dp, dp]
        _lib.orc_rk4_tlm.argtypes = [pd, ctypes.c_double, ctypes.c_int32, dp, dp]
        i32 = ctypes.c_int32
        _lib.orc_erk_tableau.argtypes = [i32, dp, dp]
        _lib.orc_erk_forward.argtypes = [pd, i32, ctypes.c_double, i32, i32, dp, dp]
        _lib.orc_erk_adjoint.argtypes = [pd, i32, ctypes.c_double, i32, i32, dp, dp]
        _lib.orc_erk_tlm.argtypes = [pd, i32, ctypes.c_double, i32, dp, dp]
        _lib.orc_misfit.argtypes = [pd, dp, dp, dp, dp]
        _lib.orc_coords.argtypes = [pd, ctypes.c_int32, dp]
        _lib.orc_mass.argtypes = [pd, dp]
        _lib.orc_project_local.argtypes = [pd, dp, dp]
        _lib.orc_num_threads.argtypes = []
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib.orc_set_threads.restype = None
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def gll(N):
    """GLL nodes xi (N+1), weights w (N+1) and derivative matrix D[(i, j)] = l_j'(xi_i)."""
    P = N + 1
    xi, w, D = np.zeros(P), np.zeros(P), np.zeros((P, P))
    _check(lib().orc_gll(N, _ptr(xi), _ptr(w), _ptr(D)), "gll")
    return xi, w, D


class Mesh:
    """Uniform periodic box of E_d elements of order N per direction, batch of fields."""

    def __init__(self, dim, N, E, L, nu, batch=1):
        E = list(E) + [1] * (3 - len(E))
        L = list(L) + [1.0] * (3 - len(L))
        self.dim, self.N, self.E, self.L, self.nu, self.batch = dim, N, E[:3], L[:3], float(nu), batch
        self.n = [E[k] * N if k < dim else 1 for k in range(3)]
        self.nodes = int(np.prod(self.n))
        self.C = dim
        self.ndof = self.nodes * self.C
        self._d = OrcDesc(dim, N, (ctypes.c_int32 * 3)(*self.E), (ctypes.c_double * 3)(*self.L),
                          self.nu, batch)

    def with_batch(self, batch):
        return Mesh(self.dim, self.N, self.E, self.L, self.nu, batch)

    @property
    def shape(self):
        """Field shape [batch][C][nz][ny][nx] with the unused directions dropped."""
        spatial = [self.n[k] for k in reversed(range(self.dim))]
        return (self.batch, self.C, *spatial)

    def zeros(self):
        return np.zeros(self.shape)

    def coords(self, k):
        x = np.zeros(self.n[k])
        _check(lib().orc_coords(ctypes.byref(self._d), k, _ptr(x)), "coords")
        return x

    def mass(self):
        """Assembled diagonal mass of one component, shaped like one component field."""
        M = np.zeros(self.nodes)
        _check(lib().orc_mass(ctypes.byref(self._d), _ptr(M)), "mass")
        return M.reshape(self.shape[2:])

    def _in(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.size == self.batch * self.ndof, (a.shape, self.shape)
        return a

    def rhs(self, u):
        u = self._in(u)
        f = np.zeros_like(u)
        _check(lib().orc_rhs(ctypes.byref(self._d), _ptr(u), _ptr(f)), "rhs")
        return f

    def jac_vec(self, u, v):
        u, v = self._in(u), self._in(v)
        out = np.zeros_like(u)
        _check(lib().orc_jac_vec(ctypes.byref(self._d), _ptr(u), _ptr(v), _ptr(out)), "jac_vec")
        return out

    def jact_vec(self, u, w):
        u, w = self._in(u), self._in(w)
        out = np.zeros_like(u)
        _check(lib().orc_jact_vec(ctypes.byref(self._d), _ptr(u), _ptr(w), _ptr(out)), "jact_vec")
        return out

    @property
    def nelem(self):
        return int(np.prod(self.E[:self.dim]))

    @property
    def nloc(self):
        return (self.N + 1) ** self.dim

    def project_local(self, loc):
        """M^{-1} Q^T (omega o loc) for an element-local field loc[batch][nelem][C][nloc]."""
        loc = np.ascontiguousarray(loc, dtype=np.float64)
        assert loc.size == self.batch * self.nelem * self.C * self.nloc
        out = self.zeros()
        _check(lib().orc_project_local(ctypes.byref(self._d), _ptr(loc), _ptr(out)), "project_local")
        return out

    def rk4_forward(self, u0, dt, nsteps, ckpt_every=None):
        """Returns (u(T), checkpoints or None).  checkpoints: [nsteps/K][batch][...]."""
        u = self._in(u0).copy()
        ck = None
        if ckpt_every:
            ck = np.zeros((nsteps // ckpt_every,) + u.shape)
        _check(lib().orc_rk4_forward(ctypes.byref(self._d), dt, nsteps, ckpt_every or 0, _ptr(u),
                                      _ptr(ck)), "rk4_forward")
        return u, ck

    def rk4_adjoint(self, ckpt, dt, nsteps, ckpt_every, lamT):
        lam = self._in(lamT).copy()
        ck = np.ascontiguousarray(ckpt, dtype=np.float64)
        _check(lib().orc_rk4_adjoint(ctypes.byref(self._d), dt, nsteps, ckpt_every, _ptr(ck), _ptr(lam)),
               "rk4_adjoint")
        return lam

    def rk4_tlm(self, u0, du0, dt, nsteps):
        u, du = self._in(u0).copy(), self._in(du0).copy()
        _check(lib().orc_rk4_tlm(ctypes.byref(self._d), dt, nsteps, _ptr(u), _ptr(du)), "rk4_tlm")
        return u, du

    # General explicit Runge-Kutta by Butcher tableau: scheme "rk4" (classical) or "rk3" (Kutta's
    # third-order method, the reading taken for the paper's three-stage RK-3).
    def erk_forward(self, scheme, u0, dt, nsteps, ckpt_every=None):
        u = self._in(u0).copy()
        ck = None
        if ckpt_every:
            ck = np.zeros((nsteps // ckpt_every,) + u.shape)
        _check(lib().orc_erk_forward(ctypes.byref(self._d), SCHEMES[scheme], dt, nsteps, ckpt_every or 0, _ptr(u),
                                      _ptr(ck)), "erk_forward")
        return u, ck

    def erk_adjoint(self, scheme, ckpt, dt, nsteps, ckpt_every, lamT):
        lam = self._in(lamT).copy()
        ck = np.ascontiguousarray(ckpt, dtype=np.float64)
        _check(lib().orc_erk_adjoint(ctypes.byref(self._d), SCHEMES[scheme], dt, nsteps, ckpt_every, _ptr(ck),
                                      _ptr(lam)), "erk_adjoint")
        return lam

    def erk_tlm(self, scheme, u0, du0, dt, nsteps):
        u, du = self._in(u0).copy(), self._in(du0).copy()
        _check(lib().orc_erk_tlm(ctypes.byref(self._d), SCHEMES[scheme], dt, nsteps, _ptr(u), _ptr(du)), "erk_tlm")
        return u, du

    def misfit(self, uT, target):
        uT, target = self._in(uT), self._in(target)
        phi = np.zeros(self.batch)
        lam = np.zeros_like(uT)
        _check(lib().orc_misfit(ctypes.byref(self._d), _ptr(uT), _ptr(target), _ptr(phi), _ptr(lam)),
               "misfit")
        return phi, lam

    def gradient(self, u0, target, dt, nsteps, ckpt_every):
        """Misfit Phi = 1/2 ||u(T) - u*||^2 per batch member and dPhi/du0 (discrete adjoint)."""
        uT, ck = self.rk4_forward(u0, dt, nsteps, ckpt_every)
        phi, lamT = self.misfit(uT, target)
        return phi, self.rk4_adjoint(ck, dt, nsteps, ckpt_every, lamT)


SCHEMES = {"rk4": 0, "rk3": 1}


def erk_tableau(scheme):
    """(A, b) of an explicit Runge-Kutta scheme as the oracle uses it."""
    A, b = np.zeros(16), np.zeros(4)
    s = lib().orc_erk_tableau(SCHEMES[scheme], _ptr(A), _ptr(b))
    if s < 0:
        raise ValueError(scheme)
    return A[: s * s].reshape(s, s).copy(), b[:s].copy()


def num_threads():
    return int(lib().orc_num_threads())


def set_threads(n):
    """Threads of later oracle calls (n < 1: all the host offers)."""
    lib().orc_set_threads(int(n))
