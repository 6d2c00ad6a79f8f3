"""ctypes binding of libsem (include/sem.h): argument marshalling only.

Every operator, integrator and adjoint runs in libsem's HIP kernels on the GPU; PyTorch only
provides device memory and the current stream.  There is no CPU fallback: if libsem.so is missing
or no GPU is present, the calls raise.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

SEM_F64, SEM_F32 = 0, 1


# time-integration schemes (sem_scheme): classical RK4 and the three-stage RK-3 (Kutta's tableau)
SCHEMES = {"rk4": 0, "rk3": 1}
_ALL_SCHEMES = {"rk4": 0, "rk3": 1, "cn": 2}


def _scheme(name):
    if name not in SCHEMES:
        raise SemError(f"unknown scheme {name!r}; expected one of {sorted(SCHEMES)}")
    return SCHEMES[name]


class NkOpts(ctypes.Structure):
    """sem_nk_opts: Newton-Krylov settings of the Crank-Nicolson calls (zeros select defaults)."""
    _fields_ = [("newton_rtol", ctypes.c_double), ("newton_maxit", ctypes.c_int32), ("gmres_rtol", ctypes.c_double),
                ("gmres_restart", ctypes.c_int32), ("gmres_maxit", ctypes.c_int32)]


class NkStats(ctypes.Structure):
    """sem_nk_stats: iteration counts of a Crank-Nicolson call."""
    _fields_ = [("newton_iters", ctypes.c_int64), ("linear_solves", ctypes.c_int64), ("gmres_iters", ctypes.c_int64),
                ("max_rel_residual", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LmvmOpts(ctypes.Structure):
    """sem_lmvm_opts (zeros select defaults)."""
    _fields_ = [("max_iters", ctypes.c_int32), ("memory", ctypes.c_int32), ("gatol", ctypes.c_double),
                ("grtol", ctypes.c_double), ("ftol", ctypes.c_double), ("gtol", ctypes.c_double),
                ("xtol", ctypes.c_double), ("max_evals", ctypes.c_int32)]


class LmvmStats(ctypes.Structure):
    """sem_lmvm_stats."""
    _fields_ = [("iters", ctypes.c_int32), ("evals", ctypes.c_int32), ("reason", ctypes.c_int32),
                ("f0", ctypes.c_double), ("f", ctypes.c_double), ("gnorm", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SemError(RuntimeError):
    pass


class SemDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("elems", ctypes.c_int32 * 3), ("order", ctypes.c_int32),
                ("length", ctypes.c_double * 3), ("nu", ctypes.c_double), ("dtype", ctypes.c_int32),
                ("batch", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
ADJOINT_STAGES = {"auto": 0, "store": 1, "recompute": 2}  # sem_adj_stages
_SIGS = {
    "sem_setup": [ctypes.POINTER(SemDesc), _vp, ctypes.POINTER(_vp)],
    "sem_destroy": [_vp],
    "sem_set_stream": [_vp, _vp],
    "sem_query": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "sem_query_path": [_vp, ctypes.POINTER(_i32)],
    "sem_node_coords": [_vp, _i32, ctypes.POINTER(_f64)],
    "sem_rhs": [_vp, _vp, _vp],
    "sem_jac_vec": [_vp, _vp, _vp, _vp],
    "sem_jact_vec": [_vp, _vp, _vp, _vp],
    "sem_rk4_forward": [_vp, _vp, _f64, _i32, _i32, _vp],
    "sem_rk4_forward_noalloc": [_vp, _vp, _f64, _i32, _i32, _vp],
    "sem_mass": [_vp, _vp],
    "sem_batch_mass": [_vp, _vp],
    "sem_rk4_adjoint": [_vp, _vp, _f64, _i32, _i32, _vp, _vp],
    "sem_workspace_bytes": [_vp, _i32, ctypes.POINTER(_i64)],
    "sem_set_adjoint_stages": [_vp, _i32],
    "sem_set_check_finite": [_vp, _i32],
    "sem_last_error": [],
    "sem_batch_setup": [ctypes.POINTER(SemDesc), ctypes.POINTER(_f64), _i32, _vp, ctypes.POINTER(_vp)],
    "sem_batch_destroy": [_vp],
    "sem_batch_query": [_vp, ctypes.POINTER(_i64)],
    "sem_batch_rhs": [_vp, _vp, _vp],
    "sem_batch_jact_vec": [_vp, _vp, _vp, _vp],
    "sem_batch_rk4_forward": [_vp, _vp, _i32, _i32, _vp],
    "sem_batch_rk4_adjoint": [_vp, _vp, _i32, _i32, _vp, _vp],
    "sem_revolve_plan": [_i32, _i32, _vp, _vp, _i64, _vp],
    "sem_rk_forward_revolve": [_vp, _i32, _vp, _f64, _i32, _i32, _vp],
    "sem_rk_adjoint_revolve": [_vp, _i32, _vp, _f64, _i32, _i32, _vp, _vp],
    "sem_revolve_workspace_bytes": [_vp, _i32, _vp],
    "sem_cn_workspace_bytes": [_vp, _i32, _vp, _vp],
    "sem_cn_forward": [_vp, _vp, _f64, _i32, _i32, _vp, _vp, _vp, _vp],
    "sem_cn_adjoint": [_vp, _vp, _f64, _i32, _i32, _vp, _vp, _vp, _vp],
    "sem_lmvm_workspace_bytes": [_vp, _i32, _i32, _i32, _vp, _vp],
    "sem_lmvm_initial_condition": [_vp, _i32, _vp, _vp, _f64, _i32, _i32, _vp, _vp, _vp, _vp],
    "sem_line_search_step": [_vp, _vp, _vp, _f64, _f64],
    "sem_rk_forward": [_vp, _i32, _vp, _f64, _i32, _i32, _vp],
    "sem_rk_adjoint": [_vp, _i32, _vp, _f64, _i32, _i32, _vp, _vp],
    "sem_batch_rk_forward": [_vp, _i32, _vp, _i32, _i32, _vp],
    "sem_batch_rk_adjoint": [_vp, _i32, _vp, _i32, _i32, _vp, _vp],
    "sem_rk_stages_bytes": [_vp, _i32, _i32, ctypes.POINTER(_i64)],
    "sem_rk_forward_stored": [_vp, _i32, _vp, _f64, _i32, _vp],
    "sem_rk_adjoint_stored": [_vp, _i32, _vp, _f64, _i32, _vp],
    "sem_batch_rk_stages_bytes": [_vp, _i32, _i32, ctypes.POINTER(_i64)],
    "sem_batch_rk_forward_stored": [_vp, _i32, _vp, _i32, _vp],
    "sem_batch_rk_adjoint_stored": [_vp, _i32, _vp, _i32, _vp],
    "sem_batch_workspace_bytes": [_vp, _i32, ctypes.POINTER(_i64)],
    "sem_batch_set_adjoint_stages": [_vp, _i32],
    "sem_batch_configure": [_vp, _i32, _i32],
    "sem_batch_set_stream": [_vp, _vp],
    "sem_batch_autotune": [_vp, ctypes.POINTER(_f64)],
    "sem_probe_fp64_rates": [_vp, _i32, _vp],
}
EXPORTED = tuple(_SIGS)


def lib():
    """Load libsem.so (built in-tree by ``python -m paper_1806_01422_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SemError(f"{LIB_PATH} is not built; run `python -m paper_1806_01422_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "sem_last_error" else ctypes.c_int
        _lib = L
    return _lib


def _call(rc):
    if rc != 0:
        msg = lib().sem_last_error().decode()
        raise SemError(f"libsem status {rc}: {msg}")


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dtype_code(dtype):
    if dtype == torch.float64:
        return SEM_F64
    if dtype == torch.float32:
        return SEM_F32
    raise SemError(f"unsupported dtype {dtype}")


def _desc(dim, order, elems, length, nu, dtype, batch):
    elems = list(elems) + [1] * (3 - len(elems))
    length = list(length) + [1.0] * (3 - len(length))
    return SemDesc(int(dim), (ctypes.c_int32 * 3)(*[int(e) for e in elems[:3]]), int(order),
                   (ctypes.c_double * 3)(*[float(x) for x in length[:3]]), float(nu), _dtype_code(dtype),
                   int(batch))


def _ptr(t):
    return _vp(t.data_ptr())


class Context:
    """One SEM Burgers problem (or a same-shape batch of fields) on the current GPU."""

    def __init__(self, dim, order, elems, length, nu, dtype=torch.float64, batch=1):
        if not torch.cuda.is_available():
            raise SemError("no GPU available: libsem runs only on the GPU")
        self.dim, self.order, self.nu, self.dtype, self.batch = dim, order, float(nu), dtype, batch
        self.elems = tuple(int(e) for e in elems)
        self.length = tuple(float(x) for x in length)
        self._h = _vp()
        d = _desc(dim, order, elems, length, nu, dtype, batch)
        _call(lib().sem_setup(ctypes.byref(d), _stream(), ctypes.byref(self._h)))
        ndof, nodes = _i64(), _i64()
        _call(lib().sem_query(self._h, ctypes.byref(ndof), ctypes.byref(nodes)))
        self.ndof, self.nodes = ndof.value, nodes.value
        self.n = tuple(e * order for e in self.elems)
        self.shape = (batch, dim) + tuple(reversed(self.n))
        path = _i32()
        _call(lib().sem_query_path(self._h, ctypes.byref(path)))
        # 0: element + summation kernels, 2: tuned 2-D kernel (orders 3, 5, 7), 3: tuned 3-D kernel (order 7)
        self.path = path.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sem_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind(self):
        _call(lib().sem_set_stream(self._h, _stream()))

    def _chk(self, t, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise SemError(f"{name} must be a CUDA tensor")
        if t.dtype != self.dtype:
            raise SemError(f"{name} has dtype {t.dtype}, context uses {self.dtype}")
        if not t.is_contiguous():
            raise SemError(f"{name} must be contiguous")
        if t.numel() != self.batch * self.ndof:
            raise SemError(f"{name} has {t.numel()} values, expected {self.batch * self.ndof}")
        return t

    def empty(self):
        return torch.empty(self.shape, dtype=self.dtype, device="cuda")

    def node_coords(self, k):
        x = np.zeros(self.n[k])
        _call(lib().sem_node_coords(self._h, k, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return x

    def rhs(self, u, out=None):
        self._chk(u, "u")
        out = self.empty() if out is None else self._chk(out, "out")
        self._bind()
        _call(lib().sem_rhs(self._h, _ptr(u), _ptr(out)))
        return out

    def jac_vec(self, u, v, out=None):
        self._chk(u, "u"), self._chk(v, "v")
        out = self.empty() if out is None else self._chk(out, "out")
        self._bind()
        _call(lib().sem_jac_vec(self._h, _ptr(u), _ptr(v), _ptr(out)))
        return out

    def jact_vec(self, u, w, out=None):
        self._chk(u, "u"), self._chk(w, "w")
        out = self.empty() if out is None else self._chk(out, "out")
        self._bind()
        _call(lib().sem_jact_vec(self._h, _ptr(u), _ptr(w), _ptr(out)))
        return out

    def set_check_finite(self, on=True):
        _call(lib().sem_set_check_finite(self._h, 1 if on else 0))

    def rk4_forward(self, u0, dt, nsteps, ckpt_every=0, inplace=False):
        """Returns (u(T), checkpoints [nsteps/K][batch][C][...] or None)."""
        self._chk(u0, "u0")
        u = u0 if inplace else u0.clone()
        ck = None
        if ckpt_every:
            ck = torch.empty((nsteps // ckpt_every,) + self.shape, dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_rk4_forward(self._h, _ptr(u), float(dt), int(nsteps), int(ckpt_every),
                                    _ptr(ck) if ck is not None else None))
        return u, ck

    def mass(self, out=None):
        """The assembled diagonal GLL mass of every node, in every component of a field-shaped array."""
        out = self.empty() if out is None else out
        self._chk(out, "out")
        self._bind()
        _call(lib().sem_mass(self._h, _ptr(out)))
        return out

    def rk4_forward_noalloc(self, u, dt, nsteps, ckpt_every=0, ckpt=None):
        """sem_rk4_forward_noalloc: RK4 in place on u (u0 in, u(T) out) with the library allocating
        nothing; the caller passes u and, if ckpt_every, the checkpoint array
        [nsteps/K][batch][C][...].  Returns (u, ckpt)."""
        self._chk(u, "u")
        if ckpt_every and (ckpt is None or not ckpt.is_contiguous() or ckpt.dtype != self.dtype or
                           ckpt.numel() != (nsteps // ckpt_every) * self.batch * self.ndof):
            raise SemError("ckpt must be a contiguous [nsteps/K][batch][C][...] array of the context's dtype")
        self._bind()
        _call(lib().sem_rk4_forward_noalloc(self._h, _ptr(u), float(dt), int(nsteps), int(ckpt_every),
                                            _ptr(ckpt) if ckpt_every else None))
        return u, ckpt

    def workspace_bytes(self, ckpt_every):
        b = _i64()
        _call(lib().sem_workspace_bytes(self._h, int(ckpt_every), ctypes.byref(b)))
        return b.value

    def set_adjoint_stages(self, mode):
        """How the RK adjoints obtain stage states: "auto", "store" or "recompute"."""
        _call(lib().sem_set_adjoint_stages(self._h, ADJOINT_STAGES[mode]))

    def _adjoint_args(self, ckpt, nsteps, ckpt_every, lamT, work):
        self._chk(lamT, "lamT")
        if not ckpt.is_contiguous() or ckpt.dtype != self.dtype:
            raise SemError("ckpt must be a contiguous tensor of the context dtype")
        if ckpt.numel() != (nsteps // ckpt_every) * self.batch * self.ndof:
            raise SemError("ckpt has the wrong size")
        if work is None:
            nbytes = self.workspace_bytes(ckpt_every)
            work = torch.empty(nbytes // (8 if self.dtype == torch.float64 else 4), dtype=self.dtype, device="cuda")
        return lamT.clone(), work

    def rk4_adjoint(self, ckpt, dt, nsteps, ckpt_every, lamT, work=None):
        """lambda_0 = dPhi/du_0 from lambda_N = dPhi/du(T) (discrete RK4 adjoint)."""
        lam, work = self._adjoint_args(ckpt, nsteps, ckpt_every, lamT, work)
        self._bind()
        _call(lib().sem_rk4_adjoint(self._h, _ptr(ckpt), float(dt), int(nsteps), int(ckpt_every), _ptr(lam),
                                    _ptr(work)))
        return lam

    def rk_forward(self, u0, dt, nsteps, ckpt_every=0, scheme="rk4", inplace=False):
        """rk4_forward for any scheme ("rk4", "rk3")."""
        self._chk(u0, "u0")
        code = _scheme(scheme)
        u = u0 if inplace else u0.clone()
        ck = None
        if ckpt_every:
            ck = torch.empty((nsteps // ckpt_every,) + self.shape, dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_rk_forward(self._h, code, _ptr(u), float(dt), int(nsteps), int(ckpt_every),
                                   _ptr(ck) if ck is not None else None))
        return u, ck

    def rk_adjoint(self, ckpt, dt, nsteps, ckpt_every, lamT, scheme="rk4", work=None):
        """rk4_adjoint for any scheme ("rk4", "rk3")."""
        code = _scheme(scheme)
        lam, work = self._adjoint_args(ckpt, nsteps, ckpt_every, lamT, work)
        self._bind()
        _call(lib().sem_rk_adjoint(self._h, code, _ptr(ckpt), float(dt), int(nsteps), int(ckpt_every), _ptr(lam),
                                   _ptr(work)))
        return lam

    def stage_states(self, scheme="rk4"):
        """States stored per step by rk_forward_stored: u_k and the stage states."""
        return 4 if _scheme(scheme) == _scheme("rk4") else 3

    def rk_forward_stored(self, u0, dt, nsteps, scheme="rk4"):
        """(u(T), stages [nsteps][S][batch][C][...]): every step's state and stage states."""
        self._chk(u0, "u0")
        code = _scheme(scheme)
        u = u0.clone()
        st = torch.empty((nsteps, self.stage_states(scheme)) + self.shape, dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_rk_forward_stored(self._h, code, _ptr(u), float(dt), int(nsteps), _ptr(st)))
        return u, st

    def rk_adjoint_stored(self, stages, dt, nsteps, lamT, scheme="rk4"):
        """lambda_0 from lambda_N with the stage states stored by rk_forward_stored (J^T only)."""
        self._chk(lamT, "lamT")
        if not stages.is_contiguous() or stages.dtype != self.dtype or \
                stages.numel() != nsteps * self.stage_states(scheme) * self.batch * self.ndof:
            raise SemError("stages must be the contiguous array rk_forward_stored returned")
        lam = lamT.clone()
        self._bind()
        _call(lib().sem_rk_adjoint_stored(self._h, _scheme(scheme), _ptr(stages), float(dt), int(nsteps), _ptr(lam)))
        return lam


    def _nk(self, opts):
        o = NkOpts()
        for k, v in (opts or {}).items():
            setattr(o, k, v)
        return o

    def cn_workspace_bytes(self, ckpt_every, opts=None):
        b = _i64()
        _call(lib().sem_cn_workspace_bytes(self._h, int(ckpt_every), ctypes.byref(self._nk(opts)), ctypes.byref(b)))
        return b.value

    def _cn_work(self, ckpt_every, opts):
        nbytes = self.cn_workspace_bytes(max(int(ckpt_every), 1), opts)
        return torch.empty(nbytes // (8 if self.dtype == torch.float64 else 4), dtype=self.dtype, device="cuda")

    def cn_forward(self, u0, dt, nsteps, ckpt_every=0, opts=None, work=None):
        """Crank-Nicolson with Newton-Krylov steps: (u(T), checkpoints or None, stats dict)."""
        self._chk(u0, "u0")
        u = u0.clone()
        ck = None
        if ckpt_every:
            ck = torch.empty((nsteps // ckpt_every,) + self.shape, dtype=self.dtype, device="cuda")
        work = self._cn_work(ckpt_every, opts) if work is None else work
        st = NkStats()
        self._bind()
        _call(lib().sem_cn_forward(self._h, _ptr(u), float(dt), int(nsteps), int(ckpt_every),
                                   _ptr(ck) if ck is not None else None, ctypes.byref(self._nk(opts)), _ptr(work),
                                   ctypes.byref(st)))
        return u, ck, st.as_dict()

    def cn_adjoint(self, ckpt, dt, nsteps, ckpt_every, lamT, opts=None, work=None):
        """Discrete Crank-Nicolson adjoint: (lambda_0, stats dict)."""
        lam, _ = self._adjoint_args(ckpt, nsteps, ckpt_every, lamT, torch.empty(0, device="cuda"))
        work = self._cn_work(ckpt_every, opts) if work is None else work
        st = NkStats()
        self._bind()
        _call(lib().sem_cn_adjoint(self._h, _ptr(ckpt), float(dt), int(nsteps), int(ckpt_every), _ptr(lam),
                                   ctypes.byref(self._nk(opts)), _ptr(work), ctypes.byref(st)))
        return lam, st.as_dict()

    def lmvm_initial_condition(self, u0, target, dt, nsteps, ckpt_every, scheme="rk4", opts=None, work=None):
        """Minimise 1/2 ||u(T; u_0) - target||^2 over u_0 by LMVM with More-Thuente steps, starting
        from u0: (u_0 found, history of the objective per iteration, stats dict)."""
        self._chk(u0, "u0")
        self._chk(target, "target")
        if scheme not in _ALL_SCHEMES:
            raise SemError(f"unknown scheme {scheme!r}")
        o = LmvmOpts()
        for k, v in (opts or {}).items():
            setattr(o, k, v)
        if work is None:
            b = _i64()
            _call(lib().sem_lmvm_workspace_bytes(self._h, _ALL_SCHEMES[scheme], int(nsteps), int(ckpt_every),
                                                 ctypes.byref(o), ctypes.byref(b)))
            work = torch.empty(b.value // (8 if self.dtype == torch.float64 else 4), dtype=self.dtype, device="cuda")
        u = u0.clone()
        hist = (ctypes.c_double * ((o.max_iters or 50) + 1))()
        st = LmvmStats()
        self._bind()
        _call(lib().sem_lmvm_initial_condition(self._h, _ALL_SCHEMES[scheme], _ptr(u), _ptr(target), float(dt),
                                               int(nsteps), int(ckpt_every), ctypes.byref(o), _ptr(work), hist,
                                               ctypes.byref(st)))
        return u, list(hist[: st.iters + 1]), st.as_dict()

    def rk_forward_revolve(self, u0, dt, nsteps, snaps, scheme="rk4"):
        """(u(T), snapshots [snaps][batch][C][...]) for binomial checkpointing with snaps slots."""
        self._chk(u0, "u0")
        code = _scheme(scheme)
        u = u0.clone()
        ck = torch.empty((int(snaps),) + self.shape, dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_rk_forward_revolve(self._h, code, _ptr(u), float(dt), int(nsteps), int(snaps), _ptr(ck)))
        return u, ck

    def rk_adjoint_revolve(self, ckpt, dt, nsteps, snaps, lamT, scheme="rk4", work=None):
        """lambda_0 from lambda_N by the binomial schedule, from rk_forward_revolve's snapshots."""
        self._chk(lamT, "lamT")
        code = _scheme(scheme)
        if not ckpt.is_contiguous() or ckpt.dtype != self.dtype or ckpt.numel() != snaps * self.batch * self.ndof:
            raise SemError("ckpt must be the contiguous [snaps][batch][...] tensor of rk_forward_revolve")
        if work is None:
            b = _i64()
            _call(lib().sem_revolve_workspace_bytes(self._h, int(snaps), ctypes.byref(b)))
            work = torch.empty(b.value // (8 if self.dtype == torch.float64 else 4), dtype=self.dtype, device="cuda")
        lam = lamT.clone()
        self._bind()
        _call(lib().sem_rk_adjoint_revolve(self._h, code, _ptr(ckpt), float(dt), int(nsteps), int(snaps), _ptr(lam),
                                           _ptr(work)))
        return lam


def probe_fp64_rates(iters=2000):
    """FP64 TFLOP/s of the matrix cores and the vector units of the current GPU, alone and
    interleaved in one instruction stream (a diagnostic; see sem_probe_fp64_rates)."""
    out = (_f64 * 4)()
    _call(lib().sem_probe_fp64_rates(_stream(), int(iters), out))
    return {"mfma_alone": out[0], "valu_alone": out[1], "interleaved_mfma": out[2], "interleaved_valu": out[3],
            "interleaved_total": out[2] + out[3]}


def revolve_plan(nsteps, snaps):
    """The binomial checkpointing schedule: (list of (kind, arg) with kinds "restore", "advance",
    "store", "adjoint"; number of forward steps it advances).  Host only."""
    n, adv = _i64(), _i64()
    _call(lib().sem_revolve_plan(int(nsteps), int(snaps), ctypes.byref(n), None, 0, ctypes.byref(adv)))
    buf = (_i64 * (2 * n.value))()
    _call(lib().sem_revolve_plan(int(nsteps), int(snaps), ctypes.byref(n), buf, n.value, ctypes.byref(adv)))
    kinds = ("restore", "advance", "store", "adjoint")
    return [(kinds[buf[2 * k]], int(buf[2 * k + 1])) for k in range(n.value)], adv.value


class SEMRhs(torch.autograd.Function):
    """f = F(u) with backward u_bar = J(u)^T f_bar (Sec. 3.3, eq. jactransvec)."""

    @staticmethod
    def forward(ctx, u, sem):
        ctx.sem = sem
        ctx.save_for_backward(u)
        return sem.rhs(u.contiguous())

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        return ctx.sem.jact_vec(u.contiguous(), g.contiguous()), None


class SEMTrajectory(torch.autograd.Function):
    """u(T) = Phi_dt^nsteps(u_0) for a time integrator ("rk4", "rk3" or Crank-Nicolson "cn"), with
    backward by the discrete adjoint of that scheme (Sec. 4.1) from uniform checkpoints every
    ckpt_every steps, recomputed segment by segment (Sec. 5.3).

    stored_tail > 0 (Runge-Kutta only): the forward sweep keeps every stage state of its last
    stored_tail segments, so the backward runs their adjoint from those states (J^T only) and
    recomputes only the segments before them, at stored_tail * ckpt_every * S extra states."""

    @staticmethod
    def forward(ctx, u0, sem, dt, nsteps, ckpt_every, scheme="rk4", stored_tail=0):
        if scheme == "cn" and stored_tail:
            raise SemError("stored_tail applies to the Runge-Kutta schemes only; the Crank-Nicolson "
                           "adjoint always recomputes from its checkpoints")
        n_tail = stored_tail * ckpt_every
        if n_tail < 0 or n_tail > nsteps:
            raise SemError(f"stored_tail * ckpt_every = {n_tail} must lie in [0, nsteps = {nsteps}]")
        n_head = nsteps - n_tail
        st = None
        if scheme == "cn":
            uT, ck, _ = sem.cn_forward(u0.contiguous(), dt, nsteps, ckpt_every)
        else:
            uT, ck = u0.contiguous(), None
            if n_head or not n_tail:
                uT, ck = sem.rk_forward(uT, dt, n_head, ckpt_every, scheme=scheme)
            if n_tail:
                uT, st = sem.rk_forward_stored(uT, dt, n_tail, scheme=scheme)
        ctx.sem, ctx.dt, ctx.K, ctx.scheme = sem, dt, ckpt_every, scheme
        ctx.n_head, ctx.n_tail = n_head, n_tail
        ctx.save_for_backward(ck, st)
        return uT

    @staticmethod
    def backward(ctx, g):
        ck, st = ctx.saved_tensors
        if ctx.scheme == "cn":
            lam0, _ = ctx.sem.cn_adjoint(ck, ctx.dt, ctx.n_head, ctx.K, g.contiguous())
        else:
            lam0 = g.contiguous()
            if ctx.n_tail:
                lam0 = ctx.sem.rk_adjoint_stored(st, ctx.dt, ctx.n_tail, lam0, scheme=ctx.scheme)
            if ctx.n_head or not ctx.n_tail:
                lam0 = ctx.sem.rk_adjoint(ck, ctx.dt, ctx.n_head, ctx.K, lam0, scheme=ctx.scheme)
        return lam0, None, None, None, None, None, None


def trajectory(u0, sem, dt, nsteps, ckpt_every, scheme="rk4", stored_tail=0):
    return SEMTrajectory.apply(u0, sem, dt, nsteps, ckpt_every, scheme, stored_tail)


class SEMTrajectoryRevolve(torch.autograd.Function):
    """SEMTrajectory with binomial (revolve) checkpointing in `snaps` state slots."""

    @staticmethod
    def forward(ctx, u0, sem, dt, nsteps, snaps, scheme="rk4"):
        uT, ck = sem.rk_forward_revolve(u0.contiguous(), dt, nsteps, snaps, scheme=scheme)
        ctx.sem, ctx.dt, ctx.nsteps, ctx.snaps, ctx.scheme = sem, dt, nsteps, snaps, scheme
        ctx.save_for_backward(ck)
        return uT

    @staticmethod
    def backward(ctx, g):
        (ck,) = ctx.saved_tensors
        lam0 = ctx.sem.rk_adjoint_revolve(ck, ctx.dt, ctx.nsteps, ctx.snaps, g.contiguous(), scheme=ctx.scheme)
        return lam0, None, None, None, None, None


def trajectory_revolve(u0, sem, dt, nsteps, snaps, scheme="rk4"):
    return SEMTrajectoryRevolve.apply(u0, sem, dt, nsteps, snaps, scheme)


class SEMTrajectoryStored(torch.autograd.Function):
    """SEMTrajectory with every stage state stored by the forward sweep: the backward applies only
    the J^T products (no recompute), at nsteps * S states of memory."""

    @staticmethod
    def forward(ctx, u0, sem, dt, nsteps, scheme="rk4"):
        uT, st = sem.rk_forward_stored(u0.contiguous(), dt, nsteps, scheme=scheme)
        ctx.sem, ctx.dt, ctx.nsteps, ctx.scheme = sem, dt, nsteps, scheme
        ctx.save_for_backward(st)
        return uT

    @staticmethod
    def backward(ctx, g):
        (st,) = ctx.saved_tensors
        lam0 = ctx.sem.rk_adjoint_stored(st, ctx.dt, ctx.nsteps, g.contiguous(), scheme=ctx.scheme)
        return lam0, None, None, None, None


def trajectory_stored(u0, sem, dt, nsteps, scheme="rk4"):
    return SEMTrajectoryStored.apply(u0, sem, dt, nsteps, scheme)


class Batch:
    """Independent 2-D (or 1-D/3-D, shared dim) problems of uneven size/order packed back to back."""

    def __init__(self, problems, dtype=torch.float64):
        """problems: list of dicts with keys dim, order, elems, length, nu, dt."""
        if not torch.cuda.is_available():
            raise SemError("no GPU available: libsem runs only on the GPU")
        self.problems = list(problems)
        self.dtype = dtype
        n = len(self.problems)
        descs = (SemDesc * n)(*[_desc(p["dim"], p["order"], p["elems"], p["length"], p["nu"], dtype, 1)
                                for p in self.problems])
        dts = (ctypes.c_double * n)(*[float(p["dt"]) for p in self.problems])
        self._h = _vp()
        _call(lib().sem_batch_setup(descs, dts, n, _stream(), ctypes.byref(self._h)))
        offs = (ctypes.c_int64 * (n + 1))()
        _call(lib().sem_batch_query(self._h, offs))
        self.offsets = [int(o) for o in offs]
        self.total = self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sem_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        return torch.empty(self.total, dtype=self.dtype, device="cuda")

    def view(self, packed, p):
        """Problem p's field [1][C][...] as a view of the packed array."""
        q = self.problems[p]
        n = [e * q["order"] for e in q["elems"]]
        return packed[self.offsets[p]:self.offsets[p + 1]].view((1, q["dim"]) + tuple(reversed(n)))

    def _bind(self):
        _call(lib().sem_batch_set_stream(self._h, _stream()))

    def _chk(self, t, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous():
            raise SemError(f"{name} must be a contiguous CUDA tensor of dtype {self.dtype}")
        if t.numel() != self.total:
            raise SemError(f"{name} has {t.numel()} values, expected {self.total}")
        return t

    def mass(self, out=None):
        """The assembled diagonal mass of every problem on a packed array (as Context.mass)."""
        out = self.empty() if out is None else self._chk(out, "out")
        self._bind()
        _call(lib().sem_batch_mass(self._h, _ptr(out)))
        return out

    def rhs(self, u, out=None):
        self._chk(u, "u")
        out = self.empty() if out is None else self._chk(out, "out")
        self._bind()
        _call(lib().sem_batch_rhs(self._h, _ptr(u), _ptr(out)))
        return out

    def jact_vec(self, u, w, out=None):
        self._chk(u, "u"), self._chk(w, "w")
        out = self.empty() if out is None else self._chk(out, "out")
        self._bind()
        _call(lib().sem_batch_jact_vec(self._h, _ptr(u), _ptr(w), _ptr(out)))
        return out

    def rk4_forward(self, u0, nsteps, ckpt_every=0):
        self._chk(u0, "u0")
        u = u0.clone()
        ck = None
        if ckpt_every:
            ck = torch.empty((nsteps // ckpt_every, self.total), dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_batch_rk4_forward(self._h, _ptr(u), int(nsteps), int(ckpt_every),
                                          _ptr(ck) if ck is not None else None))
        return u, ck

    def set_adjoint_stages(self, mode):
        """How the RK adjoints obtain stage states: "auto", "store" or "recompute"."""
        _call(lib().sem_batch_set_adjoint_stages(self._h, ADJOINT_STAGES[mode]))

    def _work(self, ckpt_every, work):
        if work is None:
            b = _i64()
            _call(lib().sem_batch_workspace_bytes(self._h, int(ckpt_every), ctypes.byref(b)))
            work = torch.empty(b.value // (8 if self.dtype == torch.float64 else 4), dtype=self.dtype, device="cuda")
        return work

    def rk4_adjoint(self, ckpt, nsteps, ckpt_every, lamT, work=None):
        self._chk(lamT, "lamT")
        lam = lamT.clone()
        work = self._work(ckpt_every, work)
        self._bind()
        _call(lib().sem_batch_rk4_adjoint(self._h, _ptr(ckpt), int(nsteps), int(ckpt_every), _ptr(lam), _ptr(work)))
        return lam

    def rk_forward(self, u0, nsteps, ckpt_every=0, scheme="rk4"):
        self._chk(u0, "u0")
        code = _scheme(scheme)
        u = u0.clone()
        ck = None
        if ckpt_every:
            ck = torch.empty((nsteps // ckpt_every, self.total), dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_batch_rk_forward(self._h, code, _ptr(u), int(nsteps), int(ckpt_every),
                                         _ptr(ck) if ck is not None else None))
        return u, ck

    def rk_adjoint(self, ckpt, nsteps, ckpt_every, lamT, scheme="rk4", work=None):
        self._chk(lamT, "lamT")
        code = _scheme(scheme)
        lam = lamT.clone()
        work = self._work(ckpt_every, work)
        self._bind()
        _call(lib().sem_batch_rk_adjoint(self._h, code, _ptr(ckpt), int(nsteps), int(ckpt_every), _ptr(lam),
                                         _ptr(work)))
        return lam

    def rk_forward_stored(self, u0, nsteps, scheme="rk4"):
        """(u(T), stages [nsteps][S][total]) as Context.rk_forward_stored, each problem with its dt."""
        self._chk(u0, "u0")
        code = _scheme(scheme)
        u = u0.clone()
        S = 4 if code == _scheme("rk4") else 3
        st = torch.empty((nsteps, S, self.total), dtype=self.dtype, device="cuda")
        self._bind()
        _call(lib().sem_batch_rk_forward_stored(self._h, code, _ptr(u), int(nsteps), _ptr(st)))
        return u, st

    def rk_adjoint_stored(self, stages, nsteps, lamT, scheme="rk4"):
        self._chk(lamT, "lamT")
        code = _scheme(scheme)
        S = 4 if code == _scheme("rk4") else 3
        if not stages.is_contiguous() or stages.dtype != self.dtype or stages.numel() != nsteps * S * self.total:
            raise SemError("stages must be the contiguous array rk_forward_stored returned")
        lam = lamT.clone()
        self._bind()
        _call(lib().sem_batch_rk_adjoint_stored(self._h, code, _ptr(stages), int(nsteps), _ptr(lam)))
        return lam

    def configure(self, persistent, param=0):
        """persistent=True: one persistent launch with `param` workgroups; False: one launch per
        order class with `param` elements per workgroup (0 = default)."""
        _call(lib().sem_batch_configure(self._h, 1 if persistent else 0, int(param)))

    def autotune(self):
        """Time the candidate launch shapes on one RK4 step and keep the fastest; returns its ms."""
        ms = _f64()
        self._bind()
        _call(lib().sem_batch_autotune(self._h, ctypes.byref(ms)))
        return ms.value
