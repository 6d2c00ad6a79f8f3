"""GPU parity: libsem (HIP, through its C ABI) against the CPU oracle, element by element.

Tolerances: FP64 per operator application <= 1e-12 and after a trajectory <= 1e-10, both measured
norm-wise as max|x - x_ref| / max|x_ref| (fields cross zero, so element-wise relative error is not
meaningful).  FP32 results are compared with the FP64 oracle at 1e-4 (rounding of 8-point
contractions in single precision, ~1e-6 expected).
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

sys.path.insert(0, os.path.dirname(__file__))

pytestmark = pytest.mark.gpu

TOL_APPLY = 1e-12
TOL_TRAJ = 1e-10


@pytest.fixture(scope="module")
def P():
    import paper_1806_01422_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = a.detach().cpu().double().numpy() if isinstance(a, torch.Tensor) else a
    b = b.detach().cpu().double().numpy() if isinstance(b, torch.Tensor) else b
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def make(P, dim, N, E, nu=0.01, batch=1, L=None, dtype=torch.float64):
    L = list(L or [1.0] * dim)
    m = oracle.Mesh(dim, N, list(E), L, nu, batch)
    c = P.Context(dim, N, list(E), L, nu, dtype=dtype, batch=batch)
    assert c.shape == m.shape
    return m, c


def fields(m, seed):
    xs = [m.coords(k) for k in range(m.dim)]
    u = np.stack([wl.fourier_field(xs, m.L[: m.dim], 3, seed + b) for b in range(m.batch)])
    v = wl.normal_field(m.shape, seed + 100)
    w = wl.normal_field(m.shape, seed + 200)
    return u, v, w


CASES = [
    (1, 8, [16]), (1, 1, [3]), (1, 12, [5]), (1, 3, [1]), (1, 5, [37]),
    (2, 7, [5, 3]), (2, 1, [2, 2]), (2, 2, [2, 2]), (2, 12, [3, 2]), (2, 5, [1, 4]), (2, 9, [7, 5]),
    (2, 6, [3, 3]),
    (3, 7, [3, 2, 4]), (3, 1, [2, 2, 2]), (3, 9, [2, 3, 2]), (3, 4, [1, 2, 3]), (3, 2, [5, 1, 1]),
    (3, 7, [1, 1, 1]), (3, 5, [3, 3, 3]),
    (3, 7, [1, 2, 2]), (3, 7, [5, 2, 6]), (3, 7, [2, 6, 4]),
    # order 7 with an x element count that is a multiple of 4 runs the tuned 3-D kernel
    (3, 7, [4, 1, 1]), (3, 7, [4, 2, 3]), (3, 7, [8, 3, 2]), (3, 7, [4, 5, 1]), (3, 7, [12, 1, 2]),
    (3, 7, [8, 2, 5]), (3, 7, [4, 4, 4]),
    # 8 workgroups per field and z-segment: the XCD-banded workgroup order is active
    (3, 7, [16, 2, 2]), (3, 7, [8, 4, 3]),
    # orders 3, 5, 7 with an x element count that is a multiple of 8 (at most 64) run the tuned
    # 2-D kernel: one or several wavefronts per workgroup, one element row, ragged row segments
    (2, 7, [8, 1]), (2, 7, [8, 2]), (2, 7, [8, 3]), (2, 7, [16, 5]), (2, 7, [24, 2]),
    (2, 5, [8, 1]), (2, 5, [16, 3]), (2, 5, [40, 2]), (2, 3, [8, 2]), (2, 3, [24, 5]), (2, 3, [64, 1]),
    # order 9 with an x element count that is a multiple of 4 runs the tuned 2-D kernel with 16
    # lanes per element, a whole row of up to 16 elements per workgroup (longer rows: see
    # test_tuned_2d_order9_segments)
    (2, 9, [4, 3]), (2, 9, [12, 5]), (2, 9, [16, 2]),
]

TUNED = {(2, 7, (8, 1)): 2, (2, 7, (64, 3)): 2, (3, 7, (4, 1, 1)): 3, (3, 7, (4, 4, 4)): 3, (2, 7, (5, 3)): 0,
         (2, 7, (72, 2)): 0, (2, 9, (8, 2)): 2, (2, 9, (64, 2)): 2, (2, 9, (6, 2)): 0, (2, 9, (20, 1)): 2, (3, 7, (3, 2, 4)): 0, (2, 5, (8, 2)): 2, (2, 3, (16, 1)): 2,
         (2, 4, (8, 2)): 0, (2, 6, (8, 2)): 0, (2, 1, (8, 2)): 0, (3, 5, (4, 1, 1)): 0}


@pytest.mark.parametrize("dim,N,E", CASES)
def test_operators_fp64(P, dim, N, E):
    note(f"operators fp64 dim={dim} N={N} E={E}")
    m, c = make(P, dim, N, E, nu=0.02)
    u, v, w = fields(m, 7)
    U, V, W = gpu(u), gpu(v), gpu(w)
    assert rel(c.rhs(U), m.rhs(u)) < TOL_APPLY
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < TOL_APPLY
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < TOL_APPLY


def test_kernel_path_selection(P):
    note("operator implementation chosen per shape")
    for (dim, N, E), path in TUNED.items():
        c = P.Context(dim, N, list(E), [1.0] * dim, 0.01)
        assert c.path == path, (dim, N, E, c.path)


# 3-D order 7 with E_x % 4 = 0 and at least 4 element layers: the FP32 F kernel sweeps z in two
# segments (the second one ragged for odd E_z), each recomputing the layer before it
@pytest.mark.parametrize("dim,N,E", [(1, 8, [16]), (2, 7, [5, 3]), (3, 7, [3, 2, 4]), (3, 5, [2, 2, 3]),
                                     (3, 7, [4, 2, 3]), (2, 7, [8, 3]), (2, 5, [8, 3]), (3, 7, [4, 1, 4]),
                                     (3, 7, [4, 2, 5]), (3, 7, [8, 1, 7]), (2, 9, [16, 3]), (2, 9, [32, 2])])
def test_operators_fp32(P, dim, N, E):
    note(f"operators fp32 dim={dim} N={N} E={E}")
    # order 9 on the unit square puts FP32's own rounding floor at 1e-4 and above for these rows
    # (tests/test_rounding_floor.py); stretched along x it is about 2e-5
    L = [E[0] / 4.0, 1.0] if N == 9 else None
    m, c = make(P, dim, N, E, nu=0.02, L=L, dtype=torch.float32)
    u, v, w = fields(m, 9)
    U, V, W = gpu(u, torch.float32), gpu(v, torch.float32), gpu(w, torch.float32)
    assert rel(c.rhs(U), m.rhs(u)) < 1e-4
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < 1e-4
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < 1e-4


@pytest.mark.parametrize("E", [[4, 1, 4], [4, 2, 5]])
def test_rk4_fp32_3d(P, E):
    # FP32 trajectories on the tuned 3-D kernels (z-segmented F with its epilogue variants, J^T)
    note(f"RK4 fp32 3-D E={E}")
    m, c = make(P, 3, 7, E, nu=0.01, dtype=torch.float32)
    u, _, w = fields(m, 23)
    dt, n, K = 2e-3, 6, 3
    uT_ref, ck_ref = m.rk4_forward(u, dt, n, K)
    uT, ck = c.rk4_forward(gpu(u, torch.float32), dt, n, K)
    assert rel(uT, uT_ref) < 1e-4
    lam = c.rk4_adjoint(ck, dt, n, K, gpu(w, torch.float32))
    assert rel(lam, m.rk4_adjoint(ck_ref, dt, n, K, w)) < 1e-4


@pytest.mark.parametrize("dim,N,E", [(1, 4, [4]), (2, 4, [4, 2]), (3, 4, [4, 2, 3]), (3, 7, [4, 2, 3])])
def test_batched_fields(P, dim, N, E):
    note(f"same-shape batch dim={dim} N={N} E={E}")
    m, c = make(P, dim, N, E, nu=0.03, batch=3)
    u, v, w = fields(m, 11)
    U, V, W = gpu(u), gpu(v), gpu(w)
    assert rel(c.rhs(U), m.rhs(u)) < TOL_APPLY
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < TOL_APPLY
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < TOL_APPLY


def test_batched_fields_fp32_segments(P):
    # FP32 3-D with E_z >= 4: the z-segmented F and J^T kernels over a same-shape batch
    note("same-shape batch fp32 3-D, z-segmented sweep")
    m, c = make(P, 3, 7, [4, 2, 5], nu=0.02, batch=2, dtype=torch.float32)
    u, v, w = fields(m, 13)
    U, V, W = gpu(u, torch.float32), gpu(v, torch.float32), gpu(w, torch.float32)
    assert rel(c.rhs(U), m.rhs(u)) < 1e-4
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < 1e-4
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < 1e-4


# Wide element rows (5 and 8 wavefronts per workgroup) on domains stretched along x, so that the
# elements stay near square.  On the unit square these meshes are so fine along x for nu = 0.02
# that the operator's FP64 rounding floor (the oracle against an extended-precision evaluation)
# exceeds the bound: 1.35e-12 for 40 x 7 elements, 6.6e-14 on [0, 5] x [0, 1], both measured by
# tests/test_rounding_floor.py::test_floor_of_wide_unit_square_rows.
@pytest.mark.parametrize("E,L", [([40, 7], [5.0, 1.0]), ([64, 3], [8.0, 0.5]), ([24, 2], [3.0, 0.5])])
def test_tuned_2d_wide_rows(P, E, L):
    note(f"tuned 2-D kernel, wide rows E={E} L={L}")
    m, c = make(P, 2, 7, E, nu=0.02, L=L)
    assert c.path == 2
    u, v, w = fields(m, 7)
    U, V, W = gpu(u), gpu(v), gpu(w)
    assert rel(c.rhs(U), m.rhs(u)) < TOL_APPLY
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < TOL_APPLY
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < TOL_APPLY


# Order 9 on rows longer than 16 elements: x-segments of one workgroup each whose left faces are
# completed in the kernel (2 and 4 segments of 16 elements, 5 segments of 4 for 20 elements), on
# domains stretched along x.  On the unit square the operator's FP64 rounding floor there is
# above the bound: 2.2e-12 for 32 x 3 and 9.1e-12 for 64 x 1 elements at nu = 0.02
# (tests/test_rounding_floor.py::test_floor_of_order9_wide_rows).
@pytest.mark.parametrize("E,L,batch", [([32, 3], [4.0, 1.0], 1), ([64, 1], [8.0, 1.0], 1), ([20, 2], [3.0, 1.0], 1),
                                       ([32, 3], [4.0, 1.0], 3)])
def test_tuned_2d_order9_segments(P, E, L, batch):
    note(f"tuned 2-D kernel, order 9, x-segments E={E} L={L} batch={batch}")
    m, c = make(P, 2, 9, E, nu=0.02, L=L, batch=batch)
    assert c.path == 2
    u, v, w = fields(m, 7)
    U, V, W = gpu(u), gpu(v), gpu(w)
    assert rel(c.rhs(U), m.rhs(u)) < TOL_APPLY
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < TOL_APPLY
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < TOL_APPLY


@pytest.mark.parametrize("E,L,batch", [([8, 3], [1.0, 1.0], 3), ([16, 32], [2.0, 4.0], 40)])
def test_tuned_2d_batched_segments(P, E, L, batch):
    # many batch members: longer row segments per workgroup (3 rows with a ragged last segment
    # for 32 rows x 40 members), checked against the oracle and against the generic kernels
    note(f"tuned 2-D kernel, batch={batch} E={E}")
    m, c = make(P, 2, 7, E, nu=0.02, batch=batch, L=L)
    assert c.path == 2
    u, v, w = fields(m, 31)
    U, V, W = gpu(u), gpu(v), gpu(w)
    f, jv, jt = c.rhs(U), c.jac_vec(U, V), c.jact_vec(U, W)
    assert rel(f, m.rhs(u)) < TOL_APPLY
    assert rel(jv, m.jac_vec(u, v)) < TOL_APPLY
    assert rel(jt, m.jact_vec(u, w)) < TOL_APPLY
    # the generic kernels through a one-problem batch (never tuned), member 0
    B = P.Batch([dict(dim=2, order=7, elems=tuple(E), length=tuple(L), nu=0.02, dt=1e-3)])
    ub, wb = B.empty(), B.empty()
    B.view(ub, 0).copy_(U[:1])
    B.view(wb, 0).copy_(W[:1])
    assert rel(f[:1], B.view(B.rhs(ub), 0)) < TOL_APPLY
    assert rel(jt[:1], B.view(B.jact_vec(ub, wb), 0)) < TOL_APPLY


def test_dot_identity_gpu(P):
    note("dot identity on the GPU, 3-D N=7")
    m, c = make(P, 3, 7, [4, 3, 2], nu=0.01)
    u, v, w = fields(m, 13)
    U, V, W = gpu(u), gpu(v), gpu(w)
    lhs = torch.dot(c.jac_vec(U, V).flatten(), W.flatten()).item()
    rhs = torch.dot(V.flatten(), c.jact_vec(U, W).flatten()).item()
    scale = (c.jac_vec(U, V).norm() * W.norm()).item()
    assert abs(lhs - rhs) < 1e-13 * scale


# ------------------------------------------------------------------------------------------------
# Full-size configurations (the shapes the benchmark times)
# ------------------------------------------------------------------------------------------------
def test_full_size_2d(P):
    cfg = wl.C2
    note("full-size 2-D 64x64 N=7 F, Jv, J^T")
    m, c = make(P, 2, cfg.N, cfg.E, nu=cfg.nu, L=cfg.L)
    xs = [m.coords(k) for k in range(2)]
    u = wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C2_SEEDS["u"])[None]
    v = wl.normal_field(m.shape, wl.C2_SEEDS["v"])
    w = wl.normal_field(m.shape, wl.C2_SEEDS["w"])
    U, V, W = gpu(u), gpu(v), gpu(w)
    assert rel(c.rhs(U), m.rhs(u)) < TOL_APPLY
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < TOL_APPLY
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < TOL_APPLY


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_size_3d(P, dtype):
    cfg = wl.C3
    note(f"full-size 3-D 32^3 N=7 F, Jv, J^T {dtype}")
    m = oracle.Mesh(3, cfg.N, list(cfg.E), list(cfg.L), cfg.nu)
    c = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu, dtype=dtype)
    xs = [m.coords(k) for k in range(3)]
    u = wl.fourier_field(xs, cfg.L, wl.C3_K, wl.C3_SEEDS["u"])[None]
    w = wl.normal_field(m.shape, wl.C3_SEEDS["w"])
    v = wl.normal_field(m.shape, wl.C3_SEEDS["v"])
    tol = TOL_APPLY if dtype == torch.float64 else 1e-4
    U, V, W = gpu(u, dtype), gpu(v, dtype), gpu(w, dtype)
    ef = rel(c.rhs(U), m.rhs(u))
    ej = rel(c.jact_vec(U, W), m.jact_vec(u, w))
    ev = rel(c.jac_vec(U, V), m.jac_vec(u, v))
    note(f"  errors F {ef:.3e}  J^T {ej:.3e}  Jv {ev:.3e}")
    assert ef < tol and ej < tol and ev < tol


def test_full_size_3d_trajectory(P):
    # the 32^3 N=7 field through the fused RK4 stage kernels (every epilogue variant of the tuned
    # 3-D kernel) and the discrete adjoint, at the benchmark's step size
    cfg = wl.C3
    note("full-size 3-D 32^3 N=7 FP64: 3 RK4 steps + adjoint (checkpointed and stored stages)")
    m = oracle.Mesh(3, cfg.N, list(cfg.E), list(cfg.L), cfg.nu)
    c = P.Context(3, cfg.N, cfg.E, cfg.L, cfg.nu)
    xs = [m.coords(k) for k in range(3)]
    u = wl.fourier_field(xs, cfg.L, wl.C3_K, wl.C3_SEEDS["u"])[None]
    w = wl.normal_field(m.shape, wl.C3_SEEDS["w"])
    dt, n, K = 1e-4, 3, 3
    uT, ck = c.rk4_forward(gpu(u), dt, n, K)
    lam = c.rk4_adjoint(ck, dt, n, K, gpu(w))
    uT_ref, ck_ref = m.rk4_forward(u, dt, n, K)
    lam_ref = m.rk4_adjoint(ck_ref, dt, n, K, w)
    eu, el = rel(uT, uT_ref), rel(lam, lam_ref)
    note(f"  errors u(T) {eu:.3e}  lambda_0 {el:.3e}")
    assert eu < TOL_TRAJ and el < TOL_TRAJ
    uS, st = c.rk_forward_stored(gpu(u), dt, n)
    assert torch.equal(uS, uT)
    c.set_adjoint_stages("store")
    assert torch.equal(c.rk_adjoint_stored(st, dt, n, gpu(w)), c.rk4_adjoint(ck, dt, n, K, gpu(w)))
    c.set_adjoint_stages("auto")


# ------------------------------------------------------------------------------------------------
# RK4 trajectories, adjoint and autograd
# ------------------------------------------------------------------------------------------------
def c1_inputs():
    m = oracle.Mesh(1, wl.C1.N, list(wl.C1.E), list(wl.C1.L), wl.C1.nu)
    x = m.coords(0)
    loc1 = wl.normal_field((1, m.nelem, 1, m.nloc), wl.C1_SEEDS["ic"])
    loc2 = wl.normal_field((1, m.nelem, 1, m.nloc), wl.C1_SEEDS["target"])
    u0 = np.sin(x)[None, None] + 0.01 * m.project_local(loc1)
    up = np.sin(x)[None, None] + 0.01 * m.project_local(loc2)
    target, _ = m.rk4_forward(up, wl.C1_DT, wl.C1_STEPS)
    return m, u0, target


def test_c1_trajectory_and_gradient(P):
    note("C1: 1-D RK4 100 steps, adjoint gradient, autograd")
    m, u0, target = c1_inputs()
    c = P.Context(1, wl.C1.N, wl.C1.E, wl.C1.L, wl.C1.nu)
    dt, n, K = wl.C1_DT, wl.C1_STEPS, 10
    uT_ref, _ = m.rk4_forward(u0, dt, n)
    uT, _ = c.rk4_forward(gpu(u0), dt, n)
    assert rel(uT, uT_ref) < TOL_TRAJ
    phi_ref, g_ref = m.gradient(u0, target, dt, n, K)
    x = gpu(u0).requires_grad_(True)
    yT = P.trajectory(x, c, dt, n, K)
    loss = 0.5 * ((yT - gpu(target)) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - phi_ref[0]) < 1e-12 * abs(phi_ref[0])
    assert rel(x.grad, g_ref) < TOL_TRAJ
    # central finite differences of the GPU trajectory on 16 random directions
    def Phi(uu):
        yy, _ = c.rk4_forward(gpu(uu), dt, n)
        return 0.5 * ((yy - gpu(target)) ** 2).sum().item()
    g = x.grad.cpu().numpy()
    for s in range(16):
        d = wl.normal_field(m.shape, 300 + s)
        eps = 1e-4 * np.linalg.norm(u0) / np.linalg.norm(d)
        fd = (8 * (Phi(u0 + eps * d) - Phi(u0 - eps * d)) - (Phi(u0 + 2 * eps * d) - Phi(u0 - 2 * eps * d))) / (
            12 * eps)
        ad = float(np.vdot(g, d))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (s, fd, ad)


@pytest.mark.parametrize("scheme", ["rk4", "rk3"])
@pytest.mark.parametrize("N", [7, 9])
def test_trajectory_stored_tail(P, scheme, N):
    # the last stored_tail segments keep their stage states in the forward sweep: the same values
    # as the checkpointed sweep (the same launches on the same states), and the oracle's gradient
    # (order 9 runs the tuned 2-D kernel with compile-time coefficients, at a 4x smaller step)
    note(f"trajectory with stored tail segments ({scheme}), 2-D 8x3 N={N}, batch 2")
    m, c = make(P, 2, N, [8, 3], nu=0.01, batch=2)
    u, _, w = fields(m, 23)
    dt, n, K = (2e-3 if N == 7 else 5e-4), 20, 5
    ref = None
    for tail in (0, 1, 3, 4):
        x = gpu(u).requires_grad_(True)
        yT = P.trajectory(x, c, dt, n, K, scheme=scheme, stored_tail=tail)
        (yT * gpu(w)).sum().backward()
        if ref is None:
            ref = (yT.detach().clone(), x.grad.clone())
            if scheme == "rk4":
                uT_ref, ck_ref = m.rk4_forward(u, dt, n, K)
                assert rel(yT, uT_ref) < TOL_TRAJ
                assert rel(x.grad, m.rk4_adjoint(ck_ref, dt, n, K, w)) < TOL_TRAJ
        else:
            assert torch.equal(yT, ref[0]) and torch.equal(x.grad, ref[1]), tail
    with pytest.raises(P.SemError):
        P.trajectory(gpu(u).requires_grad_(True), c, dt, n, K, scheme=scheme, stored_tail=5)
    # the Crank-Nicolson adjoint has no stored-stage form: a tail is an error, not ignored
    with pytest.raises(P.SemError):
        P.trajectory(gpu(u).requires_grad_(True), c, dt, n, K, scheme="cn", stored_tail=1)


@pytest.mark.parametrize("dim,N,E,batch", [(2, 5, [4, 3], 2), (3, 4, [2, 2, 3], 1), (2, 7, [3, 3], 1),
                                           (3, 7, [3, 2, 4], 1), (3, 7, [4, 2, 3], 1), (3, 7, [4, 1, 2], 2),
                                           (2, 7, [8, 3], 2), (2, 7, [8, 1], 1), (2, 5, [8, 2], 2),
                                           (2, 9, [32, 2], 2), (2, 9, [8, 3], 1), (3, 7, [8, 2, 3], 1),
                                           (3, 7, [12, 2, 2], 2)])
def test_rk4_forward_adjoint(P, dim, N, E, batch):
    note(f"RK4 forward/adjoint dim={dim} N={N} E={E} batch={batch}")
    # order 9 takes a 4x smaller step (RK4 at 2e-3 is unstable there: the oracle diverges) and the
    # 32-element rows a domain stretched along x; 3-D rows of more than 8 elements keep h_x = 1/4
    # (on the unit cube the 12-element row's oracle trajectory grows past 400 within 20 steps)
    L = [E[0] / 8.0, 1.0] if N == 9 and E[0] > 16 else [E[0] / 4.0, 1.0, 1.0] if dim == 3 and E[0] > 8 else None
    m, c = make(P, dim, N, E, nu=0.01, batch=batch, L=L)
    u, _, w = fields(m, 17)
    dt, n, K = (5e-4 if N == 9 else 2e-3), 20, 5
    uT_ref, ck_ref = m.rk4_forward(u, dt, n, K)
    assert np.isfinite(uT_ref).all()
    uT, ck = c.rk4_forward(gpu(u), dt, n, K)
    assert rel(uT, uT_ref) < TOL_TRAJ
    assert rel(ck, ck_ref) < TOL_TRAJ
    lam_ref = m.rk4_adjoint(ck_ref, dt, n, K, w)
    lam = c.rk4_adjoint(ck, dt, n, K, gpu(w))
    assert rel(lam, lam_ref) < TOL_TRAJ


@pytest.mark.parametrize("scheme", ["rk4", "rk3"])
@pytest.mark.parametrize("dim,N,E,batch", [(2, 7, [8, 3], 2), (3, 7, [4, 2, 3], 1), (2, 5, [4, 3], 2), (1, 8, [16], 1)])
def test_adjoint_stage_modes(P, scheme, dim, N, E, batch):
    # stage states stored by the segment recompute (uncaptured launches) or recomputed in every
    # adjoint step (captured graphs): the same launches on the same states, so the same values
    note(f"adjoint stage modes {scheme} dim={dim} N={N} E={E} batch={batch}")
    m, c = make(P, dim, N, E, nu=0.01, batch=batch)
    u, _, w = fields(m, 37)
    dt, n, K = (2e-3 if dim > 1 else 2e-4), 12, 4
    uT, ck = c.rk_forward(gpu(u), dt, n, K, scheme=scheme)
    c.set_adjoint_stages("recompute")
    wr = c.workspace_bytes(K)
    lam_r = c.rk_adjoint(ck, dt, n, K, gpu(w), scheme=scheme)
    c.set_adjoint_stages("store")
    assert c.workspace_bytes(K) == 4 * wr
    lam_s = c.rk_adjoint(ck, dt, n, K, gpu(w), scheme=scheme)
    assert torch.equal(lam_s, lam_r)
    ref, ckr = m.erk_forward(scheme, u, dt, n, K)
    assert rel(lam_s, m.erk_adjoint(scheme, ckr, dt, n, K, w)) < TOL_TRAJ
    c.set_adjoint_stages("auto")
    assert c.workspace_bytes(K) == wr  # these states are small: recompute by default


@pytest.mark.parametrize("scheme", ["rk4", "rk3"])
@pytest.mark.parametrize("dim,N,E,batch", [(1, 8, [16], 1), (2, 7, [8, 3], 2), (2, 5, [4, 3], 1), (3, 7, [4, 1, 2], 1),
                                           (3, 5, [2, 2, 2], 1)])
def test_stored_stages(P, scheme, dim, N, E, batch):
    # every stage stored by the forward sweep: the same states as the checkpointed forward (bitwise),
    # and the J^T-only adjoint equals the adjoint with stage states stored per segment (bitwise)
    note(f"stored stages {scheme} dim={dim} N={N} E={E} batch={batch}")
    m, c = make(P, dim, N, E, nu=0.01, batch=batch)
    u, _, w = fields(m, 41)
    dt, n, K = (2e-3 if dim > 1 else 2e-4), 8, 2
    U, W = gpu(u), gpu(w)
    uT, st = c.rk_forward_stored(U, dt, n, scheme=scheme)
    uT1, ck = c.rk_forward(U, dt, n, K, scheme=scheme)
    assert st.shape == (n, c.stage_states(scheme)) + c.shape
    assert torch.equal(uT, uT1)
    for j in range(n // K):
        assert torch.equal(st[j * K, 0], ck[j])
    lam = c.rk_adjoint_stored(st, dt, n, W, scheme=scheme)
    c.set_adjoint_stages("store")
    lam1 = c.rk_adjoint(ck, dt, n, K, W, scheme=scheme)
    c.set_adjoint_stages("auto")
    assert torch.equal(lam, lam1)
    uT_ref, ck_ref = m.erk_forward(scheme, u, dt, n, K)
    assert rel(uT, uT_ref) < TOL_TRAJ
    assert rel(lam, m.erk_adjoint(scheme, ck_ref, dt, n, K, w)) < TOL_TRAJ
    # through autograd
    u0 = U.clone().requires_grad_()
    (0.5 * P.trajectory_stored(u0, c, dt, n, scheme).pow(2).sum()).backward()
    assert rel(u0.grad, m.erk_adjoint(scheme, ck_ref, dt, n, K, uT_ref)) < TOL_TRAJ


def test_stored_stages_batch_and_errors(P):
    note("stored stages: batched set, zero steps, argument errors")
    specs, probs = batch_problems(12)
    B = P.Batch(specs)
    x = gpu(wl.normal_field((B.total,), 3)) * 0.01
    lamT = gpu(wl.normal_field((B.total,), 4))
    for scheme in ("rk4", "rk3"):
        uT, st = B.rk_forward_stored(x, 6, scheme=scheme)
        uT1, ck = B.rk_forward(x, 6, 3, scheme=scheme)
        assert torch.equal(uT, uT1)
        B.set_adjoint_stages("store")
        assert torch.equal(B.rk_adjoint_stored(st, 6, lamT, scheme=scheme), B.rk_adjoint(ck, 6, 3, lamT, scheme=scheme))
        B.set_adjoint_stages("auto")
        uT0, st0 = B.rk_forward_stored(x, 0, scheme=scheme)
        assert torch.equal(uT0, x) and st0.numel() == 0
        assert torch.equal(B.rk_adjoint_stored(st0, 0, lamT, scheme=scheme), lamT)
    m, c = make(P, 2, 3, [2, 2])
    u = torch.zeros(c.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError):
        c.rk_forward_stored(u, -1.0, 2)
    with pytest.raises(P.SemError):
        c.rk_forward_stored(u, 1e-3, 2, scheme="cn")  # implicit scheme: no stage states
    _, st = c.rk_forward_stored(u, 1e-3, 2)
    with pytest.raises(P.SemError):
        c.rk_adjoint_stored(st, 1e-3, 3, u)  # stage array of another length
    with pytest.raises(P.SemError):
        P.sem._call(P.lib().sem_rk_adjoint_stored(c._h, 0, P.sem._ptr(st), 1e-3, 2, P.sem._ptr(st)))  # aliasing
    with pytest.raises(P.SemError):  # lam inside the stage states (updated in place, so refused)
        P.sem._call(P.lib().sem_rk_adjoint_stored(c._h, 0, P.sem._ptr(st), 1e-3, 2, P.sem._ptr(st.view(-1)[7:])))
    # the checkpointed adjoint that stores stage states also updates lam in place
    c.set_adjoint_stages("store")
    _, ck = c.rk_forward(u, 1e-3, 2, 1)
    wk = torch.empty(c.workspace_bytes(1) // 8, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError):  # lam inside the work buffer
        P.sem._call(P.lib().sem_rk_adjoint(c._h, 0, P.sem._ptr(ck), 1e-3, 2, 1, P.sem._ptr(wk.view(-1)[3:]),
                                           P.sem._ptr(wk)))
    with pytest.raises(P.SemError):  # lam inside the checkpoints
        P.sem._call(P.lib().sem_rk_adjoint(c._h, 0, P.sem._ptr(ck), 1e-3, 2, 1, P.sem._ptr(ck.view(-1)[3:]),
                                           P.sem._ptr(wk)))
    c.set_adjoint_stages("auto")


@pytest.mark.parametrize("dim,N,E,batch", [(1, 8, [16], 2), (2, 7, [8, 3], 1), (2, 9, [5, 4], 2), (3, 7, [4, 2, 3], 1),
                                           (3, 4, [2, 3, 2], 2)])
def test_mass_matches_oracle(P, dim, N, E, batch):
    note(f"assembled mass dim={dim} N={N} E={E} batch={batch}")
    m, c = make(P, dim, N, E, batch=batch)
    ref = np.broadcast_to(m.mass(), m.shape)
    assert rel(c.mass(), ref) < 4e-15  # a product of three factors, rounded in either order


def test_batch_mass_matches_contexts(P):
    specs, _ = batch_problems(12)
    B = P.Batch(specs)
    mb = B.mass()
    for i, s in enumerate(specs):
        c = P.Context(2, s["order"], s["elems"], s["length"], s["nu"])
        assert torch.equal(B.view(mb, i), c.mass()), i
        c.close()
    B.close()


def test_c4_shape_batch_gradient(P):
    # the 64-IC 2-D configuration at full mesh size; a 50-step horizon keeps the oracle side short.
    cfg = wl.C4
    note("C4 shape: 64 ICs on 64x64 N=7, 50 steps, K=10 (oracle on ICs 0 and 63)")
    dt, n, K = wl.C4_DT, 50, 10
    c = P.Context(2, cfg.N, cfg.E, cfg.L, cfg.nu, batch=cfg.batch)
    m1 = oracle.Mesh(2, cfg.N, list(cfg.E), list(cfg.L), cfg.nu, 1)
    xs = [m1.coords(k) for k in range(2)]
    u0 = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_IC_SEED0 + b) for b in range(cfg.batch)])
    tg = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_TARGET_SEED0 + b) for b in range(cfg.batch)])
    x = gpu(u0).requires_grad_(True)
    yT = P.trajectory(x, c, dt, n, K)
    loss = 0.5 * ((yT - gpu(tg)) ** 2).sum()
    loss.backward()
    for b in (0, cfg.batch - 1):
        phi, g = m1.gradient(u0[b:b + 1], tg[b:b + 1], dt, n, K)
        assert rel(x.grad[b:b + 1], g) < TOL_TRAJ, b
    # central finite differences of the whole-batch misfit along 16 seeded directions
    note("  C4 shape: 16-direction central FD of the misfit")
    U0, TG = gpu(u0), gpu(tg)

    def phi_at(v):
        yT, _ = c.rk4_forward(v, dt, n)
        return float(0.5 * ((yT - TG) ** 2).sum())

    eps = 1e-4
    worst = 0.0
    for j in range(16):
        d = gpu(wl.normal_field(u0.shape, wl.C4_FD_SEED0 + j))
        fd = (phi_at(U0 + eps * d) - phi_at(U0 - eps * d)) / (2 * eps)
        ad = float((x.grad * d).sum())
        worst = max(worst, abs(fd - ad) / abs(ad))
    note(f"  worst relative FD error {worst:.2e}")
    assert worst < 1e-6


def c4_inputs(P):
    cfg = wl.C4
    c = P.Context(2, cfg.N, cfg.E, cfg.L, cfg.nu, batch=cfg.batch)
    m1 = oracle.Mesh(2, cfg.N, list(cfg.E), list(cfg.L), cfg.nu, 1)
    xs = [m1.coords(k) for k in range(2)]
    u0 = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_IC_SEED0 + b) for b in range(cfg.batch)])
    tg = np.stack([wl.fourier_field(xs, cfg.L, wl.C2_K, wl.C4_TARGET_SEED0 + b) for b in range(cfg.batch)])
    return c, m1, u0, tg


def c4_gradient(P, c, u0, tg, n, K, stored_tail=0):
    x = gpu(u0).requires_grad_(True)
    yT = P.trajectory(x, c, wl.C4_DT, n, K, stored_tail=stored_tail)
    loss = 0.5 * ((yT - gpu(tg)) ** 2).sum()
    loss.backward()
    return float(loss), x.grad


def test_c4_full_horizon_gradient(P):
    # the 64-IC gradient exactly as configured (500 RK4 steps of 2e-4, a checkpoint every 50):
    # against the oracle's gradient on ICs 0 and 63, and with the last segments' stage states kept
    # by the forward sweep (as many as the benchmark keeps) bitwise equal to the plain one
    cfg, n, K = wl.C4, wl.C4_STEPS, wl.C4_CKPT
    note(f"C4 as configured: 64 ICs on 64x64 N=7, {n} steps, K={K}")
    c, m1, u0, tg = c4_inputs(P)
    loss, g = c4_gradient(P, c, u0, tg, n, K)
    for b in (0, cfg.batch - 1):
        phi, gref = m1.gradient(u0[b:b + 1], tg[b:b + 1], wl.C4_DT, n, K)
        e = rel(g[b:b + 1], gref)
        note(f"  IC {b}: lambda_0 vs oracle {e:.2e}")
        assert e < TOL_TRAJ, b
    # one stored segment is 50 steps x 4 stage states x 64 fields x 401,408 values x 8 B = 41.1 GB
    seg = K * 4 * 8 * c.ndof * cfg.batch
    torch.cuda.empty_cache()
    tail = int(max(1, min(n // K, (torch.cuda.mem_get_info()[0] - (80 << 30)) // seg)))
    note(f"  stored tail of {tail} segments ({tail * seg / 1e9:.1f} GB)")
    loss_t, g_t = c4_gradient(P, c, u0, tg, n, K, stored_tail=tail)
    assert loss_t == loss and torch.equal(g_t, g)
    c.close()


def test_c4_full_horizon_finite_differences(P):
    # central finite differences of the whole-batch misfit along 16 seeded directions at the
    # configured horizon (Sec. 4.1 gradient; the paper's consistency check of the adjoint)
    n, K = wl.C4_STEPS, wl.C4_CKPT
    note(f"C4 as configured: 16-direction central FD of the 64-IC misfit over {n} steps")
    c, _, u0, tg = c4_inputs(P)
    _, g = c4_gradient(P, c, u0, tg, n, K)
    U0, TG = gpu(u0), gpu(tg)

    def phi_at(v):
        yT, _ = c.rk4_forward(v, wl.C4_DT, n)
        return float(0.5 * ((yT - TG) ** 2).sum())

    eps = 1e-4
    worst = 0.0
    for j in range(16):
        d = gpu(wl.normal_field(u0.shape, wl.C4_FD_SEED0 + j))
        fd = (phi_at(U0 + eps * d) - phi_at(U0 - eps * d)) / (2 * eps)
        ad = float((g * d).sum())
        worst = max(worst, abs(fd - ad) / abs(ad))
    note(f"  worst relative FD error {worst:.2e}")
    assert worst < 1e-6
    c.close()


# ------------------------------------------------------------------------------------------------
# Batched uneven problems
# ------------------------------------------------------------------------------------------------
def batch_problems(count):
    probs = wl.c5_problems(count)
    return [dict(dim=2, order=p.N, elems=(p.E, p.E), length=(1.0, 1.0), nu=p.nu, dt=p.dt) for p in probs], probs


def mixed_batch_specs(count):
    # the batched set's recipe (all of it on the tuned 2-D kernel) plus problems that run the
    # generic element and summation kernels (other orders and x element counts), so that the
    # persistent launch has work
    specs, _ = batch_problems(count)
    extra = [(6, (6, 5)), (8, (8, 8)), (4, (10, 6)), (9, (6, 6)), (7, (12, 4))]
    for i, (N, E) in enumerate(extra):
        nu = 10.0 ** (-2.5 - 0.3 * i)
        specs.append(dict(dim=2, order=N, elems=E, length=(1.0, 1.0), nu=nu,
                          dt=min(wl.stable_dt(2, N, max(E), 1.0, nu), wl.C5_T_MAX / wl.C5_STEPS)))
    return specs


def test_batch_operators_match_single(P):
    note("batched uneven set (C5 recipe, 24 problems): F and J^T vs per-problem and oracle")
    specs, probs = batch_problems(24)
    B = P.Batch(specs)
    u = B.empty()
    w = B.empty()
    for i, (s, p) in enumerate(zip(specs, probs)):
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        xs = [m.coords(k) for k in range(2)]
        B.view(u, i).copy_(gpu(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.ic_seed)[None]))
        B.view(w, i).copy_(gpu(wl.normal_field(m.shape, p.target_seed)))
    f = B.rhs(u)
    jt = B.jact_vec(u, w)
    for i, s in enumerate(specs):
        c = P.Context(2, s["order"], s["elems"], s["length"], s["nu"])
        ui, wi = B.view(u, i).contiguous(), B.view(w, i).contiguous()
        # the same kernels for each problem (generic, or the tuned 2-D kernel for order 7 with
        # 8 | E_x, whose row segmentation does not change values): bitwise
        assert torch.equal(B.view(f, i), c.rhs(ui)), (i, c.path)
        assert torch.equal(B.view(jt, i), c.jact_vec(ui, wi)), (i, c.path)
        if i % 6 == 0:
            m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
            assert rel(B.view(f, i), m.rhs(ui.cpu().numpy())) < TOL_APPLY
            assert rel(B.view(jt, i), m.jact_vec(ui.cpu().numpy(), wi.cpu().numpy())) < TOL_APPLY


def test_c5_full_set_sampled(P):
    # the whole 128-problem set in the autotuned launch configuration the benchmark times; the
    # oracle checks sampled problems (the first, the last and the largest of each order)
    note("C5 full set (128 problems, autotuned): F, J^T, 10 RK4 steps + adjoint; oracle on samples")
    specs, probs = batch_problems(wl.C5_COUNT)
    B = P.Batch(specs)
    assert B.autotune() > 0
    u, tg = B.empty(), B.empty()
    meshes = []
    for i, (s, p) in enumerate(zip(specs, probs)):
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        xs = [m.coords(k) for k in range(2)]
        B.view(u, i).copy_(gpu(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.ic_seed)[None]))
        B.view(tg, i).copy_(gpu(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.target_seed)[None]))
        meshes.append(m)
    f, jt = B.rhs(u), B.jact_vec(u, tg)
    n, K = 10, 5
    uT, ck = B.rk4_forward(u, n, K)
    lam = B.rk4_adjoint(ck, n, K, uT - tg)
    sample = {0, len(probs) - 1}
    for N in sorted({p.N for p in probs}):
        sample.add(max((i for i, p in enumerate(probs) if p.N == N), key=lambda i: probs[i].E))
    for i in sorted(sample):
        m, p = meshes[i], probs[i]
        note(f"  problem {i}: N={p.N} E={p.E} nu={p.nu:.2e} dt={p.dt:.2e}")
        ui, ti = B.view(u, i).cpu().numpy(), B.view(tg, i).cpu().numpy()
        # the FP64 rounding floor of a single apply grows with nu / h^2: on problem 50 (N=9, 64^2
        # elements, nu=2.9e-3) the oracle itself is 2.1e-12 from an extended-precision evaluation
        # of F (tests/test_rounding_floor.py::test_floor_of_batched_problem_50 asserts it lies in
        # (1e-12, 4e-12)), so the 32^2 and 64^2 meshes take 1e-11
        tol = TOL_APPLY if p.E <= 16 else 1e-11
        ref, ckr = m.rk4_forward(ui, p.dt, n, K)
        errs = (rel(B.view(f, i), m.rhs(ui)), rel(B.view(jt, i), m.jact_vec(ui, ti)), rel(B.view(uT, i), ref),
                rel(B.view(lam, i), m.rk4_adjoint(ckr, p.dt, n, K, ref - ti)))
        note(f"    F {errs[0]:.2e}  J^T {errs[1]:.2e}  u(T) {errs[2]:.2e}  lambda_0 {errs[3]:.2e}")
        assert errs[0] < tol and errs[1] < tol, i
        assert errs[2] < TOL_TRAJ and errs[3] < TOL_TRAJ, i
    # the whole horizon the benchmark measures: viscous Burgers keeps max|u| from growing (the
    # maximum principle; 1.5x leaves room for the discrete overshoot) and every gradient is finite
    note(f"  all {len(probs)} problems over {wl.C5_STEPS} steps: bounded state, finite gradients")
    uT, ck = B.rk4_forward(u, wl.C5_STEPS, 50)
    lam = B.rk4_adjoint(ck, wl.C5_STEPS, 50, uT - tg)
    for i in range(len(probs)):
        a0, aT = float(B.view(u, i).abs().max()), float(B.view(uT, i).abs().max())
        assert aT <= 1.5 * a0, (i, a0, aT)
    assert bool(torch.isfinite(lam).all())
    # full-horizon parity on the least viscous problem of each order among the meshes of at most
    # 16^2 elements (the oracle finishes those 200 steps in seconds)
    for N in sorted({p.N for p in probs}):
        i = min((i for i, p in enumerate(probs) if p.N == N and p.E <= 16), key=lambda i: probs[i].nu)
        m, p = meshes[i], probs[i]
        ui, ti = B.view(u, i).cpu().numpy(), B.view(tg, i).cpu().numpy()
        ref, ckr = m.rk4_forward(ui, p.dt, wl.C5_STEPS, 50)
        errs = (rel(B.view(uT, i), ref), rel(B.view(lam, i), m.rk4_adjoint(ckr, p.dt, wl.C5_STEPS, 50, ref - ti)))
        note(f"  problem {i}: N={p.N} E={p.E} nu={p.nu:.2e}, {wl.C5_STEPS} steps: u(T) {errs[0]:.2e}  "
             f"lambda_0 {errs[1]:.2e}")
        assert errs[0] < TOL_TRAJ and errs[1] < TOL_TRAJ, i


def test_batch_tuned_problems(P):
    # a set of tuned problems only (orders 3, 5, 7; E_x = 8, 16, 24, 64: 1, 2, 3 and 8 wavefronts),
    # plus the same set with one generic problem in front
    note("batched set of tuned 2-D problems")
    shapes = [(7, (8, 3)), (7, (16, 9)), (5, (24, 2)), (7, (64, 5)), (3, (8, 8)), (5, (8, 1)), (3, (16, 4))]
    for extra in ([], [dict(dim=2, order=5, elems=(4, 3), length=(1.0, 1.0), nu=0.01, dt=1e-3)]):
        specs = extra + [dict(dim=2, order=o, elems=e, length=(1.0 * e[0] / 8, 1.0), nu=0.02, dt=1e-3)
                         for o, e in shapes]
        B = P.Batch(specs)
        u, v = B.empty(), B.empty()
        for i, sp in enumerate(specs):
            m = oracle.Mesh(2, sp["order"], list(sp["elems"]), list(sp["length"]), sp["nu"])
            xs = [m.coords(k) for k in range(2)]
            B.view(u, i).copy_(gpu(wl.fourier_field(xs, list(sp["length"]), 3, 50 + i)[None]))
            B.view(v, i).copy_(gpu(wl.normal_field(m.shape, 60 + i)))
        f, jt = B.rhs(u), B.jact_vec(u, v)
        for i, sp in enumerate(specs):
            c = P.Context(2, sp["order"], sp["elems"], sp["length"], sp["nu"])
            ui, vi = B.view(u, i).contiguous(), B.view(v, i).contiguous()
            assert torch.equal(B.view(f, i), c.rhs(ui)), i
            assert torch.equal(B.view(jt, i), c.jact_vec(ui, vi)), i
            m = oracle.Mesh(2, sp["order"], list(sp["elems"]), list(sp["length"]), sp["nu"])
            assert rel(B.view(f, i), m.rhs(ui.cpu().numpy())) < TOL_APPLY, i
            assert rel(B.view(jt, i), m.jact_vec(ui.cpu().numpy(), vi.cpu().numpy())) < TOL_APPLY, i
        # RK4 through the batch: equal to the per-problem contexts
        n, K = 6, 3
        uT, ck = B.rk4_forward(u, n, K)
        lam = B.rk4_adjoint(ck, n, K, v)
        for i, sp in enumerate(specs):
            c = P.Context(2, sp["order"], sp["elems"], sp["length"], sp["nu"])
            ui = B.view(u, i).contiguous()
            ref, cki = c.rk4_forward(ui, sp["dt"], n, K)
            assert torch.equal(B.view(uT, i), ref), i
            assert torch.equal(B.view(lam, i), c.rk4_adjoint(cki, sp["dt"], n, K, B.view(v, i).contiguous())), i


def test_batch_trajectory_gradient(P):
    note("batched uneven set (12 problems): RK4 forward + adjoint vs per-problem oracle")
    specs, probs = batch_problems(12)
    B = P.Batch(specs)
    u = B.empty()
    lam = B.empty()
    for i, (s, p) in enumerate(zip(specs, probs)):
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        xs = [m.coords(k) for k in range(2)]
        B.view(u, i).copy_(gpu(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.ic_seed)[None]))
        B.view(lam, i).copy_(gpu(wl.normal_field(m.shape, p.target_seed)))
    n, K = 12, 4
    uT, ck = B.rk4_forward(u, n, K)
    lam0 = B.rk4_adjoint(ck, n, K, lam)
    B.set_adjoint_stages("store")  # stored stage states give the same values
    assert torch.equal(B.rk4_adjoint(ck, n, K, lam), lam0)
    B.set_adjoint_stages("auto")
    for i, s in enumerate(specs):
        if s["elems"][0] > 16:
            continue  # keep the oracle side short
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        ui = B.view(u, i).cpu().numpy()
        ref, ckr = m.rk4_forward(ui, s["dt"], n, K)
        assert rel(B.view(uT, i), ref) < TOL_TRAJ, i
        lr = m.rk4_adjoint(ckr, s["dt"], n, K, B.view(lam, i).cpu().numpy())
        assert rel(B.view(lam0, i), lr) < TOL_TRAJ, i


# ------------------------------------------------------------------------------------------------
# RK-3 (Kutta's tableau) forward and discrete adjoint: fused stage kernels vs the oracle's general
# explicit Runge-Kutta
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim,N,E,batch", [(1, 8, [16], 1), (2, 5, [4, 3], 2), (3, 4, [2, 2, 3], 1),
                                           (3, 7, [3, 2, 4], 1), (3, 7, [4, 2, 3], 1), (3, 7, [4, 1, 2], 2),
                                           (2, 7, [8, 2], 2), (2, 3, [8, 3], 1), (3, 7, [12, 2, 2], 2)])
def test_rk3_forward_adjoint(P, dim, N, E, batch):
    note(f"RK-3 forward/adjoint dim={dim} N={N} E={E} batch={batch}")
    L = [E[0] / 4.0, 1.0, 1.0] if dim == 3 and E[0] > 8 else None  # as in test_rk4_forward_adjoint
    m, c = make(P, dim, N, E, nu=0.01, batch=batch, L=L)
    u, _, w = fields(m, 19)
    dt, n, K = (2e-3 if dim > 1 else 2e-4), 20, 5  # the 1-D N=8 mesh on [0, 1] needs the smaller step
    uT_ref, ck_ref = m.erk_forward("rk3", u, dt, n, K)
    assert np.isfinite(uT_ref).all()
    uT, ck = c.rk_forward(gpu(u), dt, n, K, scheme="rk3")
    assert rel(uT, uT_ref) < TOL_TRAJ
    assert rel(ck, ck_ref) < TOL_TRAJ
    lam_ref = m.erk_adjoint("rk3", ck_ref, dt, n, K, w)
    lam = c.rk_adjoint(ck, dt, n, K, gpu(w), scheme="rk3")
    assert rel(lam, lam_ref) < TOL_TRAJ
    # the RK4 entry points and the generic ones with scheme "rk4" are the same integrator
    a, _ = c.rk4_forward(gpu(u), dt, n)
    b, _ = c.rk_forward(gpu(u), dt, n, scheme="rk4")
    assert torch.equal(a, b)


def test_rk3_trajectory_gradient_fd(P):
    note("C1 mesh: RK-3 trajectory, autograd gradient vs oracle and finite differences")
    m, u0, target = c1_inputs()
    c = P.Context(1, wl.C1.N, wl.C1.E, wl.C1.L, wl.C1.nu)
    dt, n, K = wl.C1_DT, wl.C1_STEPS, 10
    x = gpu(u0).requires_grad_(True)
    yT = P.trajectory(x, c, dt, n, K, scheme="rk3")
    loss = 0.5 * ((yT - gpu(target)) ** 2).sum()
    loss.backward()
    uT_ref, ck_ref = m.erk_forward("rk3", u0, dt, n, K)
    phi_ref, lamT = m.misfit(uT_ref, target)
    g_ref = m.erk_adjoint("rk3", ck_ref, dt, n, K, lamT)
    assert abs(loss.item() - phi_ref[0]) < 1e-12 * abs(phi_ref[0])
    assert rel(x.grad, g_ref) < TOL_TRAJ

    def Phi(uu):
        yy, _ = c.rk_forward(gpu(uu), dt, n, scheme="rk3")
        return 0.5 * ((yy - gpu(target)) ** 2).sum().item()
    g = x.grad.cpu().numpy()
    for s in range(8):
        d = wl.normal_field(m.shape, 300 + s)
        eps = 1e-4 * np.linalg.norm(u0) / np.linalg.norm(d)
        fd = (8 * (Phi(u0 + eps * d) - Phi(u0 - eps * d)) - (Phi(u0 + 2 * eps * d) - Phi(u0 - 2 * eps * d))) / (
            12 * eps)
        ad = float(np.vdot(g, d))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (s, fd, ad)


def test_batch_rk3(P):
    note("batched uneven set (8 problems): RK-3 forward + adjoint vs per-problem oracle")
    specs, probs = batch_problems(8)
    B = P.Batch(specs)
    u, lam = B.empty(), B.empty()
    for i, (s, p) in enumerate(zip(specs, probs)):
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        xs = [m.coords(k) for k in range(2)]
        B.view(u, i).copy_(gpu(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, p.ic_seed)[None]))
        B.view(lam, i).copy_(gpu(wl.normal_field(m.shape, p.target_seed)))
    n, K = 8, 4
    uT, ck = B.rk_forward(u, n, K, scheme="rk3")
    lam0 = B.rk_adjoint(ck, n, K, lam, scheme="rk3")
    for i, s in enumerate(specs):
        if s["elems"][0] > 16:
            continue  # keep the oracle side short
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        ref, ckr = m.erk_forward("rk3", B.view(u, i).cpu().numpy(), s["dt"], n, K)
        assert rel(B.view(uT, i), ref) < TOL_TRAJ, i
        lr = m.erk_adjoint("rk3", ckr, s["dt"], n, K, B.view(lam, i).cpu().numpy())
        assert rel(B.view(lam0, i), lr) < TOL_TRAJ, i


# ------------------------------------------------------------------------------------------------
# Binomial (revolve) checkpointing: same step graphs as uniform checkpointing, so bitwise equal
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", ["rk4", "rk3"])
@pytest.mark.parametrize("dim,N,E,batch,snaps", [(2, 5, [4, 3], 2, 3), (3, 7, [4, 2, 3], 1, 4), (1, 6, [9], 1, 1)])
def test_revolve_matches_uniform(P, scheme, dim, N, E, batch, snaps):
    note(f"revolve {scheme} dim={dim} N={N} E={E} batch={batch} snaps={snaps}")
    m, c = make(P, dim, N, E, nu=0.01, batch=batch)
    u, _, w = fields(m, 23)
    dt, n = (2e-3 if dim > 1 else 2e-4), 17
    uT_u, ck_u = c.rk_forward(gpu(u), dt, n, 1, scheme=scheme)
    lam_u = c.rk_adjoint(ck_u, dt, n, 1, gpu(w), scheme=scheme)
    uT_r, ck_r = c.rk_forward_revolve(gpu(u), dt, n, snaps, scheme=scheme)
    assert torch.equal(uT_r, uT_u)
    lam_r = c.rk_adjoint_revolve(ck_r, dt, n, snaps, gpu(w), scheme=scheme)
    assert torch.equal(lam_r, lam_u)
    ck_copy = ck_r.clone()
    assert torch.equal(c.rk_adjoint_revolve(ck_r, dt, n, snaps, gpu(w), scheme=scheme), lam_u)  # repeatable
    assert torch.equal(ck_r, ck_copy)  # snapshots are read only
    ref, ckr = m.erk_forward(scheme, u, dt, n, 1)
    assert rel(uT_r, ref) < TOL_TRAJ
    assert rel(lam_r, m.erk_adjoint(scheme, ckr, dt, n, 1, w)) < TOL_TRAJ


def test_revolve_trajectory_autograd(P):
    note("revolve trajectory gradient equals the uniform one")
    m, u0, target = c1_inputs()
    c = P.Context(1, wl.C1.N, wl.C1.E, wl.C1.L, wl.C1.nu)
    dt, n = wl.C1_DT, wl.C1_STEPS
    grads = []
    for f in (lambda x: P.trajectory(x, c, dt, n, 10), lambda x: P.trajectory_revolve(x, c, dt, n, 4)):
        x = gpu(u0).requires_grad_(True)
        (0.5 * ((f(x) - gpu(target)) ** 2).sum()).backward()
        grads.append(x.grad)
    assert torch.equal(grads[0], grads[1])


# ------------------------------------------------------------------------------------------------
# Crank-Nicolson with Newton-Krylov steps and its discrete adjoint, vs the dense oracle
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim,N,E,batch,n,K", [(1, 8, [16], 1, 10, 5), (2, 4, [3, 2], 2, 6, 3),
                                               (3, 2, [2, 2, 2], 1, 4, 2), (3, 7, [4, 1, 1], 1, 2, 1),
                                               (2, 7, [8, 1], 1, 2, 1)])
def test_cn_forward_adjoint(P, dim, N, E, batch, n, K):
    from oracle import cn as ocn
    note(f"Crank-Nicolson dim={dim} N={N} E={E} batch={batch} steps={n}")
    m, c = make(P, dim, N, E, nu=0.01, batch=batch)
    u, _, w = fields(m, 29)
    dt = 2e-3 if dim > 1 else 1e-3
    uT_ref, ck_ref = ocn.cn_forward(m, u, dt, n, K)
    uT, ck, st = c.cn_forward(gpu(u), dt, n, K)
    assert st["newton_iters"] >= n and st["max_rel_residual"] < 1e-10
    assert rel(uT, uT_ref) < TOL_TRAJ
    assert rel(ck, ck_ref) < TOL_TRAJ
    lam_ref = ocn.cn_adjoint(m, ck_ref, dt, n, K, w)
    lam, st = c.cn_adjoint(ck, dt, n, K, gpu(w))
    assert st["linear_solves"] >= n
    assert rel(lam, lam_ref) < TOL_TRAJ


def test_cn_trajectory_gradient(P):
    from oracle import cn as ocn
    note("C1 mesh: Crank-Nicolson trajectory, autograd gradient vs oracle and finite differences")
    m, u0, target = c1_inputs()
    c = P.Context(1, wl.C1.N, wl.C1.E, wl.C1.L, wl.C1.nu)
    dt, n, K = wl.C1_DT, 20, 5
    x = gpu(u0).requires_grad_(True)
    yT = P.trajectory(x, c, dt, n, K, scheme="cn")
    loss = 0.5 * ((yT - gpu(target)) ** 2).sum()
    loss.backward()
    uT_ref, ck_ref = ocn.cn_forward(m, u0, dt, n, K)
    phi_ref, lamT = m.misfit(uT_ref, target)
    g_ref = ocn.cn_adjoint(m, ck_ref, dt, n, K, lamT)
    assert abs(loss.item() - phi_ref[0]) < 1e-11 * abs(phi_ref[0])
    assert rel(x.grad, g_ref) < TOL_TRAJ

    def Phi(uu):
        yy, _, _ = c.cn_forward(gpu(uu), dt, n)
        return 0.5 * ((yy - gpu(target)) ** 2).sum().item()
    g = x.grad.cpu().numpy()
    for s in range(4):
        d = wl.normal_field(m.shape, 300 + s)
        eps = 1e-4 * np.linalg.norm(u0) / np.linalg.norm(d)
        fd = (8 * (Phi(u0 + eps * d) - Phi(u0 - eps * d)) - (Phi(u0 + 2 * eps * d) - Phi(u0 - 2 * eps * d))) / (
            12 * eps)
        ad = float(np.vdot(g, d))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (s, fd, ad)


def test_cn_nonconvergence_is_reported(P):
    note("Crank-Nicolson iteration limits")
    m, c = make(P, 2, 4, [3, 2], nu=0.01)
    u, _, _ = fields(m, 31)
    with pytest.raises(P.SemError):
        c.cn_forward(gpu(u), 2e-3, 2, opts={"newton_maxit": 1, "newton_rtol": 1e-30})
    with pytest.raises(P.SemError):
        c.cn_forward(gpu(u), 2e-3, 2, opts={"gmres_maxit": 1, "gmres_rtol": 1e-30})


# ------------------------------------------------------------------------------------------------
# LMVM optimal initial condition (Sec. 5, Sec. 6.1) vs the oracle's LMVM
# ------------------------------------------------------------------------------------------------
def lmvm_case(steps, dt=5e-3):
    import test_oracle as to
    return to.recovery_problem(steps, dt)


def test_lmvm_recovery_matches_oracle(P):
    from oracle import lmvm as olmvm
    note("LMVM: 1-D optimal initial condition, RK4, 15 iterations")
    m, exact0, target, guess, dt, n = lmvm_case(800)
    c = P.Context(1, 8, [16], [4.0], 0.01)
    u, hist, st = c.lmvm_initial_condition(gpu(guess), gpu(target), dt, n, 50, scheme="rk4", opts={"max_iters": 15})
    x_ref, h_ref, reason = olmvm.lmvm(olmvm.objective(m, "rk4", target, dt, n, 50), guess, max_iters=15)
    assert st["reason"] == reason == 3 and st["iters"] == 15
    np.testing.assert_allclose(hist, h_ref, rtol=1e-8)
    assert rel(u, x_ref) < 1e-7
    assert hist[-1] < 0.05 * hist[0]


@pytest.mark.parametrize("scheme", ["rk3", "cn"])
def test_lmvm_other_schemes(P, scheme):
    from oracle import lmvm as olmvm
    note(f"LMVM with {scheme}, 4 iterations")
    m, exact0, target, guess, dt, n = lmvm_case(40)
    c = P.Context(1, 8, [16], [4.0], 0.01)
    u, hist, st = c.lmvm_initial_condition(gpu(guess), gpu(target), dt, n, 10, scheme=scheme, opts={"max_iters": 4})
    x_ref, h_ref, reason = olmvm.lmvm(olmvm.objective(m, scheme, target, dt, n, 10), guess, max_iters=4)
    assert st["reason"] == reason
    np.testing.assert_allclose(hist, h_ref, rtol=1e-8)
    assert rel(u, x_ref) < 1e-7


# ------------------------------------------------------------------------------------------------
# Degenerate inputs: empty trajectories, inviscid flow and zero fields, size limits, a batch of one
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim,N,E", [(1, 8, [16]), (2, 7, [8, 2]), (2, 5, [3, 2]), (3, 7, [4, 1, 1])])
def test_zero_steps(P, dim, N, E):
    note(f"zero-step trajectories dim={dim} N={N} E={E}")
    m, c = make(P, dim, N, E)
    u, _, w = fields(m, 3)
    U, W = gpu(u), gpu(w)
    for scheme in ("rk4", "rk3"):
        uT, ck = c.rk_forward(U, 1e-3, 0, 1, scheme=scheme)
        assert torch.equal(uT, U) and ck.numel() == 0
        assert torch.equal(c.rk_adjoint(ck, 1e-3, 0, 1, W, scheme=scheme), W)
    uT, ck, _ = c.cn_forward(U, 1e-3, 0, 1)
    assert torch.equal(uT, U)
    assert torch.equal(c.cn_adjoint(ck, 1e-3, 0, 1, W)[0], W)
    # T = 0: the gradient of 1/2 |u(T)|^2 is u_0 itself
    u0 = U.clone().requires_grad_()
    (0.5 * P.trajectory(u0, c, 1e-3, 0, 1).pow(2).sum()).backward()
    assert torch.equal(u0.grad, U)


def test_zero_steps_batch(P):
    note("zero-step trajectories of a batched set")
    B = P.Batch([dict(dim=2, order=5, elems=(4, 3), length=(1.0, 1.0), nu=0.01, dt=1e-3),
                 dict(dim=2, order=7, elems=(8, 2), length=(1.0, 1.0), nu=0.02, dt=2e-3)])
    x = gpu(wl.normal_field((B.total,), 5))
    uT, ck = B.rk4_forward(x, 0, 1)
    assert torch.equal(uT, x) and ck.numel() == 0
    assert torch.equal(B.rk4_adjoint(ck, 0, 1, x), x)


@pytest.mark.parametrize("dim,N,E", [(1, 6, [5]), (2, 5, [3, 2]), (2, 7, [8, 2]), (3, 3, [2, 2, 2]),
                                     (3, 7, [4, 1, 2])])
def test_inviscid_and_zero_fields(P, dim, N, E):
    # nu = 0 (pure advection) on the generic and both tuned paths; every operator vanishes at
    # u = 0 when nu = 0, exactly (each term carries a factor u)
    note(f"nu = 0 and zero fields dim={dim} N={N} E={E}")
    m, c = make(P, dim, N, E, nu=0.0)
    u, v, w = fields(m, 11)
    U, V, W = gpu(u), gpu(v), gpu(w)
    assert rel(c.rhs(U), m.rhs(u)) < TOL_APPLY
    assert rel(c.jac_vec(U, V), m.jac_vec(u, v)) < TOL_APPLY
    assert rel(c.jact_vec(U, W), m.jact_vec(u, w)) < TOL_APPLY
    Z = torch.zeros_like(U)
    for r in (c.rhs(Z), c.jac_vec(Z, V), c.jact_vec(Z, W)):
        assert int(torch.count_nonzero(r)) == 0


def test_size_limits(P):
    note("meshes beyond the index range are rejected before any allocation")
    with pytest.raises(P.SemError, match="too large"):
        P.Context(3, 7, [2048, 2048, 64], [1.0, 1.0, 1.0], 0.01)  # >= 2^31 nodes per component
    with pytest.raises(P.SemError, match="too large"):
        P.Context(1, 8, [1 << 28], [1.0], 0.01)  # more than 2^30 grid points along a direction
    with pytest.raises(P.SemError, match="too large"):
        P.Context(2, 11, [4096, 4096], [1.0, 1.0], 0.01, batch=300)  # > 2^40 values in the field


def test_batch_of_one(P):
    # a set of one problem runs the batched machinery (no tuned single-problem kernel) and must
    # agree with the oracle and with its own context
    note("batched set of a single problem")
    spec = dict(dim=2, order=5, elems=(3, 4), length=(1.0, 1.0), nu=0.02, dt=1e-3)
    B = P.Batch([spec])
    m = oracle.Mesh(2, 5, [3, 4], [1.0, 1.0], 0.02)
    u, _, w = fields(m, 21)
    U, W = gpu(u).reshape(-1), gpu(w).reshape(-1)
    assert rel(B.rhs(U), m.rhs(u).reshape(-1)) < TOL_APPLY
    assert rel(B.jact_vec(U, W), m.jact_vec(u, w).reshape(-1)) < TOL_APPLY
    c = P.Context(2, 5, [3, 4], [1.0, 1.0], 0.02)
    uT, ck = B.rk4_forward(U, 4, 2)
    uT1, ck1 = c.rk4_forward(U.view(c.shape), 1e-3, 4, 2)
    assert rel(uT, uT1.reshape(-1)) < TOL_TRAJ
    assert rel(B.rk4_adjoint(ck, 4, 2, W), c.rk4_adjoint(ck1, 1e-3, 4, 2, W.view(c.shape)).reshape(-1)) < TOL_TRAJ


# ------------------------------------------------------------------------------------------------
# Error handling at the boundary
# ------------------------------------------------------------------------------------------------
def test_errors(P):
    note("argument errors")
    with pytest.raises(P.SemError):
        P.Context(3, 10, [2, 2, 2], [1, 1, 1], 0.1)  # order outside the compiled 3-D range
    with pytest.raises(P.SemError):
        P.Context(2, 3, [0, 2], [1, 1], 0.1)
    m, c = make(P, 2, 3, [2, 2])
    u = torch.zeros(c.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError):
        P.lib() and P.sem._call(P.lib().sem_rhs(c._h, P.sem._ptr(u), P.sem._ptr(u)))  # aliasing
    with pytest.raises(P.SemError):
        c.rk4_forward(u, 1e-3, 10, 3)  # 3 does not divide 10
    with pytest.raises(P.SemError):
        c.rk4_forward(u, -1.0, 10, 0)
    with pytest.raises(P.SemError):
        c.rhs(torch.zeros(5, dtype=torch.float64, device="cuda"))
    with pytest.raises(P.SemError):
        c.rk_forward(u, 1e-3, 10, scheme="rk2")  # unknown scheme (binding)
    with pytest.raises(P.SemError):
        P.sem._call(P.lib().sem_rk_forward(c._h, 7, P.sem._ptr(u), 1e-3, 10, 0, None))  # unknown scheme (ABI)


def test_nonfinite_detection(P):
    note("non-finite trajectory detection")
    m, c = make(P, 1, 8, [16], nu=0.01, L=[2 * np.pi])
    u = gpu(np.sin(m.coords(0))[None, None])
    c.set_check_finite(True)
    c.rk4_forward(u, 1e-3, 10)
    with pytest.raises(P.SemError):
        c.rk4_forward(u, 5.0, 200)  # far beyond the stability limit


def test_batch_launch_shapes_and_autotune(P):
    note("batched uneven set (C5 recipe, 20 problems, and 5 generic ones): launch shapes bitwise equal, autotune")
    specs = mixed_batch_specs(20)
    B = P.Batch(specs)
    u = B.empty()
    w = B.empty()
    for i, s in enumerate(specs):
        m = oracle.Mesh(2, s["order"], list(s["elems"]), [1.0, 1.0], s["nu"])
        xs = [m.coords(k) for k in range(2)]
        B.view(u, i).copy_(gpu(wl.fourier_field(xs, [1.0, 1.0], wl.C5_K, 41 + i)[None]))
        B.view(w, i).copy_(gpu(wl.normal_field(m.shape, 1041 + i)))
    B.configure(True, 1024)
    f0, j0 = B.rhs(u), B.jact_vec(u, w)
    u1, _ = B.rk4_forward(u, 6, 0)
    for persistent, param in [(True, 7), (True, 300), (False, 0), (False, 1), (False, 4), (False, 16)]:
        B.configure(persistent, param)
        assert torch.equal(B.rhs(u), f0), (persistent, param)
        assert torch.equal(B.jact_vec(u, w), j0), (persistent, param)
        assert torch.equal(B.rk4_forward(u, 6, 0)[0], u1), (persistent, param)
    ms = B.autotune()
    assert ms > 0
    assert torch.equal(B.rhs(u), f0) and torch.equal(B.rk4_forward(u, 6, 0)[0], u1)
    with pytest.raises(P.SemError):
        B.configure(True, 0)


def test_configure_right_after_unsynchronised_integration(P):
    # configure drops the captured step graphs; with graph launches of an integration still in
    # flight it must wait for them first.  Results after the change equal those before, bitwise.
    note("batched set: configure right after an unsynchronised rk4_forward / rk4_adjoint")
    specs = mixed_batch_specs(20)
    B = P.Batch(specs)
    x = gpu(wl.normal_field((B.total,), 31)) * 0.01
    B.configure(False, 0)
    ref_T, ref_ck = B.rk4_forward(x, 40, 10)
    ref_l = B.rk4_adjoint(ref_ck, 40, 10, ref_T)
    torch.cuda.synchronize()
    for persistent, param in [(True, 512), (False, 4), (False, 0)]:
        xT, ck = B.rk4_forward(x, 40, 10)   # enqueued, not waited for
        B.configure(persistent, param)      # graphs destroyed while the forward may still run
        lam = B.rk4_adjoint(ck, 40, 10, xT)
        B.configure(not persistent, 0 if persistent else 1024)
        torch.cuda.synchronize()
        assert torch.equal(xT, ref_T) and torch.equal(lam, ref_l), (persistent, param)
    B.close()


def test_side_stream(P):
    # contexts and batched sets follow torch's current stream: on a side stream (default
    # priority), with torch producing the inputs and reading the outputs on that stream, the
    # results equal the default stream's bitwise
    note("operators and trajectories on a side stream")
    m, c = make(P, 3, 7, [4, 1, 2])
    u, _, w = fields(m, 5)
    U = gpu(u)
    f0, uT0 = c.rhs(U), c.rk4_forward(U, 1e-3, 4, 2)[0]
    specs, _ = batch_problems(6)
    B = P.Batch(specs)
    x = gpu(wl.normal_field((B.total,), 9)) * 0.01
    bf0, bT0 = B.rhs(x), B.rk4_forward(x, 3, 0)[0]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        U2, x2 = U * 1.0, x * 1.0
        f1, uT1 = c.rhs(U2), c.rk4_forward(U2, 1e-3, 4, 2)[0]
        bf1, bT1 = B.rhs(x2), B.rk4_forward(x2, 3, 0)[0]
        d = torch.stack([(f1 - f0).abs().max(), (uT1 - uT0).abs().max(), (bf1 - bf0).abs().max(),
                         (bT1 - bT0).abs().max()])
    s.synchronize()
    assert float(d.max()) == 0.0, d


# ------------------------------------------------------------------------------------------------
# Resources: device memory across create / use / destroy cycles (last: a failure hides nothing)
# ------------------------------------------------------------------------------------------------
def test_lifecycle_releases_device_memory(P):
    # contexts and batched sets with their integrator buffers, captured graphs, face buffers and
    # autotuning, created and destroyed repeatedly: device memory returns to where it started
    note("create / use / destroy cycles release their device memory")
    specs, _ = batch_problems(6)

    def cycle():
        c = P.Context(3, 7, [8, 4, 4], [1.0, 1.0, 1.0], 0.01)
        u = c.empty().normal_(0, 0.1)
        uT, ck = c.rk4_forward(u, 1e-4, 2, 1)
        c.rk4_adjoint(ck, 1e-4, 2, 1, uT)
        c.rk_forward_stored(u, 1e-4, 2, scheme="rk3")
        c.close()
        B = P.Batch(specs)
        B.autotune()
        x = B.empty().normal_(0, 0.01)
        xT, ckb = B.rk4_forward(x, 2, 1)
        B.rk4_adjoint(ckb, 2, 1, xT)
        B.close()

    cycle()  # first use: library code objects, torch's allocator pools
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(4):
        cycle()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    note(f"  free before {free0 >> 20} MiB, after {free1 >> 20} MiB")
    assert free0 - free1 < (64 << 20), (free0, free1)


def test_fp64_rate_probe(P):
    # the diagnostic entry point runs and reports plausible rates (below the 78.6 TFLOP/s FP64
    # peak, with margin for the clock); its figures themselves are measurements, not parity
    note("FP64 rate probe")
    r = P.probe_fp64_rates(iters=200)
    for k in ("mfma_alone", "valu_alone", "interleaved_mfma", "interleaved_valu"):
        assert 0 < r[k] < 100, (k, r[k])
    assert r["interleaved_total"] < 100

