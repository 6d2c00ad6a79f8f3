"""Pins for the CPU oracle (no GPU).

Every check here compares the oracle with something other than itself: closed forms of the GLL
rule, exactness of quadrature and differentiation, analytic solutions printed in the paper
(Cole-Hopf Burgers, Sec. 6.1.1; frozen-speed advection-diffusion, Sec. 6.1), the strong form of
the PDE (Sec. 3, eq. burgers23d), conservation, the dot-product and polarisation identities, an
explicit Jacobian built column by column as in Sec. 6, finite differences of the whole trajectory
(Sec. 6), tangent-linear/adjoint duality, and a dense Kronecker assembly on tiny meshes.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

# ------------------------------------------------------------------------------------------------
# GLL tables (Sec. 3.2)
# ------------------------------------------------------------------------------------------------
CLOSED = {
    1: (np.array([-1.0, 1.0]), np.array([1.0, 1.0])),
    2: (np.array([-1.0, 0.0, 1.0]), np.array([1 / 3, 4 / 3, 1 / 3])),
    3: (np.array([-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0]), np.array([1 / 6, 5 / 6, 5 / 6, 1 / 6])),
    4: (np.array([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0]),
        np.array([1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10])),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(N):
    xi, w, D = oracle.gll(N)
    np.testing.assert_allclose(xi, CLOSED[N][0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, CLOSED[N][1], rtol=0, atol=1e-15)
    if N == 1:
        np.testing.assert_allclose(D, [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-15)
    if N == 2:
        np.testing.assert_allclose(D, [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]], atol=1e-15)


@pytest.mark.parametrize("N", list(range(1, 17)))
def test_gll_invariants(N):
    xi, w, D = oracle.gll(N)
    P = N + 1
    # interior nodes are the roots of P_N' (library root finder, looser accuracy)
    if N >= 2:
        r = np.sort(np.polynomial.legendre.Legendre.basis(N).deriv().roots().real)
        np.testing.assert_allclose(xi[1:-1], r, atol=1e-10)
    # symmetric nodes, weights summing to the reference length
    np.testing.assert_allclose(xi, -xi[::-1], atol=0)
    assert abs(w.sum() - 2.0) < 1e-14
    # quadrature exact to degree 2N-1
    for k in range(2 * N):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14, k
    # differentiation exact on monomials up to degree N
    for k in range(N + 1):
        dk = k * xi ** (k - 1) if k > 0 else np.zeros(P)
        np.testing.assert_allclose(D @ xi ** k, dk, atol=2e-13 * max(1, N) ** 2)
    # centro-antisymmetry D_{N-i,N-j} = -D_ij and the textbook corner values
    np.testing.assert_allclose(D[::-1, ::-1], -D, atol=1e-12 * N * N)
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-12 * N * N
    assert abs(D[N, N] - N * (N + 1) / 4) < 1e-12 * N * N
    # K = D^T W D is the exact stiffness of the Lagrange basis: x^T K x = int (p')^2 for p = x^N/x^{N-1}
    K = D.T @ np.diag(w) @ D
    for k in (N, max(N - 1, 1)):
        p = xi ** k
        exact = k * k * 2.0 / (2 * k - 1)  # int_{-1}^{1} (k x^{k-1})^2 dx
        assert abs(p @ K @ p - exact) < 1e-11 * exact


# ------------------------------------------------------------------------------------------------
# Helpers
# ------------------------------------------------------------------------------------------------
def mesh(dim, N, E, L=None, nu=0.05, batch=1):
    L = L or [1.0] * dim
    return oracle.Mesh(dim, N, E, L, nu, batch)


def grids(m):
    """Coordinates broadcast to the field layout [z][y][x] for each direction."""
    xs = [m.coords(k) for k in range(m.dim)]
    mg = np.meshgrid(*reversed(xs), indexing="ij")  # z, y, x order
    return list(reversed(mg))  # x, y, z


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rand(m, seed):
    return wl.normal_field(m.shape, seed)


# ------------------------------------------------------------------------------------------------
# F(u) against the strong form of the PDE (Sec. 3, eq. burgers23d): spectral convergence
# ------------------------------------------------------------------------------------------------
MODES = {  # component -> list of (k vector, a, b) for a cos(2 pi k.x) + b sin(2 pi k.x)
    1: [[((1,), 0.3, 1.0), ((2,), -0.2, 0.1)]],
    2: [[((1, 0), 0.2, 1.0), ((1, 1), 0.0, 0.4)], [((0, 1), 0.5, -0.3), ((2, -1), 0.1, 0.0)]],
    3: [[((1, 0, 0), 0.1, 1.0), ((0, 1, 1), 0.3, 0.0)], [((0, 1, 0), 0.4, -0.5), ((1, 0, 1), 0.0, 0.2)],
        [((0, 0, 1), -0.3, 0.6), ((1, 1, 0), 0.2, 0.1)]],
}


def analytic(dim, X):
    """u, grad u and Laplacian of the trigonometric field MODES[dim] at coordinates X (unit box)."""
    u, gu, lu = [], [], []
    for c in range(dim):
        uc = 0.0
        gc = [0.0] * dim
        lc = 0.0
        for k, a, b in MODES[dim][c]:
            th = 2 * np.pi * sum(k[j] * X[j] for j in range(dim))
            cs, sn = np.cos(th), np.sin(th)
            uc = uc + a * cs + b * sn
            for j in range(dim):
                gc[j] = gc[j] + 2 * np.pi * k[j] * (-a * sn + b * cs)
            lc = lc - (2 * np.pi) ** 2 * sum(kk * kk for kk in k) * (a * cs + b * sn)
        u.append(uc)
        gu.append(gc)
        lu.append(lc)
    return u, gu, lu


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_rhs_converges_to_strong_form(dim):
    nu = 0.05
    errs = []
    Ns = [4, 7, 10] if dim == 3 else [4, 8, 12]
    for N in Ns:
        m = mesh(dim, N, [3] * dim, nu=nu)
        X = grids(m)
        u, gu, lu = analytic(dim, X)
        f = m.rhs(np.stack(u)[None])
        exact = np.stack([nu * lu[i] - sum(u[j] * gu[i][j] for j in range(dim)) for i in range(dim)])[None]
        errs.append(rel(f, exact))
    assert errs[0] > 10 * errs[1] > 100 * errs[2] or errs[2] < 1e-9, errs
    assert errs[-1] < (1e-6 if dim == 3 else 1e-8), errs


def test_rhs_of_constant_is_zero():
    for dim in (1, 2, 3):
        m = mesh(dim, 5, [2] * dim)
        u = np.ones(m.shape) * np.arange(1.0, dim + 1).reshape((1, dim) + (1,) * dim)
        assert np.abs(m.rhs(u)).max() < 1e-12


def test_mass_sums_to_volume():
    for dim in (1, 2, 3):
        L = [1.0, 2.0, 0.5][:dim]
        m = oracle.Mesh(dim, 5, [3, 2, 4][:dim], L, 0.1)
        assert abs(m.mass().sum() - np.prod(L)) < 1e-13


def test_conservation_1d():
    # 1^T M F(u) = 0: the advective term integrates u u_x exactly (degree 2N-1) and telescopes,
    # the diffusive term annihilates constants (Sec. 3.2, eq. discrete1d with K = D^T M D).
    m = mesh(1, 8, [16], L=[2 * np.pi], nu=0.01)
    u = rand(m, 5)
    M = m.mass()
    f = m.rhs(u)
    assert abs((M * f[0, 0]).sum()) < 1e-13 * np.abs(M * f[0, 0]).sum()
    # and its derivative: J(u)^T (M 1) = 0
    jt = m.jact_vec(u, M[None, None] * np.ones(m.shape))
    assert np.abs(jt).max() < 1e-12 * np.abs(m.jact_vec(u, rand(m, 6))).max()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_shift_equivariance(dim):
    # shifting the field by one element along x shifts F by one element (bitwise)
    N = 4
    m = mesh(dim, N, [3] * dim)
    u = rand(m, 7)
    f = m.rhs(u)
    us = np.roll(u, N, axis=-1)
    np.testing.assert_array_equal(m.rhs(us), np.roll(f, N, axis=-1))


# ------------------------------------------------------------------------------------------------
# Jacobian and transpose (Sec. 3.3, eqs. jacvec, jactransvec)
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_polarization(dim):
    # F is quadratic, so (F(u+v) - F(u-v))/2 = J(u) v exactly up to rounding
    m = mesh(dim, [8, 5, 3][dim - 1], [3] * dim, nu=0.02)
    u, v = rand(m, 1), rand(m, 2)
    jv = m.jac_vec(u, v)
    pol = 0.5 * (m.rhs(u + v) - m.rhs(u - v))
    assert rel(jv, pol) < 1e-13


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_dot_identity(dim):
    m = mesh(dim, [8, 5, 3][dim - 1], [4, 3, 2][: dim], nu=0.02)
    u, v, w = rand(m, 1), rand(m, 2), rand(m, 3)
    lhs = np.vdot(m.jac_vec(u, v), w)
    rhs = np.vdot(v, m.jact_vec(u, w))
    scale = np.linalg.norm(m.jac_vec(u, v)) * np.linalg.norm(w)
    assert abs(lhs - rhs) < 1e-14 * scale


@pytest.mark.parametrize("dim,N,E", [(1, 2, 3), (2, 2, 2), (3, 2, 2), (1, 7, 2), (2, 3, 3)])
def test_explicit_jacobian_transpose(dim, N, E):
    # Sec. 6: build J explicitly by applying the matrix-free J to the identity, then check that the
    # matrix-free transpose product matches the explicit matrix's transpose.
    m = mesh(dim, N, [E] * dim, nu=0.03)
    u = rand(m, 11)
    n = m.ndof
    J = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        J[:, c] = m.jac_vec(u, e.reshape(m.shape)).ravel()
    w = rand(m, 12)
    np.testing.assert_allclose(m.jact_vec(u, w).ravel(), J.T @ w.ravel(), rtol=0,
                               atol=1e-12 * np.abs(J.T @ w.ravel()).max())


# ------------------------------------------------------------------------------------------------
# Dense Kronecker assembly on tiny meshes (independent indexing of Q, the element maps and DSS)
# ------------------------------------------------------------------------------------------------
def dense_ops(m):
    xi, wq, Dh = oracle.gll(m.N)
    P = m.N + 1
    dim = m.dim
    h = [m.L[k] / m.E[k] for k in range(dim)]
    I = np.eye(P)
    # local operators on index q = q0 + P q1 + P^2 q2 (x fastest => x is the last Kronecker factor)
    def kron_dir(A, j):
        mats = [I] * dim
        mats[j] = A
        out = np.ones((1, 1))
        for k in reversed(range(dim)):
            out = np.kron(out, mats[k])
        return out
    Dl = [kron_dir(Dh, j) * 2.0 / h[j] for j in range(dim)]
    wl_ = np.ones(1)
    for k in reversed(range(dim)):
        wl_ = np.kron(wl_, wq * h[k] / 2)
    nloc = P ** dim
    E = [m.E[k] for k in range(dim)]
    n = [m.n[k] for k in range(dim)]
    nel = int(np.prod(E))
    Q = np.zeros((nel * nloc, m.nodes))
    for e in range(nel):
        ed = np.unravel_index(e, tuple(reversed(E)))[::-1]  # x fastest
        for q in range(nloc):
            qd = np.unravel_index(q, (P,) * dim)[::-1]
            g = [(ed[k] * m.N + qd[k]) % n[k] for k in range(dim)]
            gi = np.ravel_multi_index(tuple(reversed(g)), tuple(reversed(n)))
            Q[e * nloc + q, gi] = 1.0
    Dg = [np.kron(np.eye(nel), Dk) for Dk in Dl]
    W = np.tile(wl_, nel)
    Mass = Q.T @ W
    return Q, Dg, W, Mass


@pytest.mark.parametrize("dim,N,E", [(1, 2, 3), (2, 2, 2), (3, 2, 2), (2, 4, 3)])
def test_dense_assembly(dim, N, E):
    m = mesh(dim, N, [E] * dim, nu=0.07)
    Q, Dg, W, Mass = dense_ops(m)
    u = rand(m, 21).reshape(dim, -1)
    v = rand(m, 22).reshape(dim, -1)
    U = [Q @ u[i] for i in range(dim)]
    V = [Q @ v[i] for i in range(dim)]
    F = []
    Jv = []
    for i in range(dim):
        r = -sum(Dg[j].T @ (m.nu * W * (Dg[j] @ U[i])) for j in range(dim))
        r -= W * sum(U[j] * (Dg[j] @ U[i]) for j in range(dim))
        F.append(Q.T @ r / Mass)
        rj = -sum(Dg[j].T @ (m.nu * W * (Dg[j] @ V[i])) for j in range(dim))
        rj -= W * sum(V[j] * (Dg[j] @ U[i]) + U[j] * (Dg[j] @ V[i]) for j in range(dim))
        Jv.append(Q.T @ rj / Mass)
    F = np.stack(F).reshape(m.shape)
    Jv = np.stack(Jv).reshape(m.shape)
    assert rel(m.rhs(u.reshape(m.shape)), F) < 1e-13
    assert rel(m.jac_vec(u.reshape(m.shape), v.reshape(m.shape)), Jv) < 1e-13


# ------------------------------------------------------------------------------------------------
# Time integration against the paper's closed-form solutions
# ------------------------------------------------------------------------------------------------
def cole_hopf(x, t, nu, a):
    """Sec. 6.1.1: u = 2 nu pi sin(pi x) e^{-nu pi^2 t} / (a + e^{-nu pi^2 t} cos(pi x)), period 2
    (the paper's domain [-2, 2] shifted to [0, 4]; a = 2 is the paper's value)."""
    ex = np.exp(-nu * np.pi ** 2 * t)
    return 2 * nu * np.pi * np.sin(np.pi * x) * ex / (a + ex * np.cos(np.pi * x))


@pytest.mark.parametrize("a", [2.0, 1.25])
def test_cole_hopf_spectral_in_N(a):
    nu, T, dt = 0.1, 1.0, 2e-3
    errs = []
    for N in (4, 8, 12):
        m = oracle.Mesh(1, N, [4], [4.0], nu)
        x = m.coords(0)
        uT, _ = m.rk4_forward(cole_hopf(x, 0.0, nu, a)[None, None], dt, int(round(T / dt)))
        errs.append(rel(uT[0, 0], cole_hopf(x, T, nu, a)))
    # geometric (spectral) decay: each +4 in N gains more than two orders of magnitude
    assert errs[0] > 100 * errs[1] and errs[1] > 100 * errs[2] and errs[2] < 1e-6, errs


def test_cole_hopf_fourth_order_in_dt():
    nu, a, T = 0.1, 1.25, 0.5
    m = oracle.Mesh(1, 8, [4], [4.0], nu)
    x = m.coords(0)
    u0 = cole_hopf(x, 0.0, nu, a)[None, None]
    ref, _ = m.rk4_forward(u0, 2.5e-4, 2000)  # time-converged reference on the same mesh
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        uT, _ = m.rk4_forward(u0, dt, int(round(T / dt)))
        errs.append(rel(uT, ref))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.6 < r < 4.4 for r in rates), (errs, rates)


@pytest.mark.parametrize("dim", [1, 2])
def test_frozen_speed_advection_diffusion(dim):
    # Sec. 6.1: with the nonlinearity frozen at a constant speed a, v = sum_j a_j sin(2 pi j (x - a t))
    # e^{-nu 4 pi^2 j^2 t}.  The tangent-linear model about a constant state is exactly this linear
    # problem (F(const) = 0 keeps the state fixed).
    nu, T, dt = 1e-3, 0.05, 5e-4
    amp = wl.rng(4).uniform(0.9, 1.0, 5)
    speed = [0.1, -0.07][:dim]
    m = mesh(dim, 12, [6] * dim, nu=nu)
    X = grids(m)

    def exact(t):
        fld = []
        for c in range(dim):
            s = 0.0
            for j, aj in enumerate(amp[:3], start=1):
                arg = sum(2 * np.pi * j * (X[d] - speed[d] * t) for d in range(dim))
                s = s + aj * np.sin(arg) * np.exp(-nu * 4 * np.pi ** 2 * j * j * dim * t)
            fld.append(s * (c + 1))
        return np.stack(fld)[None]

    ubar = np.stack([np.full(X[0].shape, speed[c]) for c in range(dim)])[None]
    _, vT = m.rk4_tlm(ubar, exact(0.0), dt, int(round(T / dt)))
    assert rel(vT, exact(T)) < 1e-7


# ------------------------------------------------------------------------------------------------
# Discrete adjoint (Sec. 4.1) and checkpointing (Sec. 5.3-5.4)
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


def test_projection_is_continuous_average():
    # M^{-1} Q^T (omega o n) of a field that is already continuous returns it unchanged
    m = mesh(2, 4, [3, 2])
    u = rand(m, 8)
    loc = np.zeros((1, m.nelem, m.C, m.nloc))
    P = m.N + 1
    for e in range(m.nelem):
        ex, ey = e % m.E[0], e // m.E[0]
        for q in range(m.nloc):
            qx, qy = q % P, q // P
            gx, gy = (ex * m.N + qx) % m.n[0], (ey * m.N + qy) % m.n[1]
            loc[0, e, :, q] = u[0, :, gy, gx]
    assert rel(m.project_local(loc), u) < 1e-14


def test_adjoint_gradient_vs_finite_differences():
    m, u0, target = c1_inputs()
    dt, n, K = wl.C1_DT, wl.C1_STEPS, 10
    phi, g = m.gradient(u0, target, dt, n, K)

    def Phi(u):
        uT, _ = m.rk4_forward(u, dt, n)
        return m.misfit(uT, target)[0][0]

    assert abs(Phi(u0) - phi[0]) == 0.0
    for s in range(16):
        d = wl.normal_field(m.shape, 300 + s)
        eps = 1e-4 * np.linalg.norm(u0) / np.linalg.norm(d)
        # fourth-order central stencil: its truncation error (~1e-11 here) is far below the bar;
        # the two-point stencil's error scales as eps^2 (1e-6 at this eps)
        fd = (8 * (Phi(u0 + eps * d) - Phi(u0 - eps * d)) - (Phi(u0 + 2 * eps * d) - Phi(u0 - 2 * eps * d))) \
            / (12 * eps)
        ad = np.vdot(g, d)
        assert abs(fd - ad) <= 1e-8 * abs(ad), (s, fd, ad)


def test_tangent_linear_adjoint_duality():
    m = mesh(2, 5, [3, 3], nu=0.01)
    u0 = wl.fourier_field([m.coords(0), m.coords(1)], [1, 1], 3, 9)[None]
    du0 = rand(m, 10)
    lamN = rand(m, 11)
    dt, n, K = 1e-3, 12, 4
    _, duN = m.rk4_tlm(u0, du0, dt, n)
    _, ck = m.rk4_forward(u0, dt, n, K)
    lam0 = m.rk4_adjoint(ck, dt, n, K, lamN)
    a, b = np.vdot(lam0, du0), np.vdot(lamN, duN)
    assert abs(a - b) < 1e-12 * abs(b)


def test_checkpointing_is_bitwise_store_all():
    m, u0, target = c1_inputs()
    dt, n = wl.C1_DT, 20
    lams = []
    for K in (1, 5, 20):
        uT, ck = m.rk4_forward(u0, dt, n, K)
        _, lamT = m.misfit(uT, target)
        lams.append(m.rk4_adjoint(ck, dt, n, K, lamT))
    np.testing.assert_array_equal(lams[0], lams[1])
    np.testing.assert_array_equal(lams[0], lams[2])


def test_batch_equals_single():
    m = mesh(2, 4, [3, 2], nu=0.02, batch=3)
    u, w = rand(m, 31), rand(m, 32)
    fb, jb = m.rhs(u), m.jact_vec(u, w)
    m1 = m.with_batch(1)
    for b in range(3):
        np.testing.assert_array_equal(fb[b:b + 1], m1.rhs(u[b:b + 1]))
        np.testing.assert_array_equal(jb[b:b + 1], m1.jact_vec(u[b:b + 1], w[b:b + 1]))


def test_invalid_arguments_rejected():
    with pytest.raises(RuntimeError):
        oracle.Mesh(1, 0, [2], [1.0], 0.1).rhs(np.zeros(0))
    with pytest.raises(RuntimeError):
        m = mesh(1, 3, [2])
        m.rk4_adjoint(np.zeros((3,) + m.shape), 1e-3, 10, 3, np.zeros(m.shape))


# ------------------------------------------------------------------------------------------------
# General explicit Runge-Kutta (the paper's three-stage RK-3 of Sec. 6.3; Kutta's tableau is the
# reading taken, the paper prints none) and its discrete adjoint (Sec. 4.1 for a general tableau)
# ------------------------------------------------------------------------------------------------
def test_rk3_tableau_is_three_stage_third_order():
    A, b = oracle.erk_tableau("rk3")
    c = A.sum(axis=1)
    assert A.shape == (3, 3) and np.allclose(np.triu(A), 0)  # three explicit stages
    # the four order conditions of a third-order Runge-Kutta method
    assert abs(b.sum() - 1) < 1e-15
    assert abs(b @ c - 1 / 2) < 1e-15
    assert abs(b @ c ** 2 - 1 / 3) < 1e-15
    assert abs(b @ (A @ c) - 1 / 6) < 1e-15


def test_rk3_third_order_in_dt():
    nu, a, T = 0.1, 1.25, 0.5
    m = oracle.Mesh(1, 8, [4], [4.0], nu)
    u0 = cole_hopf(m.coords(0), 0.0, nu, a)[None, None]
    ref, _ = m.rk4_forward(u0, 2.5e-4, 2000)
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        uT, _ = m.erk_forward("rk3", u0, dt, int(round(T / dt)))
        errs.append(rel(uT, ref))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.7 < r < 3.3 for r in rates), (errs, rates)


def test_generic_tableau_route_reproduces_rk4():
    # the general explicit-RK code with the classical tableau against the separately pinned RK4
    m = mesh(2, 5, [3, 2], nu=0.01)
    u0 = wl.fourier_field([m.coords(0), m.coords(1)], [1, 1], 3, 21)[None]
    lamT = rand(m, 22)
    dt, n, K = 1e-3, 8, 4
    a, cka = m.rk4_forward(u0, dt, n, K)
    b, ckb = m.erk_forward("rk4", u0, dt, n, K)
    assert rel(b, a) < 1e-15 and rel(ckb, cka) < 1e-15
    assert rel(m.erk_adjoint("rk4", ckb, dt, n, K, lamT), m.rk4_adjoint(cka, dt, n, K, lamT)) < 1e-14


def test_rk3_adjoint_gradient_vs_finite_differences():
    m, u0, target = c1_inputs()
    dt, n, K = wl.C1_DT, wl.C1_STEPS, 10
    uT, ck = m.erk_forward("rk3", u0, dt, n, K)
    _, lamT = m.misfit(uT, target)
    g = m.erk_adjoint("rk3", ck, dt, n, K, lamT)

    def Phi(u):
        return m.misfit(m.erk_forward("rk3", u, dt, n)[0], target)[0][0]

    for s in range(8):
        d = wl.normal_field(m.shape, 300 + s)
        eps = 1e-4 * np.linalg.norm(u0) / np.linalg.norm(d)
        fd = (8 * (Phi(u0 + eps * d) - Phi(u0 - eps * d)) - (Phi(u0 + 2 * eps * d) - Phi(u0 - 2 * eps * d))) \
            / (12 * eps)
        ad = np.vdot(g, d)
        assert abs(fd - ad) <= 1e-8 * abs(ad), (s, fd, ad)


def test_rk3_tangent_linear_adjoint_duality():
    m = mesh(2, 5, [3, 3], nu=0.01)
    u0 = wl.fourier_field([m.coords(0), m.coords(1)], [1, 1], 3, 9)[None]
    du0, lamN = rand(m, 10), rand(m, 11)
    dt, n, K = 1e-3, 12, 4
    _, duN = m.erk_tlm("rk3", u0, du0, dt, n)
    _, ck = m.erk_forward("rk3", u0, dt, n, K)
    lam0 = m.erk_adjoint("rk3", ck, dt, n, K, lamN)
    a, b = np.vdot(lam0, du0), np.vdot(lamN, duN)
    assert abs(a - b) < 1e-12 * abs(b)


def test_rk3_frozen_speed_advection_diffusion():
    # the linear problem of test_frozen_speed_advection_diffusion, stepped with RK-3
    nu, T, dt, dim = 1e-3, 0.05, 5e-4, 1
    amp = wl.rng(4).uniform(0.9, 1.0, 5)
    m = mesh(dim, 12, [6], nu=nu)
    X = grids(m)

    def exact(t):
        s = 0.0
        for j, aj in enumerate(amp[:3], start=1):
            s = s + aj * np.sin(2 * np.pi * j * (X[0] - 0.1 * t)) * np.exp(-nu * 4 * np.pi ** 2 * j * j * t)
        return s[None, None]

    ubar = np.full((1, 1) + X[0].shape, 0.1)
    _, vT = m.erk_tlm("rk3", ubar, exact(0.0), dt, int(round(T / dt)))
    assert rel(vT, exact(T)) < 1e-7


def test_rk3_checkpointing_is_bitwise_store_all():
    m, u0, target = c1_inputs()
    dt, n = wl.C1_DT, 20
    lams = []
    for K in (1, 5, 20):
        uT, ck = m.erk_forward("rk3", u0, dt, n, K)
        _, lamT = m.misfit(uT, target)
        lams.append(m.erk_adjoint("rk3", ck, dt, n, K, lamT))
    np.testing.assert_array_equal(lams[0], lams[1])
    np.testing.assert_array_equal(lams[0], lams[2])


# ------------------------------------------------------------------------------------------------
# Crank-Nicolson (the paper's implicit scheme, Sec. 6.3) with Newton, and its discrete adjoint
# ------------------------------------------------------------------------------------------------
from oracle import cn as ocn  # noqa: E402


def test_cn_step_solves_its_equation():
    m = mesh(2, 4, [3, 2], nu=0.02)
    u = wl.fourier_field([m.coords(0), m.coords(1)], [1, 1], 3, 31)[None]
    dt = 5e-3
    v = ocn.cn_step(m, u, dt)
    R = v - u - 0.5 * dt * (m.rhs(u) + m.rhs(v))
    assert np.abs(R).max() < 1e-14 * np.abs(v).max()


def test_cn_second_order_in_dt():
    nu, a, T = 0.1, 1.25, 0.5
    m = oracle.Mesh(1, 8, [4], [4.0], nu)
    u0 = cole_hopf(m.coords(0), 0.0, nu, a)[None, None]
    ref, _ = m.rk4_forward(u0, 2.5e-4, 2000)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        uT, _ = ocn.cn_forward(m, u0, dt, int(round(T / dt)))
        errs.append(rel(uT, ref))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.2 for r in rates), (errs, rates)


def test_cn_frozen_speed_advection_diffusion():
    nu, T, dt = 1e-3, 0.05, 5e-4
    amp = wl.rng(4).uniform(0.9, 1.0, 5)
    m = mesh(1, 12, [6], nu=nu)
    X = grids(m)

    def exact(t):
        s = 0.0
        for j, aj in enumerate(amp[:3], start=1):
            s = s + aj * np.sin(2 * np.pi * j * (X[0] - 0.1 * t)) * np.exp(-nu * 4 * np.pi ** 2 * j * j * t)
        return s[None, None]

    ubar = np.full((1, 1) + X[0].shape, 0.1)
    _, vT = ocn.cn_tlm(m, ubar, exact(0.0), dt, int(round(T / dt)))
    assert rel(vT, exact(T)) < 1e-7


def test_cn_adjoint_gradient_vs_finite_differences():
    m, u0, target = c1_inputs()
    dt, n, K = wl.C1_DT, 20, 5
    uT, ck = ocn.cn_forward(m, u0, dt, n, K)
    _, lamT = m.misfit(uT, target)
    g = ocn.cn_adjoint(m, ck, dt, n, K, lamT)

    def Phi(u):
        return m.misfit(ocn.cn_forward(m, u, dt, n)[0], target)[0][0]

    for s in range(4):
        d = wl.normal_field(m.shape, 300 + s)
        eps = 1e-4 * np.linalg.norm(u0) / np.linalg.norm(d)
        fd = (8 * (Phi(u0 + eps * d) - Phi(u0 - eps * d)) - (Phi(u0 + 2 * eps * d) - Phi(u0 - 2 * eps * d))) \
            / (12 * eps)
        ad = np.vdot(g, d)
        assert abs(fd - ad) <= 1e-8 * abs(ad), (s, fd, ad)


def test_cn_tangent_linear_adjoint_duality():
    m = mesh(2, 4, [3, 2], nu=0.01)
    u0 = wl.fourier_field([m.coords(0), m.coords(1)], [1, 1], 3, 9)[None]
    du0, lamN = rand(m, 10), rand(m, 11)
    dt, n, K = 2e-3, 6, 3
    _, duN = ocn.cn_tlm(m, u0, du0, dt, n)
    _, ck = ocn.cn_forward(m, u0, dt, n, K)
    lam0 = ocn.cn_adjoint(m, ck, dt, n, K, lamN)
    a, b = np.vdot(lam0, du0), np.vdot(lamN, duN)
    assert abs(a - b) < 1e-12 * abs(b)


def test_cn_checkpointing_is_bitwise_store_all():
    m, u0, target = c1_inputs()
    dt, n = wl.C1_DT, 10
    lams = []
    for K in (1, 5, 10):
        uT, ck = ocn.cn_forward(m, u0, dt, n, K)
        _, lamT = m.misfit(uT, target)
        lams.append(ocn.cn_adjoint(m, ck, dt, n, K, lamT))
    np.testing.assert_array_equal(lams[0], lams[1])
    np.testing.assert_array_equal(lams[0], lams[2])


# ------------------------------------------------------------------------------------------------
# LMVM with More-Thuente steps (Sec. 5) and the 1-D optimal initial condition (Sec. 6.1)
# ------------------------------------------------------------------------------------------------
from oracle import lmvm as olmvm  # noqa: E402


def recovery_problem(steps=800, dt=5e-3):
    """Sec. 6.1: target = Cole-Hopf solution at T = 4 (a = 2), first guess = its initial condition
    plus a Gaussian centred in the middle of the period-4 domain; nu = 0.01, E = 16, N = 8."""
    nu = 0.01
    m = oracle.Mesh(1, 8, [16], [4.0], nu)
    x = m.coords(0)
    exact0 = cole_hopf(x, 0.0, nu, 2.0)[None, None]
    target = cole_hopf(x, steps * dt, nu, 2.0)[None, None]
    guess = exact0 + np.exp(-4 * (x - 2) ** 2)[None, None]
    return m, exact0, target, guess, dt, steps


def test_lmvm_finds_the_minimiser_of_a_quadratic():
    r = wl.rng(50)
    Q, _ = np.linalg.qr(r.normal(size=(30, 30)))
    A = Q @ np.diag(np.logspace(0, 2, 30)) @ Q.T
    b = r.normal(size=30)
    xs = np.linalg.solve(A, b)
    x, hist, reason = olmvm.lmvm(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(30), max_iters=300,
                                 gatol=1e-6)
    # ||x - x*|| <= ||g|| / lambda_min = 1e-6 (eigenvalues in [1, 100])
    assert reason == 1 and np.linalg.norm(x - xs) <= 1e-6
    assert all(h1 < h0 for h0, h1 in zip(hist, hist[1:]))


def test_lmvm_recovers_toward_the_initial_condition():
    m, exact0, target, guess, dt, n = recovery_problem()
    fg = olmvm.objective(m, "rk4", target, dt, n, 50)
    x, hist, reason = olmvm.lmvm(fg, guess, max_iters=15)
    assert reason == 3 and len(hist) == 16
    assert all(h1 < h0 for h0, h1 in zip(hist, hist[1:]))
    assert hist[-1] < 0.05 * hist[0]
    assert np.abs(x - exact0).max() < 0.9 * np.abs(guess - exact0).max()
