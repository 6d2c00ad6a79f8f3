"""Crank-Nicolson time integration for the oracle (Sec. 6.3 names the implicit CN scheme; Sec. 2
and Sec. 5: Newton-type nonlinear solves, linear solves for the adjoint).

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`.  Plain and dense: each step solves
    R(v) = v - u - dt/2 (F(u) + F(v)) = 0
by Newton's method with the Jacobian I - dt/2 J(v) assembled column by column from the oracle's
matrix-free J v and factorised by numpy.  The discrete adjoint of the exact step map
(Sec. 4.1, eq. adjtime, for u+ = A(u) defined implicitly) is
    (I - dt/2 J(u+))^T mu = lam_{n+1},   lam_n = mu + dt/2 J(u)^T mu,
with J^T assembled column by column from the oracle's matrix-free J^T w, an independent route from
J.  Sizes are small (a few hundred DOF), so dense algebra stays fast.
"""
import numpy as np


def _one(m):
    return m.with_batch(1) if m.batch != 1 else m


def _columns(apply, n, shape):
    A = np.empty((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[k] = 1.0
        A[:, k] = apply(e.reshape(shape)).ravel()
        e[k] = 0.0
    return A


def jacobian(m, u):
    """Dense J(u) of one batch member (ndof x ndof) from the matrix-free J v."""
    m1 = _one(m)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(m1.shape)
    return _columns(lambda e: m1.jac_vec(u, e), m1.ndof, m1.shape)


def jacobian_transpose(m, u):
    """Dense J(u)^T of one batch member from the matrix-free J^T w."""
    m1 = _one(m)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(m1.shape)
    return _columns(lambda e: m1.jact_vec(u, e), m1.ndof, m1.shape)


def cn_step(m, u, dt, max_newton=30):
    """One CN step of one batch member; Newton from the explicit-Euler predictor, iterated until
    the update is at rounding level."""
    m1 = _one(m)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(m1.shape)
    base = u + 0.5 * dt * m1.rhs(u)
    v = u + dt * m1.rhs(u)
    n = m1.ndof
    for _ in range(max_newton):
        R = (v - base - 0.5 * dt * m1.rhs(v)).ravel()
        A = np.eye(n) - 0.5 * dt * jacobian(m1, v)
        dv = np.linalg.solve(A, R)
        v = v - dv.reshape(m1.shape)
        if np.abs(dv).max() <= 4e-16 * max(1.0, np.abs(v).max()):
            return v
    raise RuntimeError("CN Newton iteration did not converge")


def cn_forward(m, u0, dt, nsteps, ckpt_every=None):
    """(u(T), checkpoints [nsteps/K][batch][...] or None), as the RK routines of the oracle."""
    u = np.array(u0, dtype=np.float64).reshape(m.shape)
    ck = np.zeros((nsteps // ckpt_every,) + m.shape) if ckpt_every else None
    for b in range(m.batch):
        for k in range(nsteps):
            if ck is not None and k % ckpt_every == 0:
                ck[k // ckpt_every, b] = u[b]
            u[b] = cn_step(m, u[b], dt)[0]
    return u, ck


def cn_adjoint(m, ckpt, dt, nsteps, ckpt_every, lamT):
    """lambda_0 from lambda_N through the discrete CN adjoint, recomputing each segment of K steps
    from its checkpoint."""
    lam = np.array(lamT, dtype=np.float64).reshape(m.shape)
    m1 = _one(m)
    K = ckpt_every
    for b in range(m.batch):
        for sg in range(nsteps // K - 1, -1, -1):
            states = [ckpt[sg, b][None]]
            for _ in range(K):
                states.append(cn_step(m1, states[-1], dt))
            for k in range(K - 1, -1, -1):
                At = np.eye(m1.ndof) - 0.5 * dt * jacobian_transpose(m1, states[k + 1])
                mu = np.linalg.solve(At, lam[b].ravel()).reshape(m1.shape)
                lam[b] = (mu + 0.5 * dt * m1.jact_vec(states[k], mu))[0]
    return lam


def cn_tlm(m, u0, du0, dt, nsteps):
    """Tangent-linear CN: du_{n+1} = (I - dt/2 J(u_{n+1}))^{-1} (I + dt/2 J(u_n)) du_n."""
    u = np.array(u0, dtype=np.float64).reshape(m.shape)
    du = np.array(du0, dtype=np.float64).reshape(m.shape)
    m1 = _one(m)
    for b in range(m.batch):
        for _ in range(nsteps):
            un = u[b][None]
            up = cn_step(m1, un, dt)
            rhs = du[b][None] + 0.5 * dt * m1.jac_vec(un, du[b][None])
            A = np.eye(m1.ndof) - 0.5 * dt * jacobian(m1, up)
            du[b] = np.linalg.solve(A, rhs.ravel()).reshape(m1.shape)[0]
            u[b] = up[0]
    return u, du
