"""Limited-memory variable-metric (LMVM) minimisation of the terminal misfit over the initial
condition, for the oracle (Sec. 5: directions from a limited-memory BFGS approximation, step
lengths from the More-Thuente line search; Sec. 6.1: recover u_0 from the state at time T).

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`.  Plain numpy on the oracle's trajectories
and adjoints; the line search is SciPy's implementation of the More-Thuente method (DCSRCH), used
as a library primitive.  The algorithm's choices, which the GPU library follows too:
  - the first direction (and any restart) is -g, tried with a step of length 1 in the 2-norm;
  - later directions come from the two-loop recursion over the last `memory` pairs (s, y) with
    s.y > 0, initial inverse Hessian (s.y / y.y) I, tried with step 1;
  - a direction with g.d >= 0 restarts from -g and drops the pairs;
  - when the line search ends on an earlier step than its last trial, that step is evaluated again;
  - the iteration stops at ||g|| <= gatol, ||g|| <= grtol |Phi|, max_iters, or a failed search.
"""
import numpy as np


def _trajectory(m, scheme, u0, dt, nsteps, K):
    if scheme == "cn":
        from . import cn
        return cn.cn_forward(m, u0, dt, nsteps, K)
    if scheme == "rk4":
        return m.rk4_forward(u0, dt, nsteps, K)
    return m.erk_forward(scheme, u0, dt, nsteps, K)


def _adjoint(m, scheme, ck, dt, nsteps, K, lamT):
    if scheme == "cn":
        from . import cn
        return cn.cn_adjoint(m, ck, dt, nsteps, K, lamT)
    if scheme == "rk4":
        return m.rk4_adjoint(ck, dt, nsteps, K, lamT)
    return m.erk_adjoint(scheme, ck, dt, nsteps, K, lamT)


def objective(m, scheme, target, dt, nsteps, K):
    """Phi(u0) = 1/2 sum (u(T) - u*)^2 and its gradient (discrete adjoint)."""
    def fg(u0):
        uT, ck = _trajectory(m, scheme, u0, dt, nsteps, K)
        r = uT - target
        return 0.5 * float(np.vdot(r, r)), _adjoint(m, scheme, ck, dt, nsteps, K, r)
    return fg


def lmvm(fg, x0, max_iters=50, memory=5, gatol=1e-10, grtol=1e-10, ftol=1e-4, gtol=0.9, xtol=1e-10, max_evals=30):
    """Returns (x, history of Phi, reason) with the GPU library's reason codes."""
    from scipy.optimize._dcsrch import DCSRCH
    x = np.array(x0, dtype=np.float64)
    f, g = fg(x)
    hist = [f]
    S, Y, rho = [], [], []
    k = 0
    while True:
        gn = float(np.sqrt(np.vdot(g, g)))
        if gn <= gatol:
            return x, hist, 1
        if gn <= grtol * abs(f):
            return x, hist, 2
        if k >= max_iters:
            return x, hist, 3
        if S:
            q = g.copy()
            alpha = []
            for s, y, r in zip(reversed(S), reversed(Y), reversed(rho)):
                a = r * float(np.vdot(s, q))
                q = q - a * y
                alpha.append(a)
            q = q * (float(np.vdot(S[-1], Y[-1])) / float(np.vdot(Y[-1], Y[-1])))
            for (s, y, r), a in zip(zip(S, Y, rho), reversed(alpha)):
                b = r * float(np.vdot(y, q))
                q = q + (a - b) * s
            d = -q
            gd = float(np.vdot(g, d))
            stp0 = 1.0
        if not S or not gd < 0:
            d = -g
            gd = -gn * gn
            stp0 = 1.0 / gn
            S, Y, rho = [], [], []
        cache = {}

        def phi(t):
            if t not in cache:
                cache[t] = fg(x + t * d)
            return cache[t][0]

        def dphi(t):
            phi(t)
            return float(np.vdot(cache[t][1], d))

        ls = DCSRCH(phi, dphi, ftol, gtol, xtol, 0.0, 1e10)
        stp, _, _, task = ls(stp0, f, gd, maxiter=max_evals)
        if stp is None or not (str(task).startswith("CONV") or str(task).startswith("WARN")
                               or str(task).startswith("b'CONV") or str(task).startswith("b'WARN")):
            return x, hist, -1
        ft, gt = fg(x + stp * d) if stp not in cache else cache[stp]
        if not ft < f:
            return x, hist, -1
        xt = x + stp * d
        s, y = xt - x, gt - g
        sy = float(np.vdot(s, y))
        if sy > 0:
            S.append(s), Y.append(y), rho.append(1.0 / sy)
            if len(S) > memory:
                S.pop(0), Y.pop(0), rho.pop(0)
        x, g, f = xt, gt, ft
        hist.append(f)
        k += 1
