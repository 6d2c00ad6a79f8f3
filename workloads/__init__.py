"""Seeded synthetic workloads for the SEM Burgers path.

This module only draws random numbers and evaluates plain Fourier sums at coordinates handed to
it; it holds none of the discretisation's arithmetic (no GLL tables, no operators), so the CPU
oracle and the HIP library can both be fed from it without sharing code.

Recipes (all seeds fixed):
  * Fourier field: for every integer wave vector k with 0 < |k| <= K, in lexicographic order, and
    every component c, draw (a, b) ~ N(0, 1); u_c(x) = sum_k (a cos(2 pi k.x/L) + b sin(2 pi k.x/L))
    / |k|^2.  Optionally scaled so that max |u| over all components is 1.
  * Normal field: i.i.d. N(0, 1) per unique node and component (the w and v vectors).
  * Element-local normal field: i.i.d. N(0, 1) per element-local node (the 1-D perturbation, which
    the caller projects onto the continuous space).
"""
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice(dim: int, K: int) -> List[Tuple[int, ...]]:
    """Integer wave vectors 0 < |k|_2 <= K in lexicographic order."""
    out = []
    for k in np.ndindex(*([2 * K + 1] * dim)):
        kk = tuple(int(v) - K for v in k)
        r2 = sum(v * v for v in kk)
        if 0 < r2 <= K * K:
            out.append(kk)
    return out


def fourier_field(coords: Sequence[np.ndarray], L: Sequence[float], K: int, seed: int,
                  normalize: bool = True) -> np.ndarray:
    """Random smooth periodic vector field with dim components on the tensor grid given by the
    1-D coordinate arrays coords[d] (x first).  Returns [C][nz][ny][nx] (unused axes dropped)."""
    dim = len(coords)
    ks = lattice(dim, K)
    g = rng(seed)
    # coefficient tensors c[comp][kx][ky][kz] of sum c_k exp(2 pi i k.x / L); a cos + b sin = Re((a - ib) e)
    coef = np.zeros((dim,) + (2 * K + 1,) * dim, dtype=np.complex128)
    for k in ks:
        r2 = float(sum(v * v for v in k))
        idx = tuple(v + K for v in k)
        for c in range(dim):
            a, b = g.standard_normal(2)
            coef[(c,) + idx] += (a - 1j * b) / r2
    kr = np.arange(-K, K + 1)
    out = []
    for c in range(dim):
        t = coef[c]
        # contract direction 0 (x) first: t[kx,ky,kz] -> t[x,ky,kz] etc.; finally axes are (x, y, z)
        for d in range(dim):
            e = np.exp(2j * np.pi * np.outer(kr, coords[d]) / L[d])  # [k, x_d]
            t = np.tensordot(t, e, axes=([0], [0]))  # consumes leading k axis, appends x_d axis
        fc = t.real
        out.append(fc.transpose(tuple(reversed(range(dim)))))  # -> [z][y][x]
    u = np.ascontiguousarray(np.stack(out))
    if normalize:
        u /= np.abs(u).max()
    return u


def normal_field(shape: Sequence[int], seed: int) -> np.ndarray:
    return rng(seed).standard_normal(tuple(shape))


# ------------------------------------------------------------------------------------------------
# Workload configurations (sizes of the paper's 3-D runs are 16^3 and 64^3 elements at 8 points per
# direction; the configurations below are the single-GPU workloads measured here).
# ------------------------------------------------------------------------------------------------
@dataclass
class Problem:
    dim: int
    N: int
    E: Tuple[int, ...]
    L: Tuple[float, ...]
    nu: float
    batch: int = 1

    @property
    def n(self):
        return tuple(e * self.N for e in self.E)

    @property
    def nodes(self):
        return int(np.prod(self.n))

    @property
    def ndof(self):
        return self.nodes * self.dim

    @property
    def shape(self):
        return (self.batch, self.dim) + tuple(reversed(self.n))


# C1: 1-D periodic [0, 2 pi], E=16, N=8, nu=0.01; RK4 dt=1e-3, 100 steps.
C1 = Problem(dim=1, N=8, E=(16,), L=(2 * np.pi,), nu=0.01)
C1_DT, C1_STEPS = 1e-3, 100
C1_SEEDS = dict(ic=1, target=2, w=3)

# C2: 2-D periodic unit square, 64x64 elements, N=7, nu=1e-3; Fourier |k| <= 8.
C2 = Problem(dim=2, N=7, E=(64, 64), L=(1.0, 1.0), nu=1e-3)
C2_SEEDS = dict(u=10, v=11, w=12)
C2_K = 8

# C3: 3-D periodic unit cube, 32^3 elements, N=7, nu=1e-3; Fourier |k| <= 6.
C3 = Problem(dim=3, N=7, E=(32, 32, 32), L=(1.0, 1.0, 1.0), nu=1e-3)
C3_SEEDS = dict(u=20, w=21, v=22)
C3_K = 6

# C4: C2 mesh, RK4 dt=2e-4, 500 steps, checkpoint every 50, batch of 64 initial conditions
# (IC seeds 100..163, target seeds 200..263, finite-difference directions 300..315).
C4 = Problem(dim=2, N=7, E=(64, 64), L=(1.0, 1.0), nu=1e-3, batch=64)
C4_DT, C4_STEPS, C4_CKPT = 2e-4, 500, 50
C4_IC_SEED0, C4_TARGET_SEED0, C4_FD_SEED0 = 100, 200, 300


# C5: 128 independent 2-D problems of uneven size and order.
@dataclass
class BatchedProblem:
    E: int
    N: int
    nu: float
    dt: float
    ic_seed: int
    target_seed: int


C5_COUNT, C5_SEED, C5_STEPS = 128, 40, 200
# Gradient descent on the initial conditions: 20 iterations of u0 <- u0 - alpha d / max|d| with
# the mass-weighted direction d = W g, W = M / mean(M) per problem (M the assembled diagonal
# mass): every problem's initial field moves by at most alpha per iteration.
C5_ITERS, C5_ALPHA = 20, 0.05
C5_E = (8, 16, 32, 64)
C5_N = (5, 7, 9)
C5_K = 4
# Horizon cap of the batched set: 200 steps end by T = 0.02, about half the time 1 / (2 pi K max|u0|)
# ~ 0.04 in which the steepest mode of the initial field (K = 4, max|u0| = 1) turns into a shock
# the meshes cannot resolve at the low viscosities of the set.
C5_T_MAX = 0.02


def stable_dt(dim: int, N: int, E: int, L: float, nu: float, umax: float = 1.0, safety: float = 0.5) -> float:
    """Fixed RK4 step for a periodic SEM Burgers problem from rule-of-thumb spectral-radius
    estimates of the 1-D operators (diffusion ~0.55 N^4/h^2, advection ~0.45 N^2/h) and the RK4
    stability interval (2.78 on the negative real axis, 2.8 on the imaginary axis)."""
    h = L / E
    rho_k = 0.55 * N ** 4 / h ** 2
    rho_a = 0.45 * N ** 2 / h
    lim = min(2.78 / (dim * nu * rho_k), 2.8 / (dim * umax * rho_a))
    return safety * lim


def c5_problems(count: int = C5_COUNT, seed: int = C5_SEED) -> List[BatchedProblem]:
    g = rng(seed)
    out = []
    for p in range(count):
        E = int(g.choice(C5_E))
        N = int(g.choice(C5_N))
        nu = float(10.0 ** g.uniform(-4.0, -2.0))
        dt = min(stable_dt(2, N, E, 1.0, nu), C5_T_MAX / C5_STEPS)
        out.append(BatchedProblem(E=E, N=N, nu=nu, dt=dt, ic_seed=41 + p, target_seed=1041 + p))
    return out
