"""GPU test of sem_rk4_forward_noalloc, the RK4 forward that allocates nothing (its stage states
live in the library's file-scope device scratch array): through the C ABI, two calls in a row, the
second on a smaller state, each bitwise equal to sem_rk4_forward (the same launches and
coefficients), with no change in the device's free memory across the call, and a state beyond
the scratch's limit rejected with an error that names it."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1806_01422_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def field(P, dim, N, E, batch, seed):
    m = oracle.Mesh(dim, N, list(E), [1.0] * dim, 0.01, batch)
    xs = [m.coords(k) for k in range(dim)]
    u = np.stack([wl.fourier_field(xs, [1.0] * dim, 3, seed + b) for b in range(batch)])
    return torch.from_numpy(u).cuda()


def test_noalloc_forward_matches_forward(P):
    n, K = 12, 4
    # the first call on a 3-D state of 1.2 M values (the tuned 3-D kernel), the second on a
    # smaller 2-D one (the tuned 2-D kernel), then a 1-D one (the generic kernels)
    for dim, N, E, batch in [(3, 7, (8, 4, 4), 1), (2, 7, (8, 3), 2), (1, 8, (16,), 3)]:
        note(f"allocation-free RK4 forward: dim={dim} N={N} E={E} batch={batch}")
        dt = wl.stable_dt(dim, N, max(E), 1.0, 0.01)  # a stable step: the values stay finite
        c = P.Context(dim, N, list(E), [1.0] * dim, 0.01, batch=batch)
        U = field(P, dim, N, E, batch, 3)
        u = U.clone()
        ck = torch.empty((n // K,) + c.shape, dtype=torch.float64, device="cuda")
        # the first launch of a kernel in the process loads its code object (device memory the
        # runtime allocates once); the free memory is compared around the second call
        c.rk4_forward_noalloc(U.clone(), dt, 1)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        c.rk4_forward_noalloc(u, dt, n, K, ck)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        ref_T, ref_ck = c.rk4_forward(U, dt, n, K)
        assert bool(torch.isfinite(ref_T).all())
        assert torch.equal(u, ref_T)
        assert torch.equal(ck, ref_ck)
        # again on the same context without checkpoints: the scratch keeps the last call's
        # contents, which must not leak into the result
        u2 = U.clone()
        c.rk4_forward_noalloc(u2, dt, n)
        assert torch.equal(u2, ref_T)
        c.close()


def test_noalloc_rejects_states_beyond_the_scratch(P):
    # 64 fields of the 2-D 64^2 N=7 mesh: 25.7 M values per state, four of them exceed 64 MiB
    c = P.Context(2, 7, [64, 64], [1.0, 1.0], 1e-3, batch=64)
    u = c.empty().zero_()
    with pytest.raises(P.SemError, match="scratch"):
        c.rk4_forward_noalloc(u, 1e-4, 2)
    c.close()
