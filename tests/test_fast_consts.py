"""The order-9 coefficient constants that the build writes for the tuned 2-D kernel
(_build/gen/fast_consts.h, from the library's table routine), checked on the CPU against the GLL
tables computed separately in extended precision (tests/test_rounding_floor.py's gll_ext) and
against the oracle's: the even/odd blocks of D (Sec. 3.3 sum factorisation with the GLL
differentiation matrix), the weights, the inverse assembled 1-D mass and the line-end rows."""
import os
import re

import numpy as np
import pytest

import oracle
from test_rounding_floor import LD, gll_ext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1806_01422_amd", "_build", "gen", "fast_consts.h")


def constants():
    if not os.path.exists(HEADER):
        from paper_1806_01422_amd import build
        build.gen_headers()
    text = open(HEADER).read()
    body = text[text.index("struct FastConst<10>"):]
    out = {}
    for name, vals in re.findall(r"static constexpr double (\w+)\[\d+\] = \{([^}]*)\}", body):
        out[name] = np.array([float.fromhex(v.strip()) for v in vals.split(",")])
    return out


def expected(N, xi, w, D):
    P, H = N + 1, (N + 1) // 2
    A = np.array([[(D[i, m] - D[i, P - 1 - m]) / 2 for m in range(H)] for i in range(H)]).ravel()
    B = np.array([[(D[i, m] + D[i, P - 1 - m]) / 2 for m in range(H)] for i in range(H)]).ravel()
    imq = np.array([1 / (2 * w[0]) if q in (0, P - 1) else 1 / w[q] for q in range(P)])
    L = P - 1
    Kw = np.array([sum(D[m, L] * w[m] * D[m, n] for m in range(P)) / w[L] for n in range(P)])
    Dw = np.array([D[n, L] * w[n] / w[L] for n in range(P)])
    return dict(A=A, B=B, w=np.asarray(w), imq=imq, D7=np.asarray(D[L, :]), Kw=Kw, Dw=Dw)


@pytest.mark.skipif(np.finfo(LD).eps > 1e-18, reason="needs an extended long double")
def test_order9_constants_match_extended_gll():
    c = constants()
    xi, w, D = gll_ext(9)
    ref = expected(9, xi, w, D)
    assert set(c) == set(ref)
    for k, v in ref.items():
        v = np.asarray(v, dtype=LD)
        # within a few FP64 ulps of the row's largest entry (the scale the contractions see); an
        # entry that cancels to a small value, such as Kw[0] = -1/2, carries the rounding of the
        # FP64 D it is formed from (1.8e-15 there)
        err = np.abs(c[k].astype(LD) - v) / np.abs(v).max()
        assert float(err.max()) < 1e-15, (k, float(err.max()))


def test_order9_constants_match_oracle_gll():
    c = constants()
    ref = expected(9, *oracle.gll(9))
    for k, v in ref.items():
        scale = np.abs(v).max()
        assert np.abs(c[k] - v).max() < 1e-14 * scale, k
