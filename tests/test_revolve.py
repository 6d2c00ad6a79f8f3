"""Host-side pins of the binomial (revolve) checkpointing schedule in libsem (Sec. 5.3 recompute;
no GPU needed): its number of forward steps is the least any schedule with the same number of
snapshot slots can achieve, and replaying it symbolically visits every adjoint step once, in
reverse order, each on its own start state."""
import functools
import math
import sys

import pytest

sys.path.insert(0, __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__))))


@pytest.fixture(scope="module")
def P():
    import paper_1806_01422_amd as P
    return P


@functools.lru_cache(maxsize=None)
def least_advances(l, s):
    """Brute force over every first split: reverse l steps with s slots (the start state's included)."""
    if l == 1:
        return 0
    if s == 1:
        return l * (l - 1) // 2
    return min(m + least_advances(l - m, s - 1) + least_advances(m, s) for m in range(1, l))


def replay(acts, n, snaps):
    """Run the schedule on step indices instead of states."""
    slots, cur, order = {0: 0}, None, []
    for kind, arg in acts:
        if kind == "restore":
            assert arg in slots, "restore of an empty slot"
            cur = slots[arg]
        elif kind == "advance":
            assert arg >= 1
            cur += arg
        elif kind == "store":
            assert 0 < arg < snaps
            slots[arg] = cur
        else:
            assert cur == arg, "adjoint step on the wrong state"
            order.append(arg)
    assert order == list(range(n - 1, -1, -1))


@pytest.mark.parametrize("snaps", [1, 2, 3, 4, 6])
def test_schedule_is_optimal_and_valid(P, snaps):
    for n in range(1, 61):
        acts, adv = P.revolve_plan(n, snaps)
        assert adv == least_advances(n, snaps), (n, snaps)
        assert adv == sum(a for k, a in acts if k == "advance")
        replay(acts, n, snaps)


def test_closed_form_count(P):
    # Griewank: with t the least repetition number such that C(s + t, s) >= n, the least number
    # of forward steps is t n - C(s + t, s + 1)
    for snaps in (2, 3, 5, 10):
        for n in (7, 50, 200, 1000):
            t = 0
            while math.comb(snaps + t, snaps) < n:
                t += 1
            acts, adv = P.revolve_plan(n, snaps)
            assert adv == t * n - math.comb(snaps + t, snaps + 1), (n, snaps)
            if n <= 200:
                replay(acts, n, snaps)


def test_plan_errors(P):
    with pytest.raises(P.SemError):
        P.revolve_plan(0, 3)
    with pytest.raises(P.SemError):
        P.revolve_plan(10, 0)
