"""Host logic of the batch runner: the truncation-bound check used to keep
fixed (p, n) pairs valid agrees with the (p, n) rule."""
import numpy as np
import pytest

import oracle
from paper_1612_04929_amd.batch import taylor_ok


@pytest.mark.parametrize("theta", [0.0, 1e-3, 0.034, 0.37, 0.81, 1.22, 4.66, 5.52, 12.0])
@pytest.mark.parametrize("tol", [1e-10, 1e-15])
def test_taylor_ok_matches_rule(theta, tol):
    p, n = oracle.taylor_select(theta, tol)
    assert taylor_ok(p, n, theta, tol)
    # the chosen pair is the cheapest: no pair with fewer products holds
    G = p - 1 + n
    for n2 in range(0, 40):
        for p2 in range(2, 31):
            if p2 - 1 + n2 < G:
                assert not taylor_ok(p2, n2, theta, tol)


def test_taylor_ok_monotone_in_theta():
    p, n = oracle.taylor_select(1.0, 1e-10)
    thetas = np.linspace(0.0, 3.0, 61)
    ok = [taylor_ok(p, n, t, 1e-10) for t in thetas]
    # valid up to some theta, invalid beyond it
    first_bad = ok.index(False)
    assert all(ok[:first_bad]) and not any(ok[first_bad:])


def test_tuner_candidate_intervals():
    from paper_1612_04929_amd.tune import candidate_intervals
    assert candidate_intervals(1) == [1]
    c = candidate_intervals(5000)
    assert c == sorted(set(c)) and 64 in c and all(1 <= x <= 5000 for x in c)
    assert all(x & (x - 1) == 0 for x in c)
