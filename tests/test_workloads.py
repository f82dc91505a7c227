"""Host checks of the seeded input generators (no method arithmetic)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_config_shapes_hermitian_deterministic(name):
    p = workloads.make_config(name)
    q = workloads.make_config(name)
    assert p.H0.shape == (p.d, p.d) and p.Hk.shape == (p.M, p.d, p.d)
    assert p.u.shape == (p.M, p.N) and p.psi0.shape == (p.S, p.d)
    for H in [p.H0, *p.Hk]:
        assert np.max(np.abs(H - H.conj().T)) == 0.0
    assert np.array_equal(p.u, q.u) and np.array_equal(p.psiT, q.psiT)
    assert np.allclose(np.linalg.norm(p.psi0, axis=1), 1.0)
    assert np.allclose(np.linalg.norm(p.psiT, axis=1), 1.0)


@pytest.mark.slow
def test_config4_shapes():
    p = workloads.config4()
    assert (p.d, p.M, p.N, p.S) == (512, 18, 1000, 8)
    assert np.max(np.abs(p.H0 - np.diag(np.diag(p.H0)))) == 0.0


def test_config5_ranges():
    insts = workloads.config5(count=32)
    for p in insts:
        assert 2 <= p.d <= 128 and 100 <= p.N <= 3000 and 2 <= p.M <= 6
        for H in [p.H0, *p.Hk]:
            assert np.max(np.abs(H - H.conj().T)) < 1e-15


def test_golden_c1_matches_oracle():
    with open(os.path.join(HERE, "golden", "c1_oracle.json")) as f:
        g = json.load(f)
    out = oracle.cost_grad(workloads.config1())
    assert abs(out["C"] - g["C"]) < 1e-14
    assert np.max(np.abs(out["grad"] - np.array(g["grad"]))) < 1e-14
