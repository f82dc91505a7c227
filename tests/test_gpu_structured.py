"""Structured (sparse) Hamiltonians on the batched path: the FP64 step
norms over the union of the nonzero patterns and the gradient contraction
at the nonzeros of each H_k (Sec. IV / Conclusion: sparse matrices), against
the FP64 oracle and against the dense kernels on the same handle."""
import numpy as np
import pytest

import workloads
from paper_1612_04929_amd import qoc
from test_gpu_parity import check, compare, rel, say

pytestmark = pytest.mark.gpu


def sparse_problem(rng, d, M, N, S, per_row, dt=0.2, scale=1.5):
    """Random Hermitian drift and controls with about `per_row` nonzeros per
    row each (a tridiagonal drift, scattered controls)."""
    p = workloads.random_problem(rng, d=d, M=M, N=N, S=S, dt=dt, scale=scale)
    H0 = np.zeros((d, d), complex)
    i = np.arange(d)
    H0[i, i] = rng.normal(size=d) * scale
    H0[i[:-1], i[:-1] + 1] = rng.normal(size=d - 1) + 1j * rng.normal(size=d - 1)
    H0 = np.triu(H0) + np.triu(H0, 1).conj().T
    Hk = []
    for _ in range(M):
        A = np.zeros((d, d), complex)
        for _ in range(per_row * d // 2):
            r, c = rng.integers(0, d, size=2)
            A[r, c] += rng.normal() + 1j * rng.normal()
        Hk.append((A + A.conj().T) / 2)
    p.H0, p.Hk = H0, np.stack(Hk)
    return p


def test_spin_chain_structured_matches_oracle_and_dense():
    p = workloads.config4().with_steps(24)
    out, ref, e = compare("struct_c4_N24", p)
    check(p, e)
    h = qoc.Problem(p)
    a = h.cost_grad(p.u)
    assert a["structured"] == 1  # diagonal drift, permutation-like controls
    h.set_structure(0)
    b = h.cost_grad(p.u)
    assert b["structured"] == 0
    say(f"[struct] c4 N=24 structured vs dense: grad rel {rel(a['grad'], b['grad']):.2e}")
    assert rel(a["grad"], b["grad"]) <= 1e-5 and abs(a["C"] - b["C"]) <= 1e-12
    assert abs(a["theta_max"] - b["theta_max"]) <= 1e-13 * b["theta_max"]
    h.close()


@pytest.mark.parametrize("d,S,N,per_row,prec", [(70, 2, 40, 3, "fp32"), (100, 3, 33, 2, "fp32"),
                                                (64, 2, 25, 4, "fp64"), (128, 1, 50, 2, "bf16x3")])
def test_random_sparse_structured(d, S, N, per_row, prec):
    rng = np.random.default_rng(900 + d)
    p = sparse_problem(rng, d, 3, N, S, per_row)
    # unions of d^2 / 16 .. d^2 / 4 entries: recorded, structured on request
    out, ref, e = compare(f"struct_d{d}_{prec}", p, precision=prec, structure=1)
    assert out["structured"] == 1
    if prec == "bf16x3":
        assert e["dF"] <= 1e-5 and e["grad_rel"] <= 1e-3, e
    else:
        check(p, e, precision=prec)


def test_default_structure_on_a_denser_pattern():
    # union of d^2 / 8 .. d^2 / 4 entries: recorded and used by default;
    # dense on request
    rng = np.random.default_rng(950)
    p = sparse_problem(rng, 64, 2, 30, 2, per_row=6)
    h = qoc.Problem(p)
    st = h.cost_grad(p.u)
    if not st["structured"]:
        pytest.skip("pattern denser than d^2 / 4 for this seed")
    h.set_structure(0)
    dense = h.cost_grad(p.u)
    say(f"[struct] default: structured={st['structured']} dense={dense['structured']} "
        f"grad rel {rel(st['grad'], dense['grad']):.2e}")
    assert dense["structured"] == 0
    assert rel(st["grad"], dense["grad"]) <= 1e-5
    h.close()
    q = workloads.random_problem(np.random.default_rng(951), d=64, M=2, N=10, S=2)
    h = qoc.Problem(q)  # dense random: no pattern recorded
    with pytest.raises(qoc.QocError):
        h.set_structure(1)
    assert h.cost_grad(q.u)["structured"] == 0
    h.close()
