"""State-mode action form (QOC_PROP_ACTION): the Sec. III approximant applied
to the propagated columns by matrix-vector products (Sec. IV), no step
propagator formed, against the FP64 oracle (exact exponentials, exact
gradient) at the FP32 / FP64 parity bars:

* the spin-chain workload (d = 512, S = 8, 18 controls) at a reduced
  horizon, and its (p, n) against the oracle's rule for this form;
* the transmon-cavity workload (d = 128, level penalty) at a reduced
  horizon, FP32 and FP64;
* random sparse problems: padded d above 512 (two rows per thread),
  ragged d, forbidden states with the time-optimal term, incoherent
  fidelity, no controls;
* a dense small problem (every row full);
* the first-order gradient mode against the oracle's;
* the same polynomial as the matrix path at a fixed (p, n);
* bitwise repeatability, and the shapes it rejects.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1612_04929_amd import qoc
from test_gpu_parity import check, compare, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_case(name, prob, precision="fp32", **kw):
    out, ref, e = compare(name, prob, precision=precision, propagation="action", **kw)
    assert out["propagation"] == qoc.QOC_PROP_ACTION
    check(prob, e, precision)
    return out, ref, e


def test_spin_chain_reduced_horizon_and_rule():
    prob = workloads.config4().with_steps(40)
    out, ref, e = run_case("c4_action_N40", prob)
    # the form's own (p, n) rule on the same FP64 theta_max
    assert (out["p"], out["n"]) == oracle.action_select(ref["theta_max"], 1e-10), e


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_transmon_cavity_reduced_horizon(precision):
    prob = workloads.config3().with_steps(150)
    out, ref, e = run_case(f"c3_action_N150_{precision}", prob, precision)
    assert (out["p"], out["n"]) == oracle.action_select(ref["theta_max"],
                                                        1e-15 if precision == "fp64" else 1e-10)


@pytest.mark.parametrize("d,M,N,S,extra", [
    (600, 3, 12, 2, {}),                                         # two rows per thread
    (37, 4, 61, 3, {"fid_mode": "incoherent"}),                  # ragged d
    (50, 3, 40, 2, {"n_forbidden": 2, "alpha_time": 0.4}),       # per-step sources
    (40, 0, 30, 2, {}),                                          # no controls
])
def test_random_sparse(d, M, N, S, extra):
    rng = np.random.default_rng(2000 + d + N)
    prob = workloads.sparse_problem(rng, d, M, N, S, dt=0.15, **extra)
    run_case(f"sparse_d{d}_M{M}", prob)


def test_dense_small():
    rng = np.random.default_rng(2100)
    prob = workloads.random_problem(rng, d=20, M=3, N=50, S=2, dt=0.2, scale=1.5)
    run_case("dense_d20_action", prob)


def test_first_order_mode():
    rng = np.random.default_rng(2200)
    prob = workloads.sparse_problem(rng, 90, 3, 50, 2, dt=0.15)
    h = qoc.Problem(prob, propagation="action")
    h.set_gradient(qoc.QOC_GRAD_FIRST_ORDER)
    out = h.cost_grad(prob.u)
    h.close()
    ref = oracle.gradient_first_order(prob)
    say(f"[action] first-order vs oracle {rel(out['grad'], ref):.2e}")
    assert rel(out["grad"], ref) <= 1e-4


def test_same_polynomial_as_matrix_path():
    """At a fixed (p, n) both forms evaluate T_p(X_j / 2^n)^(2^n): cost and
    gradient agree to FP32 rounding."""
    prob = workloads.config2().with_steps(300)
    res = {}
    for prop in ("matrix", "action"):
        h = qoc.Problem(prob, propagation=prop, taylor_pn=(6, 1))
        res[prop] = h.cost_grad(prob.u)
        h.close()
    a, m = res["action"], res["matrix"]
    dG = rel(a["grad"], m["grad"])
    say(f"[action] vs matrix path at (6, 1): dC={abs(a['C'] - m['C']):.2e} grad_rel={dG:.2e}")
    assert (a["p"], a["n"]) == (6, 1)
    assert abs(a["C"] - m["C"]) <= 2e-6 * (1 + abs(m["C"]))
    assert dG <= 2e-5


def test_repeatable_and_rejected_shapes():
    rng = np.random.default_rng(2300)
    prob = workloads.sparse_problem(rng, 70, 2, 30, 2)
    h = qoc.Problem(prob, propagation="action")
    x, y = h.cost_grad(prob.u), h.cost_grad(prob.u)
    h.close()
    assert x["C"] == y["C"] and np.array_equal(x["grad"], y["grad"])
    # bf16x3 has no products to split; segments have no stacks to segment
    with pytest.raises(qoc.QocError) as ei:
        qoc.Problem(prob, precision="bf16x3", propagation="action")
    assert ei.value.status == -7
    with pytest.raises(qoc.QocError) as ei:
        qoc.Problem(prob, propagation="action", segment_steps=8)
    assert ei.value.status == -7
    # a dense d = 64 union pattern: 64 nonzeros per row
    dense = workloads.random_problem(rng, d=64, M=2, N=10, S=1)
    with pytest.raises(qoc.QocError) as ei:
        qoc.Problem(dense, propagation="action")
    assert ei.value.status == -7
