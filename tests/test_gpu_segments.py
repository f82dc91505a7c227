"""Memory-lean mode (time segments): every per-step stack holds one segment
and the backward pass forms each segment's exponentials again.

* Against the FP64 oracle at the FP32 / FP64 parity bars (the oracle keeps
  every propagator; the segmented path must reach the same cost and exact
  gradient), with ragged segments (N not a multiple of the segment length),
  ragged blocks, a checkpoint interval that is not a power of two, penalties,
  forbidden states with the time-optimal term, structured Hamiltonians and
  the first-order gradient mode.
* Against the same handle configuration without segments: the per-step
  values are formed by the same kernels, so cost, penalties and gradient
  agree to FP32 rounding of the costate at each segment's first step (it is
  formed from the step instead of from the block product).
* Memory: the handle's device bytes fall with the segment length.
* Degenerate settings: a segment at least N long is one segment; a
  negative length and a small-d handle are rejected.
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


CASES = [
    # name, d, M, N, S, L, segment_steps, precision, extras
    ("d70_L8_seg24", 70, 3, 90, 2, 8, 24, "fp32", {}),
    ("d100_L7_seg20", 100, 3, 75, 1, 7, 20, "fp32", {}),        # Ns = 21, L not 2^k
    ("d64_ext_seg16", 64, 2, 70, 2, 8, 16, "fp32", dict(n_forbidden=2, alpha_time=0.3)),
    ("d64_fp64_seg32", 64, 2, 80, 2, 16, 32, "fp64", {}),
    ("d80_bf16x3_seg16", 80, 2, 64, 2, 8, 16, "bf16x3", {}),
    ("d260_wide_seg12", 260, 2, 36, 1, 4, 12, "fp32", {}),      # per-step sweep launches
]


def make(d, M, N, S, seed, **extra):
    rng = np.random.default_rng(seed)
    return workloads.random_problem(rng, d=d, M=M, N=N, S=S, dt=0.2, scale=1.5, **extra)


@pytest.mark.parametrize("name,d,M,N,S,L,seg,prec,extra", CASES, ids=[c[0] for c in CASES])
def test_segments_match_oracle_and_whole_horizon(name, d, M, N, S, L, seg, prec, extra):
    prob = make(d, M, N, S, 1500 + d + N, **extra)
    ref = oracle.cost_grad(prob)
    out, _, e = compare(name, prob, precision=prec, oracle_out=ref, checkpoint_every=L,
                        segment_steps=seg)
    assert out["segments"] == -(-N // (-(-seg // L) * L)), out["segments"]
    if prec == "bf16x3":
        assert e["dF"] <= 1e-5 and e["grad_rel"] <= 1e-3, e
    else:
        check(prob, e, prec)
    # the same handle configuration over the whole horizon
    h = qoc.Problem(prob, precision=prec, checkpoint_every=L)
    whole = h.cost_grad(prob.u)
    h.close()
    assert whole["segments"] == 1
    tol = 1e-12 if prec == "fp64" else 2e-6
    dG = rel(out["grad"], whole["grad"])
    say(f"[segments] {name}: vs whole horizon dC={abs(out['C'] - whole['C']):.2e} "
        f"dc={np.max(np.abs(out['c'] - whole['c'])):.2e} grad_rel={dG:.2e}")
    assert abs(out["C"] - whole["C"]) <= tol * (1 + abs(whole["C"]))
    assert np.max(np.abs(out["c"] - whole["c"])) <= tol
    assert dG <= (1e-10 if prec == "fp64" else 1e-5)
    # the forward pass alone: the states of every segment
    assert out["p"] == whole["p"] and out["n"] == whole["n"]


def test_segments_structured_and_first_order():
    """The spin-chain workload (structured contraction) at a reduced
    horizon, and the first-order gradient mode, each with segments, against
    the same handles over the whole horizon (the structured path's parity
    with the oracle is covered by its own tests)."""
    prob = workloads.config4().with_steps(48)
    say("[segments] c4 N=48 structured, segments of 16")
    res = {}
    for seg in (0, 16):
        h = qoc.Problem(prob, precision="fp32", checkpoint_every=8, segment_steps=seg)
        a = h.cost_grad(prob.u)
        h.set_gradient(qoc.QOC_GRAD_FIRST_ORDER)
        b = h.cost_grad(prob.u)
        h.close()
        assert a["structured"] == 1
        res[seg] = (a, b)
    for i in range(2):
        x, y = res[16][i], res[0][i]
        dG = rel(x["grad"], y["grad"])
        say(f"[segments] c4 mode {i}: dC={abs(x['C'] - y['C']):.2e} grad_rel={dG:.2e}")
        assert abs(x["C"] - y["C"]) <= 2e-6 * (1 + abs(y["C"]))
        assert dG <= 1e-5
    assert res[16][0]["segments"] == 3


def test_segments_first_order_matches_oracle():
    prob = make(70, 3, 60, 2, 1600)
    ref = oracle.gradient_first_order(prob)
    h = qoc.Problem(prob, precision="fp32", checkpoint_every=4, segment_steps=12)
    h.set_gradient(qoc.QOC_GRAD_FIRST_ORDER)
    out = h.cost_grad(prob.u)
    h.close()
    h = qoc.Problem(prob, precision="fp32", checkpoint_every=4)
    h.set_gradient(qoc.QOC_GRAD_FIRST_ORDER)
    whole = h.cost_grad(prob.u)
    h.close()
    assert out["segments"] == 5
    assert rel(out["grad"], whole["grad"]) <= 1e-5
    assert rel(out["grad"], ref) <= 1e-4


def test_segments_reduce_device_memory():
    prob = make(128, 2, 256, 1, 1700)
    sizes = {}
    for seg in (0, 64, 16):
        h = qoc.Problem(prob, precision="fp32", checkpoint_every=16, segment_steps=seg)
        out = h.cost_grad(prob.u)
        sizes[seg] = out["device_bytes"]
        h.close()
    say(f"[segments] device bytes d=128 N=256: {sizes}")
    # the stacks dominate: a quarter / a sixteenth of the steps
    assert sizes[64] < 0.35 * sizes[0]
    assert sizes[16] < 0.6 * sizes[64]


def test_segment_settings():
    prob = make(70, 2, 40, 1, 1800)
    h = qoc.Problem(prob, checkpoint_every=8, segment_steps=40)  # one segment
    assert h.cost_grad(prob.u)["segments"] == 1
    h.close()
    h = qoc.Problem(prob, checkpoint_every=8, segment_steps=5)   # rounded up to L
    assert h.cost_grad(prob.u)["segments"] == 5
    h.close()
    with pytest.raises(qoc.QocError) as ei:
        qoc.Problem(prob, segment_steps=-1)
    assert ei.value.status == -1
    small = make(20, 2, 40, 1, 1801)
    with pytest.raises(qoc.QocError) as ei:
        qoc.Problem(small, segment_steps=8)
    assert ei.value.status == -7
