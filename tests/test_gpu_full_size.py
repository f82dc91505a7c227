"""Full-size transmon-cavity (d=128, N=5000) and spin-chain (d=512, N=1000)
workloads in the launch configuration bench.py times (the checkpoint
interval and sweep variants its autotuner picks there), against stored FP64
oracle values (tests/golden/*_full_oracle.npz, written by
make_golden.py --full, which calls only the oracle), element by element:
the whole gradient (relative l2 over the vector), every per-step penalty
c_j, the final states psi_N, the fidelity, the total cost and theta_max.

bf16x3 runs the same workloads under the automatic product-class policy
(qoc_set_bf16x3(-1)) and is held to its own targets, |dF| <= 1e-5 and
gradient relative l2 <= 1e-3, with the classes the policy chose printed.
"""
import os
import sys

import numpy as np
import pytest

import workloads
from paper_1612_04929_amd import qoc
from test_gpu_parity import psi_bound

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# (workload, checkpoint interval, sweep variants F2, F3, B2, B3)
CASES = [("c3", 64, (4, 4, 4, 4)), ("c4", 32, (2, 2, 2, 2)),
         ("c3", 71, (4, 4, 4, 4))]  # the transmon-cavity workload's stated interval
# accuracy targets per precision: |dF|, gradient rel-l2, max |dc_j|
TARGETS = {"fp32": (1e-6, 1e-4, 2e-6), "bf16x3": (1e-5, 1e-3, 2e-5)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load_golden(name):
    with np.load(os.path.join(GOLDEN, f"{name}_full_oracle.npz")) as z:
        return {k: z[k] for k in z.files}


def run_full(name, L, sweep, precision):
    ref = load_golden(name)
    p = workloads.make_config(name)
    assert (p.d, p.M, p.N, p.S) == tuple(int(ref[k]) for k in ("d", "M", "N", "S"))
    say(f"[full] {name} {precision}: d={p.d} M={p.M} N={p.N} S={p.S} L={L} sweep={sweep}")
    h = qoc.Problem(p, precision=precision, checkpoint_every=L)
    for which, v in enumerate(sweep):
        h.set_sweep(which, v)
    out = h.cost_grad(p.u)
    fwd = h.forward(p.u)
    h.close()
    g = np.asarray(out["grad"], dtype=np.float64)
    gref = ref["grad"]
    e = dict(
        dF=abs((1 - out["C_fid"]) - float(ref["F"])),
        dF_fwd=abs((1 - fwd["C_fid"]) - float(ref["F"])),
        dC=abs(out["C"] - float(ref["C"])),
        grad_rel=float(np.linalg.norm(g - gref) / np.linalg.norm(gref)),
        grad_max=float(np.max(np.abs(g - gref)) / np.linalg.norm(gref)),
        dc=float(np.max(np.abs(out["c"] - ref["c"]))),
        dc_fwd=float(np.max(np.abs(fwd["c"] - ref["c"]))),
        psiN_l2=float(np.max(np.linalg.norm(fwd["psiN"] - ref["psiN"], axis=1))),
        dtheta=abs(out["theta_max"] - float(ref["theta_max"])) / float(ref["theta_max"]),
        p=out["p"], n=out["n"], L=out["block_len"], classes=out["bf16x3_classes"],
        flags=out["flags"])
    say(f"[full] {name} {precision}: " + " ".join(
        f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}" for k, v in e.items()))
    return p, ref, e


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name,L,sweep", CASES)
def test_full_size_matches_stored_oracle(name, L, sweep, precision):
    p, ref, e = run_full(name, L, sweep, precision)
    tF, tG, tc = TARGETS[precision]
    assert e["L"] == L
    assert e["dF"] <= tF and e["dF_fwd"] <= tF, e
    assert e["grad_rel"] <= tG, e
    assert e["dc"] <= tc and e["dc_fwd"] <= tc, e
    assert e["psiN_l2"] <= psi_bound(p, "fp32") * (1.0 if precision == "fp32" else 8.0), e
    # the cost adds |psi_j|^2 of the states over all N steps to the fidelity
    # term: its error is within the fidelity's plus N times the per-step one
    assert e["dC"] <= tF + p.alpha_pen * p.N * tc, e
    assert e["dtheta"] <= 1e-12, e
