"""Full-size transmon-cavity (d=128, N=5000) and spin-chain (d=512, N=1000)
workloads in the launch configuration bench.py times (the checkpoint
interval and sweep variants its autotuner picks there), against stored FP64
oracle values (tests/golden/*_full_oracle.json, written by
make_golden.py --full, which calls only the oracle): fidelity, cost,
theta_max and penalty sum directly; the gradient through its l2 norm and a
seeded sample of entries (plus the largest ones), the sampled error measured
against the full norm."""
import json
import os
import sys

import numpy as np
import pytest

import workloads
from paper_1612_04929_amd import qoc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# (workload, checkpoint interval, sweep variants F2, F3, B2, B3)
CASES = [("c3", 64, (4, 4, 4, 4)), ("c4", 32, (2, 2, 2, 2))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,L,sweep", CASES)
def test_full_size_fp32_matches_stored_oracle(name, L, sweep):
    ref = json.load(open(os.path.join(GOLDEN, f"{name}_full_oracle.json")))
    p = workloads.make_config(name)
    assert (p.d, p.M, p.N, p.S) == (ref["d"], ref["M"], ref["N"], ref["S"])
    say(f"[full] {name}: d={p.d} M={p.M} N={p.N} S={p.S} L={L} sweep={sweep}")
    h = qoc.Problem(p, precision="fp32", checkpoint_every=L)
    for which, v in enumerate(sweep):
        h.set_sweep(which, v)
    out = h.cost_grad(p.u)
    h.close()
    g = np.asarray(out["grad"], dtype=np.float64).ravel()
    idx = np.asarray(ref["grad_index"])
    gs = np.asarray(ref["grad_sample"])
    dF = abs((1 - out["C_fid"]) - ref["F"])
    dC = abs(out["C"] - ref["C"])
    sample_err = float(np.max(np.abs(g[idx] - gs))) / ref["grad_l2"]
    norm_err = abs(float(np.linalg.norm(g)) - ref["grad_l2"]) / ref["grad_l2"]
    dtheta = abs(out["theta_max"] - ref["theta_max"]) / ref["theta_max"]
    dpen = abs(float(np.sum(out["c"])) - ref["penalty_sum"]) / max(1.0, abs(ref["penalty_sum"]))
    say(f"[full] {name}: dF={dF:.2e} dC={dC:.2e} sample_err={sample_err:.2e} "
        f"norm_err={norm_err:.2e} dtheta={dtheta:.2e} dpen={dpen:.2e} p={out['p']} n={out['n']}")
    assert out["block_len"] == L
    assert dF <= 1e-6
    # the cost and the penalty sum add |psi_j|^2 of FP32 states over all N
    # steps: their relative error follows the FP32 state error (norm drift
    # ~1e-6 at these sizes), so 1e-5 relative; the fidelity is held to 1e-6
    assert dC <= 1e-5 * max(1.0, abs(ref["C"]))
    assert dtheta <= 1e-12
    assert dpen <= 1e-5
    # each sampled entry within 1e-4 of the gradient's l2 norm, and the norm
    # itself within 1e-4 (the FP32 target is rel-l2 <= 1e-4 on the vector)
    assert sample_err <= 1e-4
    assert norm_err <= 1e-4
