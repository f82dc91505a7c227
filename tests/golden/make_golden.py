"""Writes the stored expected values under tests/golden/ by calling only the
FP64 oracle (``oracle/``) on seeded inputs from ``workloads``.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    p = workloads.config1()
    out = oracle.cost_grad(p)
    pn = oracle.taylor_select(out["theta_max"], 1e-10)
    rec = {
        "source": "oracle.cost_grad on workloads.config1() (single qubit, X gate)",
        "C": out["C"], "C_fid": out["C_fid"], "theta_max": out["theta_max"],
        "taylor_pn_tau1e-10": list(pn),
        "grad": np.asarray(out["grad"]).round(17).tolist(),
        "psiN_re": out["psiN"].real.tolist(), "psiN_im": out["psiN"].imag.tolist(),
    }
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote c1_oracle.json")


if __name__ == "__main__":
    main()
