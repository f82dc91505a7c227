"""Writes the stored expected values under tests/golden/ by calling only the
FP64 oracle (``oracle/``) on seeded inputs from ``workloads``.

Run from the repository root:  python tests/golden/make_golden.py
(the single-qubit fixture),  python tests/golden/make_golden.py --full c3 c4
(full-size transmon-cavity and spin-chain workloads; minutes of CPU time) and
python tests/golden/make_golden.py --c5 (full-length instances of the batched
uneven workload).  The full-size records hold every output the GPU tests
compare element by element: the whole gradient, every per-step penalty c_j
and the final states psi_N (``*_full_oracle.npz``, read with numpy.load and
its default allow_pickle=False), beside a JSON file of the scalars.
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


def save_arrays(fname, p, out):
    """Every output of one oracle call, as plain numeric arrays."""
    np.savez_compressed(
        os.path.join(HERE, fname),
        d=p.d, M=p.M, N=p.N, S=p.S, C=out["C"], C_fid=out["C_fid"], F=out["F"],
        theta_max=out["theta_max"], C_pen=out["C_pen"], C_amp=out["C_amp"],
        C_var=out["C_var"], unitarity_drift=out["unitarity_drift"],
        grad=np.asarray(out["grad"], dtype=np.float64),
        c=np.asarray(out["c"], dtype=np.float64),
        psiN=np.asarray(out["psiN"], dtype=np.complex128))
    print("wrote", fname, flush=True)


def full(name, samples=256, top=16):
    """Full-size workload: cost, fidelity, theta_max, the gradient's l2 norm
    and a seeded sample of gradient entries (plus the largest ones) in JSON,
    and every output in the .npz beside it; the GPU tests compare the
    full-size run against them."""
    p = workloads.make_config(name)
    out = oracle.cost_grad(p)
    save_arrays(f"{name}_full_oracle.npz", p, out)
    g = np.asarray(out["grad"], dtype=np.float64).ravel()
    rng = np.random.default_rng(2024)
    idx = set(rng.choice(g.size, size=min(samples, g.size), replace=False).tolist())
    idx |= set(np.argsort(-np.abs(g))[:top].tolist())
    idx = sorted(int(i) for i in idx)
    c = np.asarray(out["c"], dtype=np.float64)
    rec = {
        "source": f"oracle.cost_grad on workloads.make_config({name!r}) ({p.name})",
        "d": p.d, "M": p.M, "N": p.N, "S": p.S,
        "C": out["C"], "C_fid": out["C_fid"], "F": out["F"], "theta_max": out["theta_max"],
        "grad_l2": float(np.linalg.norm(g)),
        "grad_index": idx, "grad_sample": [float(g[i]) for i in idx],
        "penalty_sum": float(c.sum()),
    }
    fname = f"{name}_full_oracle.json"
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", fname)


def c5_instances(probs):
    """Full-length instances of the batched uneven workload that the GPU
    tests check one by one: the largest d, the longest N and the largest
    d^3 N (ties to the lower index)."""
    by = lambda key: max(range(len(probs)), key=lambda i: (key(probs[i]), -i))
    picks = [by(lambda p: p.d), by(lambda p: p.N), by(lambda p: p.d ** 3 * p.N)]
    return sorted(set(picks))


def c5():
    probs = workloads.config5()
    for i in c5_instances(probs):
        p = probs[i]
        print(f"c5 instance {i}: d={p.d} M={p.M} N={p.N}", flush=True)
        save_arrays(f"c5_{i:03d}_oracle.npz", p, oracle.cost_grad(p))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--full":
        for name in sys.argv[2:] or ["c3", "c4"]:
            full(name)
    elif len(sys.argv) > 1 and sys.argv[1] == "--c5":
        c5()
    else:
        main()
