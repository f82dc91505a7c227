"""Uneven batches (the 256-instance transmon-chain workload, cut down):
batched multi-stream calls with fixed (p, n) against the FP64 oracle, and
HIP-graph replays of whole optimizer iterations against eager iterations."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch(count=12, nmax=200):
    probs = workloads.config5()[:count]
    return [p.with_steps(min(p.N, nmax)) for p in probs]


def test_batched_calls_match_oracle():
    from paper_1612_04929_amd.batch import Batch
    probs = small_batch()
    say("[batch] instances: " + ", ".join(f"d{p.d}/N{p.N}/M{p.M}" for p in probs))
    b = Batch(probs, precision="fp32", streams=3)
    b.cost_grad()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        ref = oracle.cost_grad(p)
        dF = abs((1 - float(b.out[i][1])) - ref["F"])
        g = b.grad[i][: p.M * p.N].cpu().numpy().reshape(p.M, p.N)
        # some instances have F = 0 and a zero gradient for every u (the
        # controls never connect the initial and target levels): absolute floor
        err, nrm = float(np.linalg.norm(g - ref["grad"])), float(np.linalg.norm(ref["grad"]))
        say(f"[batch] {p.name} d={p.d} N={p.N} pn={b.pn[i]} dF={dF:.2e} "
            f"grad_err={err:.2e} |grad|={nrm:.2e}")
        assert dF <= 1e-6 and err <= 1e-4 * nrm + 1e-9
    assert b.taylor_warnings() == []
    b.close()


def test_graph_replays_equal_eager_iterations():
    from paper_1612_04929_amd.batch import Batch
    probs = small_batch(count=8, nmax=150)
    say("[batch] graph vs eager, 8 instances")
    a = Batch(probs, precision="fp32", streams=2)
    for _ in range(5):
        a.iteration()
    b = Batch(probs, precision="fp32", streams=2)
    b.capture(warmup=3)
    b.replay()
    torch.cuda.synchronize()
    b.replay()
    torch.cuda.synchronize()
    for i in range(len(probs)):
        ua, ub = a.u[i].detach().cpu().numpy(), b.u[i].detach().cpu().numpy()
        assert np.allclose(ua, ub, rtol=0, atol=1e-12), (i, np.max(np.abs(ua - ub)))
    ca, cb = a.costs(), b.costs()
    say(f"[batch] costs eager {ca[:3]} graph {cb[:3]}")
    assert np.allclose(ca, cb, rtol=1e-12, atol=1e-12)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_full_length_instances_match_stored_oracle(precision):
    """Full-length instances of the 256-instance workload (the largest d, the
    longest N and the largest d^3 N; tests/golden/c5_*_oracle.npz, written
    by make_golden.py --c5 from the oracle alone) through a Batch with its
    fixed (p, n), element by element: fidelity, every c_j (zero here), the
    whole gradient."""
    import glob
    import os
    from paper_1612_04929_amd.batch import Batch
    here = os.path.dirname(os.path.abspath(__file__))
    files = sorted(glob.glob(os.path.join(here, "golden", "c5_*_oracle.npz")))
    assert len(files) >= 3
    allp = workloads.config5()
    idx = [int(os.path.basename(f)[3:6]) for f in files]
    probs = [allp[i] for i in idx]
    say(f"[batch] full-length {precision}: " + ", ".join(f"d{p.d}/N{p.N}/M{p.M}" for p in probs))
    b = Batch(probs, precision=precision, streams=2)
    b.cost_grad()
    torch.cuda.synchronize()
    tF, tG = (1e-6, 1e-4) if precision == "fp32" else (1e-5, 1e-3)
    for f, i, p in zip(files, range(len(probs)), probs):
        with np.load(f) as z:
            ref = {k: z[k] for k in z.files}
        assert (p.d, p.M, p.N) == (int(ref["d"]), int(ref["M"]), int(ref["N"]))
        dF = abs((1 - float(b.out[i][1])) - float(ref["F"]))
        g = b.grad[i][: p.M * p.N].cpu().numpy().reshape(p.M, p.N)
        c = b.out[i][2:].cpu().numpy()
        err, nrm = float(np.linalg.norm(g - ref["grad"])), float(np.linalg.norm(ref["grad"]))
        say(f"[batch] {p.name} d={p.d} N={p.N} pn={b.pn[i]} dF={dF:.2e} "
            f"grad_rel={err / max(nrm, 1e-300):.2e} |grad|={nrm:.2e}")
        assert dF <= tF
        assert err <= tG * nrm + 1e-9
        assert np.max(np.abs(c - ref["c"])) <= 2e-6
    b.close()


def test_adam_kernel_matches_reference():
    """qoc_adam_step against Adam written out in FP64 on the host (the
    update of Kingma and Ba with bias corrections), three steps in a row,
    the step count kept on the device."""
    from paper_1612_04929_amd import qoc
    rng = np.random.default_rng(1200)
    n = 10007
    u0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * s for s in (1.0, 0.3, 2.0)]
    dev = torch.device("cuda:0")
    u = torch.tensor(u0, dtype=torch.float64, device=dev)
    m = torch.zeros_like(u)
    v = torch.zeros_like(u)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    ru, rm, rv = u0.copy(), np.zeros(n), np.zeros(n)
    st = torch.cuda.current_stream(dev).cuda_stream
    for k, gk in enumerate(grads, start=1):
        g = torch.tensor(gk, dtype=torch.float64, device=dev)
        qoc.adam_step(n, u.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), t.data_ptr(),
                      lr, (b1, b2), eps, st)
        torch.cuda.synchronize()
        rm = b1 * rm + (1 - b1) * gk
        rv = b2 * rv + (1 - b2) * gk * gk
        mh, vh = rm / (1 - b1 ** k), rv / (1 - b2 ** k)
        ru = ru - lr * mh / (np.sqrt(vh) + eps)
        assert float(t.item()) == k
        assert np.max(np.abs(u.cpu().numpy() - ru)) <= 1e-13
    with pytest.raises(qoc.QocError):
        qoc.adam_step(n, u.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), t.data_ptr(),
                      lr, (1.0, b2), eps, st)
