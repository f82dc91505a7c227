"""torch.autograd.Function bridge: argument checks on the CPU, and on the GPU
the backward pass against the C-ABI gradient and the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1612_04929_amd import qoc
from paper_1612_04929_amd.autograd import QocCostGrad, _check_u


class _Shape:
    M, N = 2, 5


def test_rejects_cpu_tensor():
    # no CPU fallback: a host tensor is refused before any library call
    with pytest.raises(ValueError, match="GPU"):
        _check_u(torch.zeros(2, 5, dtype=torch.float64), _Shape())


def test_rejects_wrong_dtype_and_shape():
    with pytest.raises(TypeError):
        _check_u(np.zeros((2, 5)), _Shape())


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.gpu
def test_autograd_matches_abi_and_oracle():
    prob = workloads.make_config("c2").with_steps(300)
    say(f"[autograd] c2 N=300 d={prob.d}")
    ref = oracle.cost_grad(prob)
    h = qoc.Problem(prob, precision="fp32")
    abi = h.cost_grad(prob.u)
    dev = torch.device("cuda:0")
    u = torch.tensor(prob.u, dtype=torch.float64, device=dev, requires_grad=True)
    C, C_fid, c = QocCostGrad.apply(u, h)
    (3.0 * C).backward()
    g = u.grad.cpu().numpy() / 3.0
    h.close()
    assert abs(float(C) - abi["C"]) <= 1e-12 * max(1.0, abs(abi["C"]))
    assert abs(float(C_fid) - abi["C_fid"]) <= 1e-12
    assert np.allclose(c.cpu().numpy(), abi["c"], rtol=0, atol=1e-12)
    assert np.max(np.abs(g - abi["grad"])) <= 1e-12 * max(1.0, np.max(np.abs(abi["grad"])))
    rel = np.linalg.norm(g - ref["grad"]) / np.linalg.norm(ref["grad"])
    say(f"[autograd] grad rel vs oracle {rel:.3e}")
    assert rel <= 1e-4


@pytest.mark.gpu
def test_autograd_adam_descends():
    # a few optimizer steps on the single-qubit gate problem lower the cost
    prob = workloads.make_config("c1")
    say(f"[autograd] c1 Adam d={prob.d} N={prob.N}")
    h = qoc.Problem(prob, precision="fp32")
    dev = torch.device("cuda:0")
    u = torch.tensor(prob.u, dtype=torch.float64, device=dev, requires_grad=True)
    opt = torch.optim.Adam([u], lr=1e-2)
    costs = []
    for _ in range(20):
        opt.zero_grad()
        C, _, _ = QocCostGrad.apply(u, h)
        C.backward()
        opt.step()
        costs.append(float(C))
    h.close()
    say(f"[autograd] costs {costs[0]:.6f} -> {costs[-1]:.6f}")
    assert costs[-1] < costs[0]
