"""The no-alloc entry point (qoc_cost_grad_device_noalloc) against
qoc_cost_grad_device through the C ABI: the same cost, penalties and
gradient, bit for bit (the same kernels on the same inputs; only where the
per-call work space lives differs), on two calls in a row of which the
second has a smaller input, and for several paths (padded d 16, a small
chain at padded d 48, batched large-d chains with a fixed pair at padded
d 64 and 256, the
memory-lean mode's time segments, the action form); a call
whose work space exceeds the static scratch is rejected with
QOC_ERR_UNSUPPORTED."""
import sys

import numpy as np
import pytest
import torch

import workloads
from paper_1612_04929_amd import qoc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_both(prob, precision="fp32", **kw):
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev).cuda_stream
    u = torch.from_numpy(np.ascontiguousarray(prob.u)).to(dev)
    res = []
    for noalloc in (False, True):
        h = qoc.Problem(prob, precision=precision, **kw)
        out = torch.full((2 + prob.N,), float("nan"), dtype=torch.float64, device=dev)
        grad = torch.full((max(1, prob.M * prob.N),), float("nan"), dtype=torch.float64,
                          device=dev)
        call = h.cost_grad_device_noalloc if noalloc else h.cost_grad_device
        call(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), grad.cpu().numpy()))
        h.close()
    return res


@pytest.mark.parametrize("case", ["d16", "d40", "d64_fixed", "d256_fixed", "d70_segments",
                                  "action"])
def test_noalloc_matches_device_entry_point_twice(case):
    rng = np.random.default_rng(900)
    if case == "d16":
        big, small = workloads.config2().with_steps(600), workloads.config2().with_steps(150)
        kw = {}
    elif case == "d40":
        big = workloads.random_problem(rng, d=40, M=3, N=120, S=3, dt=0.2, scale=1.5)
        small = workloads.random_problem(rng, d=20, M=2, N=33, S=2, dt=0.2, scale=1.5)
        kw = {}
    elif case == "d64_fixed":
        big = workloads.random_problem(rng, d=64, M=3, N=90, S=2, dt=0.2, scale=1.5)
        small = workloads.random_problem(rng, d=64, M=2, N=40, S=2, dt=0.2, scale=1.5)
        kw = dict(taylor_pn=(9, 2))
    elif case == "d256_fixed":
        # 64 x 128 stage tiles
        big = workloads.random_problem(rng, d=256, M=2, N=24, S=2, dt=0.1, scale=1.5)
        small = workloads.random_problem(rng, d=256, M=2, N=10, S=1, dt=0.1, scale=1.5)
        kw = dict(taylor_pn=(9, 2))
    elif case == "d70_segments":
        # memory-lean mode: the segment's stacks carved from the scratch
        big = workloads.random_problem(rng, d=70, M=3, N=96, S=2, dt=0.2, scale=1.5)
        small = workloads.random_problem(rng, d=70, M=2, N=41, S=1, dt=0.2, scale=1.5)
        kw = dict(taylor_pn=(9, 2), checkpoint_every=8, segment_steps=24)
    else:
        # action form: the kept product inputs and cotangents in the scratch
        big = workloads.sparse_problem(rng, 90, 3, 80, 2, dt=0.15)
        small = workloads.sparse_problem(rng, 90, 2, 30, 1, dt=0.15)
        kw = dict(propagation="action")
    for prob in (big, small):
        say(f"[noalloc] {case}: d={prob.d} M={prob.M} N={prob.N} S={prob.S}")
        (o1, g1), (o2, g2) = run_both(prob, **kw)
        assert np.all(np.isfinite(o2)) and np.all(np.isfinite(g2[: prob.M * prob.N]))
        assert np.array_equal(o1, o2), np.max(np.abs(o1 - o2))
        assert np.array_equal(g1[: prob.M * prob.N], g2[: prob.M * prob.N])


def test_noalloc_rejects_work_space_beyond_the_scratch():
    # padded d 128, N 5000: the levels alone need far more than 256 MiB
    prob = workloads.config3()
    say(f"[noalloc] oversize: d={prob.d} N={prob.N}")
    dev = torch.device("cuda:0")
    h = qoc.Problem(prob, precision="fp32", taylor_pn=(8, 5))
    u = torch.from_numpy(np.ascontiguousarray(prob.u)).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    grad = torch.zeros(prob.M * prob.N, dtype=torch.float64, device=dev)
    with pytest.raises(qoc.QocError) as ei:
        h.cost_grad_device_noalloc(u.data_ptr(), out.data_ptr(), grad.data_ptr(),
                                   torch.cuda.current_stream(dev).cuda_stream)
    assert ei.value.status == -7 and "static device scratch" in str(ei.value)
    torch.cuda.synchronize()
    h.close()
