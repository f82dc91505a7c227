"""Diagnostics and error paths of the C ABI on the GPU.

* The FP64 unitarity check max_j max_{r,c} |(U_j^H U_j - I)_{rc}| (U_j = I +
  D_j) against the same quantity of the Taylor approximant the oracle
  evaluates in FP64 (oracle.taylor_squaring_expm), with a deliberately
  short series so that the drift is large enough to compare: for p = 2,
  n = 0, T^H T - I = X^4 / 4 exactly (X^H = -X).
* QOC_WARN_DRIFT and QOC_WARN_UNITARITY forced by a tiny threshold.
* QOC_ERR_NONFINITE for NaN amplitudes on the host entry points, and
  QOC_WARN_NO_PAIR after a device-pointer call with NaN amplitudes.
* QOC_ERR_NOMEM for a problem larger than the GPU's memory.
* QOC_ERR_UNSUPPORTED from a call that would synchronise under HIP graph
  capture, and for fixed pairs beyond a path's capacity.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1612_04929_amd import qoc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def approximant_drift(prob, p, n, steps):
    """max over `steps` of max |T^H T - I| for T the order-p Taylor
    approximant with n squarings of exp(-i dt H_j), in FP64 (oracle)."""
    H = oracle.step_hamiltonians(prob)
    out = 0.0
    for j in steps:
        T = oracle.taylor_squaring_expm(-1j * prob.dt * H[j], p, n)
        out = max(out, float(np.max(np.abs(T.conj().T @ T - np.eye(prob.d)))))
    return out


@pytest.mark.parametrize("d,prec,stride", [(5, "fp32", 1), (40, "fp32", 1), (70, "fp32", 1),
                                           (70, "fp32", 4), (20, "fp64", 1), (64, "bf16x3", 1)])
def test_unitarity_check_matches_approximant(d, prec, stride):
    rng = np.random.default_rng(800 + d)
    prob = workloads.random_problem(rng, d=d, M=2, N=30, S=2, dt=0.25, scale=1.5)
    pn = (2, 0)
    say(f"[diag] unitarity d={d} {prec} stride={stride}")
    h = qoc.Problem(prob, precision=prec, taylor_pn=pn)
    h.set_unitarity_check(stride)
    out = h.cost_grad(prob.u)
    steps = list(range(prob.N - 1, -1, -stride))
    ref = approximant_drift(prob, *pn, steps)
    got = out["unitarity_drift"]
    say(f"[diag] drift gpu={got:.6e} ref={ref:.6e} theta={out['theta_max']:.3f}")
    assert ref > 1e-4  # a short series: far from unitary
    # FP32 step propagators carry rounding errors of a few 2^-24 |D| that
    # enter D + D^H linearly: 1e-4 relative plus 1e-6 absolute; FP64 chains:
    # the FP32 storage of the reported maximum (2^-24 relative)
    if prec == "fp64":
        assert abs(got - ref) <= 2.0 ** -23 * ref
    else:
        assert abs(got - ref) <= 1e-4 * ref + 1e-6
    assert out["flags"] & qoc.QOC_WARN_UNITARITY  # above the default drift_warn 1e-4
    h.set_unitarity_check(0)
    assert h.cost_grad(prob.u)["unitarity_drift"] == -1.0
    h.close()


def test_unitarity_check_default_pair_and_thresholds():
    prob = workloads.config2().with_steps(300)
    h = qoc.Problem(prob, precision="fp32")
    h.set_unitarity_check(1)
    out = h.cost_grad(prob.u)
    say(f"[diag] c2 N=300 unitarity {out['unitarity_drift']:.3e} norm drift {out['norm_drift']:.3e}")
    assert 0.0 < out["unitarity_drift"] < 1e-5       # FP32 rounding, a converged series
    assert not out["flags"] & (qoc.QOC_WARN_UNITARITY | qoc.QOC_WARN_DRIFT)
    h.close()
    # a threshold below FP32 rounding raises both drift flags
    h = qoc.Problem(prob, precision="fp32", drift_warn=1e-14)
    h.set_unitarity_check(1)
    out = h.cost_grad(prob.u)
    assert out["flags"] & qoc.QOC_WARN_UNITARITY and out["flags"] & qoc.QOC_WARN_DRIFT
    h.close()


def test_nonfinite_amplitudes():
    prob = workloads.config2().with_steps(50)
    u = prob.u.copy()
    u[1, 7] = np.nan
    h = qoc.Problem(prob, precision="fp32")
    for call in (h.cost_grad, h.forward):
        with pytest.raises(qoc.QocError) as ei:
            call(u)
        assert ei.value.status == -4
    # device pointers are not scanned on the host: the device-side (p, n)
    # choice sees a NaN theta_max and reports it
    dev = torch.device("cuda:0")
    ud = torch.from_numpy(u).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    g = torch.zeros(prob.M * prob.N, dtype=torch.float64, device=dev)
    h.cost_grad_device(ud.data_ptr(), out.data_ptr(), g.data_ptr(),
                       torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    assert h.info()["flags"] & qoc.QOC_WARN_NO_PAIR
    with pytest.raises(qoc.QocError):
        h.check_last()
    # a finite call afterwards is clean again
    assert h.cost_grad(prob.u)["flags"] & qoc.QOC_WARN_NO_PAIR == 0
    h.close()


def test_out_of_memory_is_reported():
    # d = 1024, N = 2^22: the step stack alone would be 32 TiB
    d, N = 1024, 1 << 22
    prob = workloads.Problem("huge", d, 0, N, 1, 0.1, np.zeros((d, d), complex),
                             np.zeros((0, d, d), complex), np.zeros((0, N)),
                             np.eye(d, dtype=complex)[:1], np.eye(d, dtype=complex)[:1])
    say("[diag] NOMEM d=1024 N=2^22")
    with pytest.raises(qoc.QocError) as ei:
        qoc.Problem(prob, precision="fp32")
    assert ei.value.status == -5
    # the device is still usable
    p2 = workloads.config1()
    h = qoc.Problem(p2)
    assert np.isfinite(h.cost_grad(p2.u)["C"])
    h.close()


def test_fixed_pair_beyond_capacity_rejected():
    prob = workloads.config2().with_steps(20)  # padded d 16: small path, p, n <= 16
    h = qoc.Problem(prob)
    with pytest.raises(qoc.QocError) as ei:
        h.set_taylor(20, 2)
    assert ei.value.status == -7
    with pytest.raises(qoc.QocError):
        qoc.Problem(prob, taylor_pn=(8, 17))
    h.set_taylor(16, 16)  # at the caps
    h.close()


def test_capture_of_a_synchronising_call_is_rejected():
    """A batched-path handle (padded d 64) without a fixed pair must read
    theta_max back to the host: under HIP graph capture the call returns
    QOC_ERR_UNSUPPORTED instead of synchronising the capturing stream; with
    profiling enabled it is rejected before any launch.  The capture is
    ended and discarded."""
    rng = np.random.default_rng(810)
    prob = workloads.random_problem(rng, d=64, M=2, N=20, S=2, dt=0.2)
    dev = torch.device("cuda:0")
    h = qoc.Problem(prob, precision="fp32")
    u = torch.from_numpy(np.ascontiguousarray(prob.u)).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    g = torch.zeros(prob.M * prob.N, dtype=torch.float64, device=dev)
    h.cost_grad_device(u.data_ptr(), out.data_ptr(), g.data_ptr(),
                       torch.cuda.current_stream(dev).cuda_stream)  # buffers sized
    torch.cuda.synchronize()
    say("[diag] capture guard")
    side = torch.cuda.Stream(dev)
    errors = []
    for prof in (False, True):
        h.profile_enable(prof)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                try:
                    h.cost_grad_device(u.data_ptr(), out.data_ptr(), g.data_ptr(),
                                       side.cuda_stream)
                except qoc.QocError as e:
                    errors.append(e)
        torch.cuda.synchronize()
        del graph
    h.profile_enable(False)
    assert len(errors) == 2 and all(e.status == -7 for e in errors)
    assert "theta_max" in str(errors[0]) and "profiling" in str(errors[1])
    # a fixed pair makes the same call capturable, and the replay matches eager
    h.set_taylor(*qoc.taylor_select(h.info()["theta_max"] * 1.1, 1e-10))
    h.cost_grad_device(u.data_ptr(), out.data_ptr(), g.data_ptr(),
                       torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    ref = (out.clone(), g.clone())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            h.cost_grad_device(u.data_ptr(), out.data_ptr(), g.data_ptr(), side.cuda_stream)
    for _ in range(3):
        out.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref[0]) and torch.equal(g, ref[1])
    h.close()


@pytest.mark.parametrize("case", ["d16", "d40", "d100", "c4_structured", "ext"])
def test_results_are_bitwise_deterministic(case):
    """Every reduction runs in a fixed order (no floating-point atomics): two
    calls on one handle and a call on a fresh handle give the same bits."""
    rng = np.random.default_rng(1300)
    if case == "d16":
        p = workloads.config2().with_steps(300)
    elif case == "d40":
        p = workloads.random_problem(rng, d=40, M=3, N=90, S=3, dt=0.2, scale=1.5)
    elif case == "d100":
        p = workloads.random_problem(rng, d=100, M=3, N=70, S=2, dt=0.2, scale=1.5)
    elif case == "c4_structured":
        p = workloads.config4().with_steps(30)
    else:
        p = workloads.random_problem(rng, d=24, M=2, N=80, S=2, dt=0.2, scale=1.5,
                                     n_forbidden=2, alpha_time=0.3)
    say(f"[diag] determinism {case}")
    h1 = qoc.Problem(p)
    a = h1.cost_grad(p.u)
    b = h1.cost_grad(p.u)
    h1.close()
    h2 = qoc.Problem(p)
    c = h2.cost_grad(p.u)
    h2.close()
    for x in (b, c):
        assert x["C"] == a["C"] and x["C_fid"] == a["C_fid"]
        assert np.array_equal(x["c"], a["c"]) and np.array_equal(x["grad"], a["grad"])
