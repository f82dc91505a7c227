"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP32 chains): |F_gpu - F_oracle| <= 1e-6 and gradient relative
l2 error <= 1e-4 (the accuracy targets of the FP32 path).  FP64 chains:
|dF| <= 1e-11, gradient relative error <= 1e-9.  Per-step penalties and
the total cost are compared against bounds derived in the design notes from
FP32 state rounding: |dc_j| <= 2e-6 * max(1, max|c|) and
|dC| <= 1e-6 * (1 + |C|) + a_pen * N * 2e-6.

Every case prints its name, shape and the achieved errors (flushed) before
and after the GPU call.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from paper_1612_04929_amd import qoc

pytestmark = pytest.mark.gpu

REPORT = os.environ.get("QOC_PARITY_REPORT")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def compare(name, prob, precision="fp32", oracle_out=None, sweep=None, **kw):
    say(f"[parity] {name}: d={prob.d} M={prob.M} N={prob.N} S={prob.S} prec={precision}")
    ref = oracle_out if oracle_out is not None else oracle.cost_grad(prob)
    h = qoc.Problem(prob, precision=precision, **kw)
    if sweep is not None:
        h.set_sweep(-1, sweep)
    out = h.cost_grad(prob.u)
    fwd = h.forward(prob.u)
    h.close()
    errs = dict(
        dF=abs((1 - out["C_fid"]) - ref["F"]),
        dC=abs(out["C"] - ref["C"]),
        dc=float(np.max(np.abs(out["c"] - ref["c"]))) if prob.N else 0.0,
        grad_rel=rel(out["grad"], ref["grad"]) if prob.M else 0.0,
        psiN=float(np.max(np.abs(fwd["psiN"] - ref["psiN"]))),
        psiN_l2=float(np.max(np.linalg.norm(fwd["psiN"] - ref["psiN"], axis=1))),
        dF_fwd=abs((1 - fwd["C_fid"]) - ref["F"]),
        p=out["p"], n=out["n"], theta=out["theta_max"], theta_ref=ref["theta_max"],
        drift=out["norm_drift"], L=out["block_len"], nb=out["n_blocks"])
    say(f"[parity] {name}: " + json.dumps({k: (float(v) if isinstance(v, (float, np.floating)) else v)
                                           for k, v in errs.items()}))
    if REPORT:
        with open(REPORT, "a") as f:
            f.write(json.dumps({"case": name, "precision": precision, **{
                k: (float(v) if isinstance(v, (float, np.floating)) else v)
                for k, v in errs.items()}}) + "\n")
    return out, ref, errs


def psi_bound(prob, precision):
    """Bound on the l2 error of each final state psi_N^s.  Each step's
    propagator carries about G = p - 1 + n products whose rounding errors
    (unit roundoff u: 2^-24 FP32, 2^-53 FP64) enter at the scale of the
    operands, |D| <= 2 after the squarings, and independent errors of the N
    steps add in quadrature: 8 G u sqrt(N) with G <= 24, floored at 1e-6
    (FP32) / 1e-12 (FP64)."""
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    floor = 1e-12 if precision == "fp64" else 1e-6
    return max(floor, 8 * 24 * u * np.sqrt(prob.N))


def check(prob, errs, precision="fp32"):
    if precision == "fp64":
        tF, tG, tc = 1e-11, 1e-9, 1e-11
    else:
        tF, tG, tc = 1e-6, 1e-4, 2e-6
    assert errs["dF"] <= tF, errs
    assert errs["dF_fwd"] <= tF, errs
    # qoc_forward's psiN output (planar device states to interleaved doubles)
    assert errs["psiN_l2"] <= psi_bound(prob, precision), errs
    if prob.M:
        assert errs["grad_rel"] <= tG, errs
    pen = prob.w is not None or getattr(prob, "forbidden", None) is not None
    if pen:
        assert errs["dc"] <= tc, errs
    # the time-optimal term averages N fidelities, each within tF
    budget = (prob.alpha_fid * tF + (prob.alpha_pen * prob.N * tc if pen else 0.0)
              + abs(getattr(prob, "alpha_time", 0.0)) * tF + 1e-9)
    assert errs["dC"] <= budget, errs
    # the GPU chooses (p, n) from its own FP64 theta_max by the same rule
    assert abs(errs["theta"] - errs["theta_ref"]) <= 1e-12 * max(1.0, errs["theta_ref"]), errs


def test_config1_qubit_x_gate():
    p = workloads.config1()
    out, ref, e = compare("c1", p)
    check(p, e)
    assert (e["p"], e["n"]) == oracle.taylor_select(ref["theta_max"], 1e-10)


def test_config2_transmon_cnot_full():
    p = workloads.config2()
    out, ref, e = compare("c2", p)
    check(p, e)
    assert (e["p"], e["n"]) == oracle.taylor_select(ref["theta_max"], 1e-10)


@pytest.mark.parametrize("d,S,N,mode", [
    (5, 1, 37, "coherent"),        # ragged d (pad 16), ragged N
    (5, 5, 40, "coherent"),        # full unitary: rank compression in the adjoint
    (20, 3, 100, "incoherent"),    # pad 32, incoherent fidelity
    (64, 2, 70, "coherent"),       # 64-tiled product kernels
    (70, 4, 33, "coherent"),       # pad 80, 16-tiled kernels on a non-64 multiple
    (3, 2, 1, "coherent"),         # a single step
    (64, 48, 20, "coherent"),      # batched adjoint: rank compression at the first level
    (100, 3, 25, "incoherent"),    # batched adjoint on pad 112 (partial 64-tiles)
    (256, 2, 8, "coherent"),       # 64 x 128 stage tiles (4 x 2 per matrix)
    (384, 3, 5, "incoherent"),     # 64 x 128 stage tiles (6 x 3 per matrix)
])
def test_random_problems(d, S, N, mode):
    rng = np.random.default_rng(100 + d + N)
    p = workloads.random_problem(rng, d=d, M=3, N=N, S=S, dt=0.2, scale=2.0, fid_mode=mode)
    out, ref, e = compare(f"rand_d{d}_S{S}_N{N}_{mode}", p)
    check(p, e)


@pytest.mark.parametrize("L", [1, 2, 8, 64, 3, 7, 71])
def test_checkpoint_interval_does_not_change_results(L):
    rng = np.random.default_rng(7)
    p = workloads.random_problem(rng, d=12, M=2, N=50, S=2, dt=0.3, scale=1.5)
    out, ref, e = compare(f"ckpt_L{L}", p, checkpoint_every=L)
    check(p, e)
    assert e["L"] == L


@pytest.mark.parametrize("d,S,N,L,pen,mode,prec", [
    (16, 4, 203, 16, True, "coherent", "fp32"),    # ragged last block: sub-blocks of 8 and 3
    (12, 2, 131, 32, True, "incoherent", "fp32"),  # last block of 3 steps (one short sub-block)
    (16, 4, 250, 64, True, "coherent", "fp32"),    # 8 sub-blocks a block, last block of 58
    (9, 1, 257, 64, True, "coherent", "fp32"),     # last block one step (seven idle wavefronts)
    (16, 3, 100, 32, False, "coherent", "fp32"),   # no penalty: no partial costates
    (16, 4, 40, 64, True, "coherent", "fp32"),     # one block shorter than L
    (16, 2, 77, 128, True, "coherent", "fp32"),    # L above the split's limit: unsplit passes
    (16, 2, 90, 32, True, "coherent", "fp64"),     # FP64 chains: unsplit passes
])
def test_split_in_block_passes(d, S, N, L, pen, mode, prec):
    # padded d 16 with L a multiple of 8: the in-block passes (forward replay
    # with the block penalty costate, costate replay) run over sub-blocks of
    # 8 steps from the sub-block products of the block-product kernel
    rng = np.random.default_rng(300 + d + N + L)
    p = workloads.random_problem(rng, d=d, M=2, N=N, S=S, dt=0.2, scale=1.5,
                                 with_penalty=pen, fid_mode=mode)
    out, ref, e = compare(f"split_d{d}_S{S}_N{N}_L{L}_{prec}", p, precision=prec,
                          checkpoint_every=L, sweep=1)
    check(p, e, precision=prec)
    assert e["L"] == L


@pytest.mark.parametrize("L", [1, 4, 64, 3, 12, 71])
def test_wide_sweeps_checkpoint_intervals(L):
    # padded d 96: per-step launches of the sweeps, ragged last block, penalty
    rng = np.random.default_rng(17)
    p = workloads.random_problem(rng, d=90, M=2, N=50, S=3, dt=0.25, scale=1.5)
    out, ref, e = compare(f"wide_L{L}", p, checkpoint_every=L)
    check(p, e)
    assert e["L"] == L


@pytest.mark.parametrize("d,S,N,L", [(64, 2, 45, 8), (70, 3, 50, 16), (120, 1, 70, 32),
                                     (100, 2, 33, 1), (128, 1, 300, 71), (64, 2, 100, 9)])
def test_chain_workgroup_sweeps(d, S, N, L):
    # sweep variant 4 on padded d 64 / 80 / 128 / 112: every sweep as one
    # 8 d_pad-thread workgroup per block, ragged last block, penalty
    rng = np.random.default_rng(500 + d + N)
    p = workloads.random_problem(rng, d=d, M=2, N=N, S=S, dt=0.2, scale=1.5)
    out, ref, e = compare(f"chain_d{d}_S{S}_L{L}", p, checkpoint_every=L, sweep=4)
    check(p, e)
    assert e["L"] == L


@pytest.mark.parametrize("pn", [(4, 3), (5, 3), (9, 2), (12, 1), (16, 0)])
def test_batched_taylor_orders(pn):
    # padded d 80: Paterson-Stockmeyer blocks s = 2, 3, 4 and both endings
    rng = np.random.default_rng(41)
    p = workloads.random_problem(rng, d=70, M=2, N=30, S=2, dt=0.15, scale=1.5)
    out, ref, e = compare(f"orders_p{pn[0]}_n{pn[1]}", p, taylor_pn=pn)
    check(p, e)
    assert (e["p"], e["n"]) == pn


@pytest.mark.parametrize("pn", [(9, 2), (12, 1), (10, 0)])
def test_wide_tile_taylor_orders(pn):
    # padded d 256 (64 x 128 stage tiles): Paterson-Stockmeyer blocks with
    # a second output, extra addends and both endings, then squarings
    rng = np.random.default_rng(43)
    p = workloads.random_problem(rng, d=256, M=2, N=6, S=2, dt=0.1, scale=1.5)
    out, ref, e = compare(f"wide_orders_p{pn[0]}_n{pn[1]}", p, taylor_pn=pn)
    check(p, e)
    assert (e["p"], e["n"]) == pn


def test_fixed_taylor_parameters():
    p = workloads.config2().with_steps(400)
    out, ref, e = compare("c2_fixed_pn", p, taylor_pn=(12, 2))
    check(p, e)
    assert (e["p"], e["n"]) == (12, 2)


@pytest.mark.parametrize("d,S,pn", [(30, 2, (9, 2)), (40, 3, (10, 3)), (40, 40, (8, 2))])
def test_fixed_pair_small_path_batched_adjoint(d, S, pn):
    # padded d 32 / 48 with a fixed pair: device-side chains, batched adjoint
    rng = np.random.default_rng(300 + d + S)
    p = workloads.random_problem(rng, d=d, M=3, N=45, S=S, dt=0.2, scale=2.0)
    out, ref, e = compare(f"fixed_small_d{d}_S{S}", p, taylor_pn=pn)
    check(p, e)
    assert (e["p"], e["n"]) == pn


def test_no_controls_and_no_penalty():
    rng = np.random.default_rng(11)
    p = workloads.random_problem(rng, d=6, M=0, N=20, S=2, with_penalty=False)
    out, ref, e = compare("rand_M0", p)
    check(p, e)


def test_fp64_chains_match_oracle_tightly():
    p = workloads.config2().with_steps(500)
    out, ref, e = compare("c2_fp64", p, precision="fp64")
    check(p, e, precision="fp64")
    rng = np.random.default_rng(12)
    q = workloads.random_problem(rng, d=70, M=2, N=20, S=3, dt=0.3, scale=2.0)
    out, ref, e = compare("rand_d70_fp64", q, precision="fp64")
    check(q, e, precision="fp64")


def test_config3_transmon_cavity_reduced_steps():
    p = workloads.config3().with_steps(800)
    out, ref, e = compare("c3_N800", p)
    check(p, e)


def test_config4_spin_chain_reduced_steps():
    p = workloads.config4().with_steps(24)
    out, ref, e = compare("c4_N24", p)
    check(p, e)


def test_directional_derivative_fp64_gpu():
    """Central difference of the GPU cost along a random direction equals
    <grad, v> (FP64 chains), at the full two-transmon size."""
    p = workloads.config2()
    h = qoc.Problem(p, precision="fp64", taylor_pn=(10, 2))
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p.u.shape)
    g = h.cost_grad(p.u)["grad"]
    eps = 1e-5
    cp = h.cost_grad(p.u + eps * v)["C"]
    cm = h.cost_grad(p.u - eps * v)["C"]
    fd = (cp - cm) / (2 * eps)
    an = float(np.sum(g * v))
    say(f"[parity] fd_direction: fd={fd!r} analytic={an!r}")
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
    h.close()
