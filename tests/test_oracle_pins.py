"""Pins of the FP64 oracle against facts it does not compute itself.

Each test checks the oracle against something independent of its own code:
closed forms (Pauli rotations, Rabi drive, diagonal Hamiltonians),
library routines with different algorithms (scipy's Pade expm and
expm_frechet, mpmath at 50 digits), brute-force central finite differences,
and invariances of the cost.  A dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from workloads import (Problem, SIGMA_X, SIGMA_Y, SIGMA_Z, config1, random_problem,
                       haar_state)


def rabi_problem(theta, N=20, dt=0.1, S=2, w=None, alpha_pen=0.0):
    """Constant resonant drive on a qubit: total angle theta about x."""
    H0 = np.zeros((2, 2), complex)
    Hk = np.stack([SIGMA_X / 2, SIGMA_Y / 2])
    u = np.zeros((2, N))
    u[0, :] = theta / (N * dt)
    if S == 2:
        psi0 = np.eye(2, dtype=complex)
        psiT = SIGMA_X.T.copy()
    else:
        psi0 = np.array([[1, 0]], complex)
        psiT = np.array([[0, 1]], complex)
    return Problem("rabi", 2, 2, N, S, dt, H0, Hk, u, psi0, psiT, w=w,
                   alpha_fid=1.0, alpha_pen=alpha_pen)


def fd_grad(prob, h=1e-6):
    g = np.zeros_like(prob.u)
    for k in range(prob.M):
        for j in range(prob.N):
            up = prob.u.copy(); up[k, j] += h
            um = prob.u.copy(); um[k, j] -= h
            g[k, j] = (oracle.cost(prob, up)["C"] - oracle.cost(prob, um)["C"]) / (2 * h)
    return g


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ------------------------------------------------------------ exponentials
def test_expm_diagonal_exact_phases():
    rng = np.random.default_rng(1)
    d, N = 5, 4
    h0 = rng.normal(size=d)
    hk = rng.normal(size=(2, d))
    p = Problem("diag", d, 2, N, 1, 0.3, np.diag(h0).astype(complex),
                np.stack([np.diag(x).astype(complex) for x in hk]),
                rng.normal(size=(2, N)), np.eye(d, dtype=complex)[:1],
                np.eye(d, dtype=complex)[:1])
    U, _, _ = oracle.propagators(p)
    for j in range(N):
        e = h0 + p.u[0, j] * hk[0] + p.u[1, j] * hk[1]
        assert np.allclose(U[j], np.diag(np.exp(-1j * 0.3 * e)), atol=1e-14, rtol=0)


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, math.pi, 5.9])
def test_expm_pauli_closed_form(theta):
    nvec = np.array([0.48, -0.6, 0.64])
    ns = nvec[0] * SIGMA_X + nvec[1] * SIGMA_Y + nvec[2] * SIGMA_Z
    dt = 0.25
    p = Problem("pauli", 2, 1, 1, 1, dt, np.zeros((2, 2), complex),
                (ns / 2)[None], np.array([[theta / dt]]), np.eye(2, dtype=complex)[:1],
                np.eye(2, dtype=complex)[:1])
    U, _, _ = oracle.propagators(p)
    ref = math.cos(theta / 2) * np.eye(2) - 1j * math.sin(theta / 2) * ns
    assert np.max(np.abs(U[0] - ref)) < 1e-14


def test_expm_matches_scipy_pade():
    rng = np.random.default_rng(2)
    p = random_problem(rng, d=8, M=3, N=6, S=2, dt=0.7, scale=2.0)
    U, _, _ = oracle.propagators(p)
    H = oracle.step_hamiltonians(p)
    for j in range(p.N):
        assert np.max(np.abs(U[j] - sla.expm(-1j * p.dt * H[j]))) < 1e-13


def test_expm_matches_mpmath_50_digits():
    rng = np.random.default_rng(3)
    p = random_problem(rng, d=3, M=1, N=2, S=1, dt=0.9, scale=1.5)
    U, _, _ = oracle.propagators(p)
    H = oracle.step_hamiltonians(p)
    mpmath.mp.dps = 50
    for j in range(p.N):
        A = mpmath.matrix([[(-1j * p.dt * H[j][a, b]) for b in range(3)] for a in range(3)])
        E = mpmath.expm(A)
        ref = np.array([[complex(E[a, b]) for b in range(3)] for a in range(3)])
        assert np.max(np.abs(U[j] - ref)) < 1e-14


def test_unitarity_and_semigroup():
    rng = np.random.default_rng(4)
    p = random_problem(rng, d=6, M=2, N=3, S=1, dt=0.4, scale=3.0)
    U, _, _ = oracle.propagators(p)
    for j in range(p.N):
        assert np.max(np.abs(U[j].conj().T @ U[j] - np.eye(6))) < 1e-13
    assert oracle.cost(p)["unitarity_drift"] < 1e-13
    # e^A e^A = e^{2A}: two steps of dt equal one step of 2 dt
    p1 = p.with_u(np.repeat(p.u[:, :1], 2, axis=1)).with_steps(2)
    p2 = Problem("x", 6, 2, 1, 1, 2 * p.dt, p.H0, p.Hk, p.u[:, :1], p.psi0, p.psiT)
    U1, _, _ = oracle.propagators(p1)
    U2, _, _ = oracle.propagators(p2)
    assert np.max(np.abs(U1[1] @ U1[0] - U2[0])) < 1e-13


# ------------------------------------------------------- propagation + cost
@pytest.mark.parametrize("theta", [0.0, 0.4, 1.0, math.pi / 2, 2.5, math.pi, 4.0])
def test_rabi_cost_closed_form(theta):
    out = oracle.cost(rabi_problem(theta))
    assert abs(out["C"] - math.cos(theta / 2) ** 2) < 1e-14
    assert abs(out["F"] - math.sin(theta / 2) ** 2) < 1e-14


@pytest.mark.parametrize("theta", [0.3, 1.3, 2.9])
def test_rabi_gradient_closed_form(theta):
    p = rabi_problem(theta, N=12)
    g = oracle.cost_grad(p)["grad"]
    assert np.max(np.abs(g[0] - (-(p.dt / 2) * math.sin(theta)))) < 1e-13
    assert np.max(np.abs(g[1])) < 1e-13


def test_rabi_penalty_closed_form():
    theta, N = 2.2, 16
    p = rabi_problem(theta, N=N, S=1, w=np.array([0.0, 1.0]), alpha_pen=0.7)
    out = oracle.cost(p)
    th_j = theta * np.arange(1, N + 1) / N
    assert np.max(np.abs(out["c"] - np.sin(th_j / 2) ** 2)) < 1e-14
    # S=1: |0> -> |1> has C_fid = cos^2(theta/2)
    assert abs(out["C_fid"] - math.cos(theta / 2) ** 2) < 1e-14
    assert abs(out["C"] - (out["C_fid"] + 0.7 * out["c"].sum())) < 1e-13


def test_penalty_with_unit_weights_is_constant():
    rng = np.random.default_rng(5)
    p = random_problem(rng, d=4, M=2, N=7, S=3, alphas=(1.0, 0.4, 0.0, 0.0))
    p.w = np.ones(4)
    out = oracle.cost_grad(p)
    assert np.max(np.abs(out["c"] - 1.0)) < 1e-14
    q = random_problem(np.random.default_rng(5), d=4, M=2, N=7, S=3,
                       alphas=(1.0, 0.0, 0.0, 0.0))
    assert np.max(np.abs(out["grad"] - oracle.cost_grad(q)["grad"])) < 1e-13


def test_regularizers_closed_form():
    N = 9
    u = np.vstack([np.full(N, 0.3), 0.1 * np.arange(N)])
    c_amp, c_var = oracle.regularizers(u)
    assert abs(c_amp - (N * 0.09 + 0.01 * sum(j * j for j in range(N)))) < 1e-14
    assert abs(c_var - (N - 1) * 0.01) < 1e-14


def test_full_basis_equals_gate_infidelity():
    """S = d with identity columns reproduces 1 - |tr(K_T^dag K_N)/D|^2."""
    rng = np.random.default_rng(6)
    d = 4
    p = random_problem(rng, d=d, M=2, N=5, S=d, with_penalty=False,
                       alphas=(1.0, 0, 0, 0))
    KT = sla.expm(-1j * (lambda A: A + A.conj().T)(rng.normal(size=(d, d)) + 0j))
    p.psi0 = np.eye(d, dtype=complex)
    p.psiT = KT.T.copy()                     # row s = column s of K_T
    H = oracle.step_hamiltonians(p)
    K = np.eye(d, dtype=complex)
    for j in range(p.N):
        K = sla.expm(-1j * p.dt * H[j]) @ K
    ref = 1.0 - abs(np.trace(KT.conj().T @ K) / d) ** 2
    assert abs(oracle.cost(p)["C_fid"] - ref) < 1e-13


# ------------------------------------------------------------ gradients
@pytest.mark.parametrize("mode", ["coherent", "incoherent"])
@pytest.mark.parametrize("seed", [7, 8])
def test_gradient_matches_central_fd(mode, seed):
    rng = np.random.default_rng(seed)
    p = random_problem(rng, d=3, M=2, N=5, S=2, dt=0.35, scale=1.3,
                       fid_mode=mode, alphas=(1.0, 0.3, 0.05, 0.02))
    g = oracle.cost_grad(p)["grad"]
    assert rel(g, fd_grad(p)) < 1e-7


def test_gradient_fd_single_column_and_no_controls_edge():
    rng = np.random.default_rng(9)
    p = random_problem(rng, d=4, M=1, N=3, S=1, dt=0.5)
    assert rel(oracle.cost_grad(p)["grad"], fd_grad(p)) < 1e-7
    q = random_problem(rng, d=3, M=0, N=4, S=1)
    out = oracle.cost_grad(q)
    assert out["grad"].shape == (0, 4)


def test_frechet_matches_scipy_and_block_formula():
    rng = np.random.default_rng(10)
    d, dt = 5, 0.6
    A0 = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    H = (A0 + A0.conj().T) / 2
    E = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    lam, V = np.linalg.eigh(H)
    A = -1j * dt * H
    L = oracle.frechet_exp_skew(lam, V, dt, E)
    _, L_sp = sla.expm_frechet(A, E)
    assert np.max(np.abs(L - L_sp)) < 1e-13
    blk = sla.expm(np.block([[A, E], [np.zeros((d, d)), A]]))[:d, d:]
    assert np.max(np.abs(L - blk)) < 1e-13
    La = oracle.frechet_exp_skew(lam, V, dt, E, adjoint=True)
    _, La_sp = sla.expm_frechet(A.conj().T, E)
    assert np.max(np.abs(La - La_sp)) < 1e-13


def test_frechet_degenerate_eigenvalues():
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    H = Q @ np.diag([1.0, 1.0, -0.5, 1.0]) @ Q.conj().T
    E = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    lam, V = np.linalg.eigh(H)
    _, L_sp = sla.expm_frechet(-1j * 0.8 * H, E)
    assert np.max(np.abs(oracle.frechet_exp_skew(lam, V, 0.8, E) - L_sp)) < 1e-13


def test_adjoint_identity_trace():
    rng = np.random.default_rng(12)
    d, dt = 4, 0.9
    A0 = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    H = (A0 + A0.conj().T) / 2
    lam, V = np.linalg.eigh(H)
    G = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    E = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    _, L = sla.expm_frechet(-1j * dt * H, E)
    lhs = np.vdot(G, L)
    rhs = np.vdot(oracle.frechet_exp_skew(lam, V, dt, G, adjoint=True), E)
    assert abs(lhs - rhs) < 1e-12


def test_commuting_case_exact_equals_first_order():
    rng = np.random.default_rng(13)
    d, N = 4, 6
    p = Problem("diag", d, 2, N, 2, 0.4,
                np.diag(rng.normal(size=d)).astype(complex),
                np.stack([np.diag(rng.normal(size=d)).astype(complex) for _ in range(2)]),
                rng.uniform(-1, 1, size=(2, N)),
                np.stack([haar_state(rng, d) for _ in range(2)]),
                np.stack([haar_state(rng, d) for _ in range(2)]), alpha_fid=1.0)
    g = oracle.cost_grad(p)["grad"]
    assert np.max(np.abs(g - oracle.gradient_first_order(p))) < 1e-13
    # fidelity-only, commuting: dC/du_{k,j} does not depend on j
    assert np.max(np.abs(g - g[:, :1])) < 1e-13
    assert rel(g, fd_grad(p)) < 1e-7


def test_first_order_gradient_is_only_approximate():
    rng = np.random.default_rng(14)
    p = random_problem(rng, d=3, M=2, N=5, S=2, dt=0.6, scale=2.0,
                       alphas=(1.0, 0.0, 0.0, 0.0), with_penalty=False)
    exact = oracle.cost_grad(p)["grad"]
    assert rel(oracle.gradient_first_order(p), exact) > 1e-2


# ------------------------------------------------------------ invariances
def test_invariance_target_phase_and_energy_shift():
    rng = np.random.default_rng(15)
    p = random_problem(rng, d=4, M=2, N=6, S=2)
    base = oracle.cost_grad(p)
    q = random_problem(np.random.default_rng(15), d=4, M=2, N=6, S=2)
    q.psiT = np.exp(0.77j) * q.psiT
    q.H0 = q.H0 + 1.9 * np.eye(4)
    out = oracle.cost_grad(q)
    assert abs(out["C"] - base["C"]) < 1e-13
    assert np.max(np.abs(out["grad"] - base["grad"])) < 1e-12


# ------------------------------------------------------------ (p, n) rule
@pytest.mark.parametrize("theta", [1e-3, 0.034, 0.37, 1.0, 4.66, 12.0])
def test_taylor_rule_meets_tolerance(theta):
    rng = np.random.default_rng(16)
    A0 = rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6))
    H = (A0 + A0.conj().T) / 2
    H = H * theta / np.abs(H).sum(axis=0).max()        # ||H||_1 = theta, dt = 1
    for tau in (1e-10, 1e-14):
        p, n = oracle.taylor_select(theta, tau)
        err = np.max(np.abs(oracle.taylor_squaring_expm(-1j * H, p, n) - sla.expm(-1j * H)))
        assert err <= tau + 1e-14
        # brute force: no pair with fewer products satisfies the bound
        G = p - 1 + n
        for nn in range(G + 1):
            for pp in range(2, G - nn + 2):
                if pp - 1 + nn < G:
                    assert oracle.taylor_bound(theta, pp, nn) > tau


def test_taylor_approximant_converges_to_expm():
    rng = np.random.default_rng(17)
    A0 = rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5))
    A = -1j * (A0 + A0.conj().T)
    assert np.max(np.abs(oracle.taylor_squaring_expm(A, 30, 6) - sla.expm(A))) < 1e-13
    # p = 1, n = 0 is the first-order (Euler) formula I + A
    assert np.allclose(oracle.taylor_squaring_expm(A, 1, 0), np.eye(5) + A)


def test_config1_theta_and_cost_sane():
    p = config1()
    out = oracle.cost_grad(p)
    assert 0.0 <= out["C"] <= 1.0
    assert out["grad"].shape == (2, 200)
    assert oracle.taylor_select(out["theta_max"], 1e-10)[1] == 0


@pytest.mark.parametrize("theta", [0.5, 2.0, 7.0])
def test_taylor_bound_is_tight_on_scalar_rotation(theta):
    """For the 1x1 generator -i theta the squared Taylor error is ~2^n x^(p+1)/(p+1)!:
    the bound must hold, and be within a factor of a few of the true error."""
    for n in range(0, 6):
        for p in range(2, 9):
            approx = oracle.taylor_squaring_expm(np.array([[-1j * theta]]), p, n)[0, 0]
            err = abs(approx - np.exp(-1j * theta))
            b = oracle.taylor_bound(theta, p, n)
            if err > 1e-13:
                assert err <= b * (1 + 1e-9)
                if theta / 2 ** n <= 1.0 and err < 1e-2:
                    assert b <= 4.0 * math.exp(theta / 2 ** n) * err


# ------------------------------------------------------------ step norms
def test_step_norms_closed_forms():
    """theta_j = ||dt H_j||_1, the largest column absolute sum (Sec. III).
    Diagonal H_j: dt max_m |h_m(j)|.  A dense real symmetric H with column
    absolute sums (3, 5) separates the 1-norm (5) from the Frobenius norm
    (sqrt(18)) and the spectral norm (1 + 2 sqrt(2))."""
    rng = np.random.default_rng(18)
    d, N, dt = 5, 6, 0.3
    h0 = rng.normal(size=d)
    hk = rng.normal(size=(2, d))
    u = rng.normal(size=(2, N))
    p = Problem("diag", d, 2, N, 1, dt, np.diag(h0).astype(complex),
                np.stack([np.diag(x).astype(complex) for x in hk]), u,
                np.eye(d, dtype=complex)[:1], np.eye(d, dtype=complex)[:1])
    ref = [dt * np.max(np.abs(h0 + u[0, j] * hk[0] + u[1, j] * hk[1])) for j in range(N)]
    assert np.max(np.abs(oracle.step_norms(p) - np.array(ref))) < 1e-14
    H = np.array([[1.0, 2.0], [2.0, -3.0]], dtype=complex)
    q = Problem("dense", 2, 1, 2, 1, 0.5, H, np.zeros((1, 2, 2), complex),
                np.array([[0.0, 1.0]]), np.eye(2, dtype=complex)[:1],
                np.eye(2, dtype=complex)[:1])
    q.Hk[0] = np.array([[0.0, 1j], [-1j, 0.0]])           # adds |i| to both columns at j=1
    th = oracle.step_norms(q)
    assert abs(th[0] - 0.5 * 5.0) < 1e-15
    assert abs(th[1] - 0.5 * (3.0 + abs(2.0 + 1j))) < 1e-15


# ------------------------------------------- forbidden states (C5), C6 / C7
def test_forbidden_basis_states_equal_level_weights():
    """Forbidden states sqrt(w_m) e_m give the per-step penalties, cost and
    gradient of the level weights w (Table I, C5: a set of forbidden states
    enters upon summation)."""
    rng = np.random.default_rng(19)
    p = random_problem(rng, d=4, M=2, N=6, S=2, dt=0.4, scale=1.5)
    q = random_problem(np.random.default_rng(19), d=4, M=2, N=6, S=2, dt=0.4, scale=1.5)
    q.forbidden = np.diag(np.sqrt(q.w)).astype(complex)
    q.w = None
    a, b = oracle.cost_grad(p), oracle.cost_grad(q)
    assert np.max(np.abs(a["c"] - b["c"])) < 1e-14
    assert abs(a["C"] - b["C"]) < 1e-13
    assert np.max(np.abs(a["grad"] - b["grad"])) < 1e-13


def test_forbidden_state_rabi_closed_form_and_phase():
    """Rabi drive |0> -> |1> with the forbidden state e^{i phi}|1>:
    c_j = sin^2(theta_j / 2) whatever the phase phi."""
    theta, N = 2.2, 16
    p = rabi_problem(theta, N=N, S=1, alpha_pen=0.7)
    p.forbidden = np.array([[0.0, np.exp(0.9j)]])
    out = oracle.cost(p)
    th_j = theta * np.arange(1, N + 1) / N
    assert np.max(np.abs(out["c"] - np.sin(th_j / 2) ** 2)) < 1e-14
    # a superposition forbidden state: |<F|psi_j>|^2 with psi_j = cos|0> - i sin|1>
    f = np.array([0.6, 0.8j])
    p.forbidden = f[None]
    ref = np.abs(0.6 * np.cos(th_j / 2) + (-0.8j) * (-1j * np.sin(th_j / 2))) ** 2
    assert np.max(np.abs(oracle.cost(p)["c"] - ref)) < 1e-14


@pytest.mark.parametrize("theta", [0.7, 2.0, 3.0])
def test_time_optimal_rabi_closed_form(theta):
    """C7 on the Rabi drive |0> -> |1>: F_j = sin^2(theta_j / 2), so
    C_time = 1 - (1/N) sum_j sin^2(theta_j / 2), and its gradient along the
    x control is -(1/N) sum_{k > j} (dt / 2) sin(theta_k), zero along y."""
    N, dt = 12, 0.1
    p = rabi_problem(theta, N=N, dt=dt, S=1)
    p.alpha_fid, p.alpha_time = 0.0, 1.0
    out = oracle.cost_grad(p)
    th = theta * np.arange(1, N + 1) / N
    assert abs(out["C_time"] - (1 - np.mean(np.sin(th / 2) ** 2))) < 1e-14
    assert abs(out["C"] - out["C_time"]) < 1e-14
    gx = np.array([-(dt / 2) * np.sum(np.sin(th[j:])) / N for j in range(N)])
    assert np.max(np.abs(out["grad"][0] - gx)) < 1e-14
    assert np.max(np.abs(out["grad"][1])) < 1e-14


def test_time_optimal_single_step_equals_final_fidelity():
    rng = np.random.default_rng(20)
    for mode in ("coherent", "incoherent"):
        p = random_problem(rng, d=3, M=2, N=1, S=2, fid_mode=mode, with_penalty=False,
                           alphas=(0.0, 0.0, 0.0, 0.0), alpha_time=1.0)
        out = oracle.cost_grad(p)
        assert abs(out["C_time"] - out["C_fid"]) < 1e-15
        q = random_problem(np.random.default_rng(20 if mode == "coherent" else 0), d=3, M=2,
                           N=1, S=2, fid_mode=mode, with_penalty=False,
                           alphas=(1.0, 0.0, 0.0, 0.0))
        if mode == "coherent":
            assert np.max(np.abs(out["grad"] - oracle.cost_grad(q)["grad"])) < 1e-14


@pytest.mark.parametrize("mode", ["coherent", "incoherent"])
def test_forbidden_and_time_optimal_gradient_matches_fd(mode):
    rng = np.random.default_rng(21)
    p = random_problem(rng, d=3, M=2, N=5, S=2, dt=0.35, scale=1.3, fid_mode=mode,
                       alphas=(1.0, 0.3, 0.05, 0.02), n_forbidden=2, alpha_time=0.6)
    assert rel(oracle.cost_grad(p)["grad"], fd_grad(p)) < 1e-7


# ------------------------------------------------------------ action form
def test_taylor_action_equals_matrix_approximant_and_expm():
    """The series applied to the columns is the same polynomial as the
    matrix approximant (exactly, up to rounding), and within the Taylor
    bound of the exact exponential."""
    rng = np.random.default_rng(30)
    d = 7
    A0 = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    H = (A0 + A0.conj().T) / 2
    H = H * 1.7 / np.abs(H).sum(axis=0).max()      # ||H||_1 = 1.7
    psi = np.stack([haar_state(rng, d) for _ in range(3)])
    for p, n in [(2, 0), (5, 1), (9, 3), (12, 0)]:
        got = oracle.taylor_action(-1j * H, psi, p, n)
        mat = psi @ oracle.taylor_squaring_expm(-1j * H, p, n).T
        assert np.max(np.abs(got - mat)) < 1e-13
        exact = psi @ sla.expm(-1j * H).T
        assert np.max(np.abs(got - exact)) <= oracle.taylor_bound(1.7, p, n) * (1 + 1e-9) + 1e-14


def test_taylor_action_diagonal_and_pauli_closed_forms():
    # diagonal generator: each component is the scalar truncated series,
    # applied 2^n times
    lam = np.array([0.3, -0.8, 1.1])
    psi = np.array([[1.0, 2.0, -1.0j]])
    p, n = 4, 2
    x = -1j * lam / 4
    scal = sum(x ** k / math.factorial(k) for k in range(p + 1)) ** 4
    got = oracle.taylor_action(np.diag(-1j * lam), psi, p, n)
    assert np.max(np.abs(got[0] - scal * psi[0])) < 1e-15
    # Pauli rotation exp(-i theta sigma_x / 2) |0> = (cos, -i sin), long series
    theta = 1.3
    got = oracle.taylor_action(-1j * theta / 2 * SIGMA_X, np.array([[1.0, 0.0]]), 30, 2)
    assert np.max(np.abs(got[0] - [math.cos(theta / 2), -1j * math.sin(theta / 2)])) < 1e-15


def test_action_rule_hand_values_and_brute_force():
    """theta = 0.81: order 11 leaves 3.7e-10 > 1e-10, order 12 2.3e-11, and
    n = 1 needs order 9 (18 products): (12, 0).  theta = 3: n >= 2 for
    theta / 2^n <= 1; n = 2 needs order 12 (48 products), n = 3 order 10
    (80): (12, 2).  Every choice meets the bound and no pair with fewer
    products (and theta / 2^n <= 1) does."""
    assert oracle.action_select(0.81, 1e-10) == (12, 0)
    assert oracle.action_select(3.0, 1e-10) == (12, 2)
    assert oracle.action_select(0.0, 1e-10) == (2, 0)
    for theta in (1e-3, 0.37, 0.81, 1.0, 3.0, 12.0, 70.0):
        for tau in (1e-10, 1e-15):
            p, n = oracle.action_select(theta, tau)
            assert oracle.taylor_bound(theta, p, n) <= tau and theta / 2 ** n <= 1.0
            for nn in range(0, 12):
                for pp in range(2, 31):
                    if pp * 2 ** nn < p * 2 ** n and theta / 2 ** nn <= 1.0:
                        assert oracle.taylor_bound(theta, pp, nn) > tau


def test_action_rule_meets_tolerance_on_a_generator():
    rng = np.random.default_rng(31)
    d = 6
    A0 = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    H = (A0 + A0.conj().T) / 2
    psi = np.stack([haar_state(rng, d) for _ in range(2)])
    for theta in (0.2, 2.5, 9.0):
        Hs = H * theta / np.abs(H).sum(axis=0).max()
        p, n = oracle.action_select(theta, 1e-12)
        err = np.max(np.abs(oracle.taylor_action(-1j * Hs, psi, p, n) - psi @ sla.expm(-1j * Hs).T))
        assert err <= 1e-12


# ------------------------------------------------------------ PS product count
def _ps_counted(X, p, s):
    """T_p(X) by Paterson-Stockmeyer with block size s, counting the matrix
    products actually performed (a scalar-identity top block is scaled, not
    multiplied)."""
    count = [0]

    def mul(A, B):
        count[0] += 1
        return A @ B

    I = np.eye(X.shape[0], dtype=complex)
    pw = [I, X]
    for _ in range(2, s + 1):
        pw.append(mul(pw[-1], X))
    c = [1.0 / math.factorial(k) for k in range(p + 1)]
    Q = p // s

    def block(q):
        return sum(c[q * s + r] * pw[r] for r in range(s) if q * s + r <= p)

    if p % s == 0:  # top block c_p I: its Horner step is a scaling
        W = block(Q - 1) + c[p] * pw[s]
        top = Q - 2
    else:
        W = block(Q)
        top = Q - 1
    for q in range(top, -1, -1):
        W = block(q) + mul(pw[s], W)
    return W, count[0]


def test_ps_products_counted():
    rng = np.random.default_rng(40)
    X = (rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5))) * 0.3
    for p in range(2, 21):
        ref = oracle.taylor_squaring_expm(X, p, 0)
        counts = [p - 1]  # Horner
        for s in range(2, min(p, 4) + 1):
            W, k = _ps_counted(X, p, s)
            assert np.max(np.abs(W - ref)) < 1e-13
            counts.append(k)
        assert oracle.ps_products(p) == min(counts), (p, counts)


def test_ps_rule_hand_values_and_brute_force():
    """theta = 0.81: (12, 0) takes 5 products, (9, 1) 4 + 1 (tie: the lower
    order), (8, 2) 4 + 2.  theta = 3: n >= 2; (12, 2) takes 5 + 2, n = 3
    needs order 10 (5 + 3)."""
    assert oracle.taylor_select_ps(0.81, 1e-10) == (9, 1)
    assert oracle.taylor_select_ps(3.0, 1e-10) == (12, 2)
    for theta in (1e-3, 0.37, 0.81, 1.0, 3.0, 4.83, 12.0, 70.0):
        for tau in (1e-10, 1e-15):
            p, n = oracle.taylor_select_ps(theta, tau)
            assert oracle.taylor_bound(theta, p, n) <= tau and theta / 2 ** n <= 1.0
            cost = oracle.ps_products(p) + n
            for nn in range(0, 12):
                for pp in range(2, 31):
                    cheaper = oracle.ps_products(pp) + nn < cost
                    tie_lower = oracle.ps_products(pp) + nn == cost and pp < p
                    if (cheaper or tie_lower) and theta / 2 ** nn <= 1.0:
                        assert oracle.taylor_bound(theta, pp, nn) > tau
