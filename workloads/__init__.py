"""Seeded synthetic inputs for the piecewise-constant optimal-control problem.

This module builds *inputs only*: drift and control Hamiltonians, control
amplitudes, initial and target states, forbidden-level weights and cost
weights.  It contains none of the method's arithmetic (no exponentials, no
propagation, no costs, no gradients), so that the FP64 oracle and the GPU
path can both draw their inputs from it without sharing any computation.

The physical models follow the systems of the paper's showcase section
(Sec. IV: coupled transmons, a transmon dispersively coupled to a cavity,
a spin chain with sigma_z sigma_z coupling), re-parameterised as stated per
configuration below.  Units: hbar = 1, Hamiltonians in rad/ns, dt in ns
(Sec. II sets hbar = 1 after eq. (3)).

Conventions shared by every generator
-------------------------------------
* ``a`` is the truncated annihilator with ``a[m-1, m] = sqrt(m)``;
  ``n = a^dagger a``; Paulis are the standard ones.
* Kronecker order puts the first-named subsystem as the most significant
  index (``index = n_1 * levels_2 + n_2``).
* States are stored as rows: ``psi0[s]`` is the s-th initial state (a
  length-``d`` complex vector), ``psiT[s]`` the s-th target state.
* Controls are stored ``u[k, j]`` (control k, time step j).
* RNG: ``numpy.random.default_rng(1000 + c)`` for configuration ``c``
  (1-based), draws in the order: on-site fields, controls, initial states,
  target states.  The batched configuration uses
  ``numpy.random.SeedSequence(1005).spawn(256)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Problem:
    """One optimal-control instance (inputs of the cost and gradient).

    Field names follow the paper's notation (Sec. II, Table I): ``H0`` is the
    drift Hamiltonian, ``Hk[k]`` the k-th control Hamiltonian, ``u[k, j]``
    the control amplitude of control k on step j, ``dt`` the step length.
    """

    name: str
    d: int
    M: int
    N: int
    S: int
    dt: float
    H0: np.ndarray            # (d, d) complex128, Hermitian
    Hk: np.ndarray            # (M, d, d) complex128, Hermitian
    u: np.ndarray             # (M, N) float64
    psi0: np.ndarray          # (S, d) complex128, row s = initial state s
    psiT: np.ndarray          # (S, d) complex128, row s = target state s
    w: Optional[np.ndarray] = None   # (d,) float64 forbidden-level weights, or None
    alpha_fid: float = 1.0
    alpha_pen: float = 0.0
    alpha_amp: float = 0.0
    alpha_var: float = 0.0
    fid_mode: str = "coherent"       # "coherent" (C2-sigma) or "incoherent"
    meta: dict = field(default_factory=dict)
    forbidden: Optional[np.ndarray] = None   # (F, d) complex128 forbidden states, or None
    alpha_time: float = 0.0          # weight of the time-optimal term (Table I, C6 / C7)

    def with_u(self, u: np.ndarray) -> "Problem":
        return replace(self, u=np.ascontiguousarray(u, dtype=np.float64))

    def with_steps(self, N: int) -> "Problem":
        """Same physics, first ``N`` steps of the control array."""
        return replace(self, N=int(N), u=np.ascontiguousarray(self.u[:, :N]))


# ----------------------------------------------------------------- operators
def annihilator(levels: int) -> np.ndarray:
    a = np.zeros((levels, levels), dtype=np.complex128)
    for m in range(1, levels):
        a[m - 1, m] = math.sqrt(m)
    return a


def number_op(levels: int) -> np.ndarray:
    return np.diag(np.arange(levels, dtype=np.float64)).astype(np.complex128)


SIGMA_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)


def embed(ops_by_site: dict, dims: List[int]) -> np.ndarray:
    """Kronecker product over sites, first site most significant."""
    out = np.ones((1, 1), dtype=np.complex128)
    for i, n in enumerate(dims):
        out = np.kron(out, ops_by_site.get(i, np.eye(n, dtype=np.complex128)))
    return out


def basis(d: int, m: int) -> np.ndarray:
    v = np.zeros(d, dtype=np.complex128)
    v[m] = 1.0
    return v


def haar_state(rng: np.random.Generator, d: int) -> np.ndarray:
    """Normalised complex Gaussian vector (Haar-distributed pure state)."""
    v = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------- configurations
def config1(seed: int = 1001) -> Problem:
    """Single qubit, d=2: H0=0, controls sigma_x/2 and sigma_y/2, X gate.

    N=200, dt=0.1 ns, u ~ U[-0.5, 0.5] rad/ns, S=2 columns of the identity
    mapped to the columns of X; fidelity weight only.
    """
    rng = np.random.default_rng(seed)
    H0 = np.zeros((2, 2), dtype=np.complex128)
    Hk = np.stack([SIGMA_X / 2, SIGMA_Y / 2])
    N = 200
    u = rng.uniform(-0.5, 0.5, size=(2, N))
    psi0 = np.eye(2, dtype=np.complex128)
    psiT = SIGMA_X.T.copy()      # rows = columns of X
    return Problem("c1_qubit_x", 2, 2, N, 2, 0.1, H0, Hk, u, psi0, psiT,
                   alpha_fid=1.0)


def config2(seed: int = 1002) -> Problem:
    """Two transmons x 4 levels (d=16), rotating frame, CNOT on 4 columns.

    H0 = sum_i [Delta_i n_i + (alpha/2) n_i (n_i - 1)] + g (a1^+ a2 + a1 a2^+),
    Delta = (0, 2pi*0.1), alpha = -2pi*0.22, g = 2pi*0.005 (rad/ns).
    Controls: a1+a1^+, i(a1-a1^+), a2+a2^+, i(a2-a2^+).  N=2000, dt=0.05.
    u ~ N(0, (2pi*0.02)^2).  Columns e0,e1,e4,e5 -> e0,e1,e5,e4 (transmon 1
    is the control qubit).  Forbidden weights: levels with n1=3 or n2=3.
    Cost weights: fid 1, pen 1e-2, amp 1e-4, var 1e-3.
    """
    rng = np.random.default_rng(seed)
    L = 4
    dims = [L, L]
    a, n = annihilator(L), number_op(L)
    delta = (0.0, TWO_PI * 0.1)
    alpha = -TWO_PI * 0.22
    g = TWO_PI * 0.005
    I = np.eye(L, dtype=np.complex128)
    H0 = np.zeros((16, 16), dtype=np.complex128)
    for i in range(2):
        H0 += embed({i: delta[i] * n + 0.5 * alpha * n @ (n - I)}, dims)
    a1, a2 = embed({0: a}, dims), embed({1: a}, dims)
    H0 += g * (a1.conj().T @ a2 + a1 @ a2.conj().T)
    Hk = np.stack([a1 + a1.conj().T, 1j * (a1 - a1.conj().T),
                   a2 + a2.conj().T, 1j * (a2 - a2.conj().T)])
    N = 2000
    u = rng.normal(0.0, TWO_PI * 0.02, size=(4, N))
    cols_in = [0, 1, 4, 5]
    cols_out = [0, 1, 5, 4]
    psi0 = np.stack([basis(16, m) for m in cols_in])
    psiT = np.stack([basis(16, m) for m in cols_out])
    w = np.array([1.0 if (m // L == 3 or m % L == 3) else 0.0 for m in range(16)])
    return Problem("c2_transmon_cnot", 16, 4, N, 4, 0.05, H0, Hk, u, psi0, psiT,
                   w=w, alpha_fid=1.0, alpha_pen=1e-2, alpha_amp=1e-4,
                   alpha_var=1e-3)


def config3(seed: int = 1003) -> Problem:
    """Transmon (4 levels) x cavity (32 levels), d=128, |g,0> -> |g,3>.

    H0 = (alpha/2) nq (nq - 1) + chi nq nc, alpha = -2pi*0.2,
    chi = -2pi*0.002.  Controls: b+b^+, i(b-b^+), a+a^+, i(a-a^+) (b the
    transmon, a the cavity).  N=5000, dt=0.5, u ~ N(0, (2pi*0.02)^2).
    Forbidden weights on cavity levels nc >= 28; alpha_pen = 1e-2.
    """
    rng = np.random.default_rng(seed)
    Lq, Lc = 4, 32
    dims = [Lq, Lc]
    b, nq = annihilator(Lq), number_op(Lq)
    a, nc = annihilator(Lc), number_op(Lc)
    alpha = -TWO_PI * 0.2
    chi = -TWO_PI * 0.002
    Iq = np.eye(Lq, dtype=np.complex128)
    H0 = embed({0: 0.5 * alpha * nq @ (nq - Iq)}, dims) + chi * embed({0: nq, 1: nc}, dims)
    B, A = embed({0: b}, dims), embed({1: a}, dims)
    Hk = np.stack([B + B.conj().T, 1j * (B - B.conj().T),
                   A + A.conj().T, 1j * (A - A.conj().T)])
    N = 5000
    u = rng.normal(0.0, TWO_PI * 0.02, size=(4, N))
    d = Lq * Lc
    psi0 = basis(d, 0)[None, :]
    psiT = basis(d, 3)[None, :]
    w = np.array([1.0 if (m % Lc) >= 28 else 0.0 for m in range(d)])
    return Problem("c3_transmon_cavity", d, 4, N, 1, 0.5, H0, Hk, u, psi0, psiT,
                   w=w, alpha_fid=1.0, alpha_pen=1e-2)


def config4(seed: int = 1004, spins: int = 9) -> Problem:
    """Spin chain of 9 spins (d=512): sigma_z sigma_z coupling + fields.

    H0 = sum_i J sz_i sz_{i+1} + sum_i h_i sz_i, J = 2pi*0.01,
    h_i ~ U[-2pi*0.05, 2pi*0.05].  Controls sx_1..sx_9, sy_1..sy_9 (M=18).
    N=1000, dt=0.2, u ~ N(0, (2pi*0.02)^2).  S=8 Haar-random initial states
    mapped to 8 Haar-random targets; fidelity weight only.
    """
    rng = np.random.default_rng(seed)
    dims = [2] * spins
    d = 2 ** spins
    J = TWO_PI * 0.01
    h = rng.uniform(-TWO_PI * 0.05, TWO_PI * 0.05, size=spins)
    H0 = np.zeros((d, d), dtype=np.complex128)
    for i in range(spins - 1):
        H0 += J * embed({i: SIGMA_Z, i + 1: SIGMA_Z}, dims)
    for i in range(spins):
        H0 += h[i] * embed({i: SIGMA_Z}, dims)
    Hk = np.stack([embed({i: SIGMA_X}, dims) for i in range(spins)]
                  + [embed({i: SIGMA_Y}, dims) for i in range(spins)])
    N = 1000
    M = 2 * spins
    u = rng.normal(0.0, TWO_PI * 0.02, size=(M, N))
    S = 8
    psi0 = np.stack([haar_state(rng, d) for _ in range(S)])
    psiT = np.stack([haar_state(rng, d) for _ in range(S)])
    return Problem("c4_spin_chain", d, M, N, S, 0.2, H0, Hk, u, psi0, psiT,
                   alpha_fid=1.0, meta={"h": h})


def transmon_chain(rng: np.random.Generator, d: int, M: int, N: int,
                   name: str = "c5_instance") -> Problem:
    """One instance of the batched uneven workload.

    q = max(1, ceil(log4 d)) transmons with 4 levels each, the two-transmon
    drift form extended to a chain (detuning 2pi*0.1*(i-1), anharmonicity
    -2pi*0.22, nearest-neighbour exchange 2pi*0.005), truncated to the d
    levels of lowest drift diagonal (ties broken by index, kept in index
    order).  Controls in the order x_1, y_1, x_2, y_2, ..., then n_1, n_2,
    ...; the first M are used.  u ~ U[-0.5, 0.5], dt = 0.1, S = 2,
    e0, e1 -> e1, e0.
    """
    L = 4
    q = max(1, math.ceil(math.log(d, 4) - 1e-12))
    dims = [L] * q
    a, n = annihilator(L), number_op(L)
    I = np.eye(L, dtype=np.complex128)
    alpha = -TWO_PI * 0.22
    g = TWO_PI * 0.005
    D = L ** q
    H0 = np.zeros((D, D), dtype=np.complex128)
    ai = [embed({i: a}, dims) for i in range(q)]
    for i in range(q):
        H0 += embed({i: TWO_PI * 0.1 * i * n + 0.5 * alpha * n @ (n - I)}, dims)
    for i in range(q - 1):
        H0 += g * (ai[i].conj().T @ ai[i + 1] + ai[i] @ ai[i + 1].conj().T)
    ctrl = []
    for i in range(q):
        ctrl.append(ai[i] + ai[i].conj().T)
        ctrl.append(1j * (ai[i] - ai[i].conj().T))
    for i in range(q):
        ctrl.append(ai[i].conj().T @ ai[i])
    while len(ctrl) < M:              # only reachable for q=1 and M>3
        ctrl.append(ctrl[len(ctrl) % 3])
    diag = np.real(np.diag(H0))
    keep = np.sort(np.argsort(diag, kind="stable")[:d])
    sel = np.ix_(keep, keep)
    H0 = np.ascontiguousarray(H0[sel])
    Hk = np.stack([np.ascontiguousarray(c[sel]) for c in ctrl[:M]])
    u = rng.uniform(-0.5, 0.5, size=(M, N))
    psi0 = np.stack([basis(d, 0), basis(d, 1)])
    psiT = np.stack([basis(d, 1), basis(d, 0)])
    return Problem(name, d, M, N, 2, 0.1, H0, Hk, u, psi0, psiT, alpha_fid=1.0)


def config5(count: int = 256, seed: int = 1005) -> List[Problem]:
    """256 independent instances: d log-uniform in 2..128, N in 100..3000,
    M in 2..6 (see :func:`transmon_chain`)."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        d = int(round(math.exp(rng.uniform(math.log(2), math.log(128)))))
        d = min(max(d, 2), 128)
        N = int(rng.integers(100, 3001))
        M = int(rng.integers(2, 7))
        out.append(transmon_chain(rng, d, M, N, name=f"c5_{i:03d}"))
    return out


CONFIGS = {"c1": config1, "c2": config2, "c3": config3, "c4": config4}


def make_config(name: str, **kw) -> Problem:
    return CONFIGS[name](**kw)


def random_problem(rng: np.random.Generator, d: int, M: int, N: int, S: int,
                   dt: float = 0.1, scale: float = 1.0, u_scale: float = 0.5,
                   with_penalty: bool = True, fid_mode: str = "coherent",
                   alphas=(1.0, 0.3, 0.05, 0.02), n_forbidden: int = 0,
                   alpha_time: float = 0.0) -> Problem:
    """Dense random Hermitian drift/controls for small property tests.
    ``n_forbidden`` > 0 adds that many Haar-random forbidden states (drawn
    after the targets and the weights); ``alpha_time`` weights the
    time-optimal term."""
    def herm():
        A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        return scale * (A + A.conj().T) / (2.0 * math.sqrt(d))
    H0 = herm()
    Hk = np.stack([herm() for _ in range(M)]) if M else np.zeros((0, d, d), np.complex128)
    u = rng.uniform(-u_scale, u_scale, size=(M, N))
    psi0 = np.stack([haar_state(rng, d) for _ in range(S)])
    psiT = np.stack([haar_state(rng, d) for _ in range(S)])
    w = rng.uniform(0.0, 1.0, size=d) if with_penalty else None
    forb = (np.stack([haar_state(rng, d) for _ in range(n_forbidden)])
            if n_forbidden > 0 else None)
    af, ap, aa, av = alphas
    return Problem(f"rand_d{d}_M{M}_N{N}_S{S}", d, M, N, S, dt, H0, Hk, u, psi0,
                   psiT, w=w, alpha_fid=af,
                   alpha_pen=ap if (with_penalty or n_forbidden > 0) else 0.0,
                   alpha_amp=aa, alpha_var=av, fid_mode=fid_mode, forbidden=forb,
                   alpha_time=float(alpha_time))


def sparse_problem(rng: np.random.Generator, d: int, M: int, N: int, S: int,
                   dt: float = 0.1, couplings: int = 2, u_scale: float = 0.5,
                   with_penalty: bool = True, fid_mode: str = "coherent",
                   alphas=(1.0, 0.3, 0.05, 0.02), n_forbidden: int = 0,
                   alpha_time: float = 0.0) -> Problem:
    """Random sparse Hermitian drift and controls: H_0 a random diagonal plus
    ``couplings`` random pairings of the basis states (one off-diagonal
    entry per row and pairing, Hermitian), each H_k one such pairing, so
    that a row of H_j holds at most 1 + couplings + M nonzeros."""
    def pairing():
        A = np.zeros((d, d), np.complex128)
        perm = rng.permutation(d)
        for i in range(0, d - 1, 2):
            a, b = perm[i], perm[i + 1]
            v = (rng.standard_normal() + 1j * rng.standard_normal()) / math.sqrt(2.0)
            A[a, b] = v
            A[b, a] = np.conj(v)
        return A
    H0 = np.diag(rng.standard_normal(d)).astype(np.complex128)
    for _ in range(couplings):
        H0 = H0 + pairing()
    Hk = np.stack([pairing() for _ in range(M)]) if M else np.zeros((0, d, d), np.complex128)
    u = rng.uniform(-u_scale, u_scale, size=(M, N))
    psi0 = np.stack([haar_state(rng, d) for _ in range(S)])
    psiT = np.stack([haar_state(rng, d) for _ in range(S)])
    w = rng.uniform(0.0, 1.0, size=d) if with_penalty else None
    forb = (np.stack([haar_state(rng, d) for _ in range(n_forbidden)])
            if n_forbidden > 0 else None)
    af, ap, aa, av = alphas
    return Problem(f"sparse_d{d}_M{M}_N{N}_S{S}", d, M, N, S, dt, H0, Hk, u, psi0,
                   psiT, w=w, alpha_fid=af,
                   alpha_pen=ap if (with_penalty or n_forbidden > 0) else 0.0,
                   alpha_amp=aa, alpha_var=av, fid_mode=fid_mode, forbidden=forb,
                   alpha_time=float(alpha_time))
