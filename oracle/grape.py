"""Plain FP64 reference for the GRAPE-style cost and its exact gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written for clarity,
not speed: every step follows the definition it cites, with no blocking,
fusion or reordering beyond it.

Notation (paper Sec. II and Table I):
  H_j = H_0 + sum_k u[k, j] H_k                       eq. (1)
  U_j = exp(-i H_j dt)                                 eq. (3)
  psi_{j+1} = U_j psi_j, psi_0 given, j = 0..N-1       eqs. (2), (4)
  z   = (1/S) sum_s <T_s | psi_N^s>                    composite C2-sigma (Sec. II.A)
  C_fid = 1 - |z|^2                                    (coherent; equals C1 of Table I
                                                        for S = d, psi_0 = identity)
  c_j = (1/S) sum_s [sum_m w_m |psi_j^s[m]|^2          Table I, C5: forbidden basis levels
                     + sum_f |<F_f|psi_j^s>|^2], j=1..N  (weights w) and forbidden states F_f
  C_amp = sum_{k,j} u_{k,j}^2                          Table I, C3
  C_var = sum_k sum_{j=1}^{N-1} (u_{k,j}-u_{k,j-1})^2  Table I, C4
  C_time = 1 - (1/N) sum_{j=1}^N F_j                   Table I, C6 (coherent, gate) / C7
                                                        (incoherent, states); F_j the
                                                        fidelity of psi_j against the targets
  C = a_fid C_fid + a_pen sum_j c_j + a_amp C_amp + a_var C_var + a_time C_time
                                                       Sec. II (weighted sum)

States are stored as rows: ``psi[j, s]`` is the length-d vector psi_j^s.

Readings where the paper is silent or ambiguous (each listed in the design
notes): N steps j = 0..N-1 with psi_0 the initial state; the 1/S
normalisation sits inside |.|^2; the projector P_S is implicit (targets
vanish outside the subspace); C5 sums j = 1..N over a diagonal weight
vector and a set of forbidden states (summed, Sec. II.A) with a 1/S mean
over columns; C6/C7 average the fidelity of the same mode as C_fid over
j = 1..N; C4 runs over j = 1..N-1; hbar = 1.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np


# --------------------------------------------------------------------- a1
def step_hamiltonians(prob, u: Optional[np.ndarray] = None) -> np.ndarray:
    """H_j = H_0 + sum_k u_{k,j} H_k for j = 0..N-1 (eq. (1)).  Shape (N, d, d)."""
    u = prob.u if u is None else u
    H = np.broadcast_to(prob.H0, (prob.N, prob.d, prob.d)).copy()
    for k in range(prob.M):
        H += u[k][:, None, None] * prob.Hk[k][None, :, :]
    return H


# --------------------------------------------------------------------- a2
def step_norms(prob, u: Optional[np.ndarray] = None) -> np.ndarray:
    """theta_j = || dt H_j ||_1 (maximum column absolute sum), shape (N,).

    The paper fixes one global truncation order p and squaring count n from
    a conservative look at the step generators (Sec. III); this is the
    quantity the selection rule :func:`taylor_select` is applied to.
    """
    H = step_hamiltonians(prob, u)
    return prob.dt * np.abs(H).sum(axis=1).max(axis=1)


def taylor_bound(theta: float, p: int, n: int) -> float:
    """Upper bound on || T_p(A/2^n)^(2^n) - exp(A) || for ||A|| <= theta.

    Truncated Taylor series of order p (Sec. III, eq. (6)) applied to
    A / 2^n: the remainder is at most x^(p+1)/(p+1)! e^x with x = theta/2^n;
    n squarings of a near-unitary factor amplify it at most 2^n-fold.
    """
    x = theta / 2.0 ** n
    return 2.0 ** n * x ** (p + 1) / math.factorial(p + 1) * math.exp(x)


def taylor_select(theta: float, tau: float = 1e-10, p_max: int = 30,
                  n_max: int = 60) -> tuple:
    """Global (p, n) for scaling and squaring (Sec. III, text after eq. (6)).

    The paper gives no rule for its "conservative" global choice; this
    reading picks the pair with the fewest matrix products
    G = (p - 1) + n subject to ``taylor_bound(theta, p, n) <= tau``,
    breaking ties toward fewer squarings, with p >= 2.
    """
    best = None
    for n in range(n_max):
        for p in range(2, p_max + 1):
            if taylor_bound(theta, p, n) <= tau:
                G = p - 1 + n
                if best is None or G < best[0]:
                    best = (G, p, n)
                break
    if best is None:
        raise ValueError(f"no (p, n) meets tau={tau} for theta={theta}")
    return best[1], best[2]


def ps_products(p: int) -> int:
    """Matrix products that evaluate T_p(X) (p >= 1) in Paterson-Stockmeyer
    form, or by Horner's rule when that takes fewer: the powers X^2 .. X^s
    (s - 1 products, 2 <= s <= min(p, 4)), then Horner's rule in Y = X^s
    over the floor(p/s) + 1 blocks of s coefficients (one product per block
    below the top one, which is a scalar multiple of the identity when s
    divides p, so that its product falls away)."""
    best = p - 1  # Horner's rule
    for s in range(2, min(p, 4) + 1):
        q, rem = divmod(p, s)
        best = min(best, (s - 1) + q - (1 if rem == 0 else 0))
    return best


def taylor_select_ps(theta: float, tau: float = 1e-10, p_max: int = 30,
                     n_max: int = 60) -> tuple:
    """Global (p, n) for steps evaluated as batched matrix products with
    Paterson-Stockmeyer Taylor polynomials (Sec. III, the conservative
    global choice).  Reading: the pair with the fewest evaluated products
    ps_products(p) + n subject to ``taylor_bound(theta, p, n) <= tau`` and
    theta / 2^n <= 1 (the series terms do not grow), ties toward the lower
    order p (the exact derivative runs p - 1 reverse Horner stages), p >= 2."""
    best = None
    for n in range(n_max):
        if theta / 2.0 ** n > 1.0:
            continue
        for p in range(2, p_max + 1):
            if taylor_bound(theta, p, n) <= tau:
                cost = ps_products(p) + n
                if best is None or cost < best[0] or (cost == best[0] and p < best[1]):
                    best = (cost, p, n)
                break
    if best is None:
        raise ValueError(f"no (p, n) meets tau={tau} for theta={theta}")
    return best[1], best[2]


def taylor_squaring_expm(A: np.ndarray, p: int, n: int) -> np.ndarray:
    """[sum_{k=0}^p (A/2^n)^k / k!]^(2^n)  (Sec. III, eq. (6)), in FP64."""
    X = A / 2.0 ** n
    term = np.eye(A.shape[0], dtype=np.complex128)
    T = term.copy()
    for k in range(1, p + 1):
        term = term @ X / k
        T = T + term
    for _ in range(n):
        T = T @ T
    return T


# --------------------------------------------------------------------- f2
def action_select(theta: float, tau: float = 1e-10, p_max: int = 30,
                  n_max: int = 60) -> tuple:
    """Global (p, n) for the state-mode action form (Sec. IV: U_j|psi> as a
    series of matrix-vector products, no U_j formed).

    The approximant is the one of Sec. III, T_p(A/2^n)^(2^n), applied to the
    columns, which costs p 2^n matrix-vector products per step.  Reading
    (the paper gives no rule for this form): the pair with the fewest
    products p 2^n subject to ``taylor_bound(theta, p, n) <= tau`` and
    theta / 2^n <= 1 (the series terms do not grow, so no large terms
    cancel), ties toward fewer squarings, p >= 2.
    """
    best = None
    for n in range(n_max):
        if theta / 2.0 ** n > 1.0:
            continue
        for p in range(2, p_max + 1):
            if taylor_bound(theta, p, n) <= tau:
                products = p * 2 ** n
                if best is None or products < best[0]:
                    best = (products, p, n)
                break
    if best is None:
        raise ValueError(f"no (p, n) meets tau={tau} for theta={theta}")
    return best[1], best[2]


def taylor_action(A: np.ndarray, psi: np.ndarray, p: int, n: int) -> np.ndarray:
    """T_p(A/2^n)^(2^n) applied to the states (rows of psi) without forming
    the matrix: 2^n times the truncated series sum_{k=0}^p (A/2^n)^k v / k!,
    its terms by repeated matrix-vector products (Sec. IV, the series for
    U_j|Psi>), in FP64."""
    X = A / 2.0 ** n
    v = psi.T.astype(np.complex128)  # columns
    for _ in range(2 ** n):
        term = v
        acc = v.copy()
        for k in range(1, p + 1):
            term = X @ term / k
            acc = acc + term
        v = acc
    return v.T


# --------------------------------------------------------------------- a3/a4
def propagators(prob, u: Optional[np.ndarray] = None):
    """Exact step propagators U_j = exp(-i H_j dt) (eq. (3)).

    H_j is Hermitian, so H_j = V diag(lam) V^dagger (LAPACK eigh) and
    U_j = V diag(exp(-i dt lam)) V^dagger exactly.
    Returns (U, lam, V) with shapes (N,d,d), (N,d), (N,d,d).
    """
    H = step_hamiltonians(prob, u)
    lam, V = np.linalg.eigh(H)
    phase = np.exp(-1j * prob.dt * lam)
    U = (V * phase[:, None, :]) @ np.conj(np.swapaxes(V, 1, 2))
    return U, lam, V


# --------------------------------------------------------------------- a5
def propagate(U: np.ndarray, psi0: np.ndarray) -> np.ndarray:
    """psi_{j+1}^s = U_j psi_j^s for j = 0..N-1 (eqs. (2), (4)).

    Returns psi with shape (N+1, S, d); psi[0] = psi0.
    """
    N = U.shape[0]
    psi = np.empty((N + 1,) + psi0.shape, dtype=np.complex128)
    psi[0] = psi0
    for j in range(N):
        psi[j + 1] = psi[j] @ U[j].T
    return psi


# --------------------------------------------------------------------- a7
def fidelity(psiN: np.ndarray, psiT: np.ndarray, mode: str = "coherent"):
    """Fidelity of the final states against the targets (Sec. II.A, Table I).

    coherent:   z = (1/S) sum_s <T_s|psi_N^s>, F = |z|^2 (composite C2-sigma)
    incoherent: o_s = <T_s|psi_N^s>, F = (1/S) sum_s |o_s|^2 (mean of C2)
    Returns (overlaps o_s, z, F); C_fid = 1 - F.
    """
    S = psiN.shape[0]
    ov = np.array([np.vdot(psiT[s], psiN[s]) for s in range(S)])
    z = ov.sum() / S
    if mode == "coherent":
        F = abs(z) ** 2
    elif mode == "incoherent":
        F = float(np.sum(np.abs(ov) ** 2) / S)
    else:
        raise ValueError(mode)
    return ov, z, float(F)


# --------------------------------------------------------------------- a6
def step_penalties(psi: np.ndarray, w: Optional[np.ndarray],
                   forbidden: Optional[np.ndarray] = None) -> np.ndarray:
    """c_j = (1/S) sum_s [sum_m w_m |psi_j^s[m]|^2 + sum_f |<F_f|psi_j^s>|^2]
    for j = 1..N (Table I, C5).

    Forbidden basis levels carry weights w; general forbidden states F_f
    (rows of ``forbidden``) enter "upon summation" (Sec. II.A).  Returns
    shape (N,).
    """
    N = psi.shape[0] - 1
    S = psi.shape[1]
    c = np.zeros(N)
    if w is not None:
        c = c + np.einsum("jsm,m->j", np.abs(psi[1:]) ** 2, w) / S
    if forbidden is not None:
        ov = np.einsum("fm,jsm->jsf", np.conj(forbidden), psi[1:])
        c = c + np.sum(np.abs(ov) ** 2, axis=(1, 2)) / S
    return c


# --------------------------------------------------------------------- C6/C7
def time_fidelities(psi: np.ndarray, psiT: np.ndarray, mode: str = "coherent") -> np.ndarray:
    """F_j, j = 1..N: the fidelity of psi_j against the targets, in the mode
    of the final fidelity (coherent: Table I, C6, for a target gate on a
    basis; incoherent: C7, for target states).  C_time = 1 - mean_j F_j
    rewards reaching the target early ("at every time step", Sec. II.A).
    Returns shape (N,)."""
    return np.array([fidelity(psi[j], psiT, mode)[2] for j in range(1, psi.shape[0])])


# --------------------------------------------------------------------- C3/C4
def regularizers(u: np.ndarray):
    """C_amp = |u|^2 (Table I, C3); C_var = sum |u_{k,j} - u_{k,j-1}|^2, j>=1 (C4)."""
    c_amp = float(np.sum(u * u))
    du = np.diff(u, axis=1)
    c_var = float(np.sum(du * du))
    return c_amp, c_var


def _forward(prob, u):
    U, lam, V = propagators(prob, u)
    psi = propagate(U, prob.psi0)
    ov, z, F = fidelity(psi[-1], prob.psiT, prob.fid_mode)
    c = step_penalties(psi, prob.w, getattr(prob, "forbidden", None))
    c_amp, c_var = regularizers(u)
    C_fid = 1.0 - F
    C_time = 1.0 - float(np.mean(time_fidelities(psi, prob.psiT, prob.fid_mode)))
    C = (prob.alpha_fid * C_fid + prob.alpha_pen * float(c.sum())
         + prob.alpha_amp * c_amp + prob.alpha_var * c_var
         + getattr(prob, "alpha_time", 0.0) * C_time)
    eye = np.eye(prob.d)
    drift = float(np.max(np.abs(np.conj(np.swapaxes(U, 1, 2)) @ U - eye)))
    out = dict(C=C, C_fid=C_fid, F=F, z=z, overlaps=ov, c=c, C_pen=float(c.sum()),
               C_amp=c_amp, C_var=c_var, C_time=C_time, psiN=psi[-1].copy(),
               unitarity_drift=drift,
               theta_max=float(step_norms(prob, u).max()))
    return out, U, lam, V, psi


def cost(prob, u: Optional[np.ndarray] = None) -> dict:
    """All cost terms for controls u (defaults to ``prob.u``)."""
    u = prob.u if u is None else np.asarray(u, dtype=np.float64)
    return _forward(prob, u)[0]


# --------------------------------------------------------------------- a10
def frechet_exp_skew(lam: np.ndarray, V: np.ndarray, dt: float, E: np.ndarray,
                     adjoint: bool = False) -> np.ndarray:
    """Frechet derivative of exp at A = -i dt H (or at A^dagger = +i dt H).

    With H = V diag(lam) V^dagger, the Daleckii-Krein formula gives
    L(A, E) = V [ (V^dagger E V) o Phi ] V^dagger with divided differences
    Phi_ab = (e^{mu_a} - e^{mu_b}) / (mu_a - mu_b), mu = -i dt lam, which for
    a skew-Hermitian A equal e^{-i dt (lam_a+lam_b)/2} sinc(dt (lam_a-lam_b)/2)
    (continuous at equal eigenvalues).  ``adjoint=True`` evaluates at
    A^dagger, which conjugates the phase.
    """
    half = 0.5 * dt * (lam[:, None] + lam[None, :])
    x = 0.5 * dt * (lam[:, None] - lam[None, :])
    phase = np.exp(1j * half) if adjoint else np.exp(-1j * half)
    Phi = phase * np.sinc(x / np.pi)
    Vh = np.conj(V.T)
    return V @ ((Vh @ E @ V) * Phi) @ Vh


# --------------------------------------------------------------------- a8-a11
def _fidelity_costate(prob, ov, z, weight):
    """d(weight (1 - F))/d(psi^*) at a state set with overlaps ov and z."""
    S = prob.S
    if prob.fid_mode == "coherent":
        return -weight * (z / S) * prob.psiT
    return -weight * (ov[:, None] / S) * prob.psiT


def _step_source(prob, psi_j):
    """dC/d(psi_j^*) of the per-step terms at one step j >= 1: the C5
    penalties (weighted levels and forbidden states) and the time-optimal
    term a_time (1 - F_j) / N."""
    S = prob.S
    src = np.zeros_like(psi_j)
    if prob.alpha_pen != 0.0:
        if prob.w is not None:
            src = src + prob.alpha_pen / S * prob.w[None, :] * psi_j
        forb = getattr(prob, "forbidden", None)
        if forb is not None:
            ovf = np.conj(forb) @ psi_j.T               # (F, S): <F_f|psi_j^s>
            src = src + prob.alpha_pen / S * (ovf.T @ forb)
    a_time = getattr(prob, "alpha_time", 0.0)
    if a_time != 0.0:
        ovt, zt, _ = fidelity(psi_j, prob.psiT, prob.fid_mode)
        src = src + _fidelity_costate(prob, ovt, zt, a_time / prob.N)
    return src


def _costate_final(prob, psiN, ov, z):
    """lambda_N = dC/d(psi_N^*): the final fidelity and the j = N step terms."""
    return _fidelity_costate(prob, ov, z, prob.alpha_fid) + _step_source(prob, psiN)


def _regularizer_grad(prob, u):
    g = 2.0 * prob.alpha_amp * u
    if prob.alpha_var != 0.0 and u.shape[1] > 1:
        du = np.diff(u, axis=1)                 # du[:, j-1] = u_j - u_{j-1}
        gv = np.zeros_like(u)
        gv[:, 1:] += 2.0 * du
        gv[:, :-1] -= 2.0 * du
        g = g + prob.alpha_var * gv
    return g


def cost_grad(prob, u: Optional[np.ndarray] = None) -> dict:
    """Cost terms and the exact gradient dC/du_{k,j}.

    Adjoint form (reverse accumulation, Sec. II.B), with costates
    lambda_j = dC/d(psi_j^*) so that dC = 2 Re <lambda, d psi>:
      lambda_N from the fidelity and the j = N penalty;
      for j = N-1..0:
        G_j   = sum_s lambda_{j+1}^s (psi_j^s)^dagger   (cotangent of U_j)
        W_j   = L(A_j^dagger, G_j)                      exact Frechet adjoint
        g_kj  = 2 Re tr(W_j^dagger dA_j/du_kj) = 2 dt Im tr(W_j^dagger H_k)
        lambda_j = U_j^dagger lambda_{j+1} + s_j(psi_j)   (per-step terms for j >= 1:
                   a_pen/S [w o psi_j + sum_f <F_f|psi_j> F_f] and the time-optimal
                   -a_time/N dF_j/d(psi_j^*))
    plus the closed-form gradients of C3 and C4.  The adjoint identity
    tr(G^dagger L(A,E)) = tr(L(A^dagger,G)^dagger E) lets one Frechet
    evaluation per step serve every control.
    """
    u = prob.u if u is None else np.asarray(u, dtype=np.float64)
    out, U, lamH, V, psi = _forward(prob, u)
    N, S = prob.N, prob.S
    g = np.zeros((prob.M, N))
    lam = _costate_final(prob, psi[N], out["overlaps"], out["z"])
    for j in range(N - 1, -1, -1):
        G = lam.T @ np.conj(psi[j])             # sum_s lam^s (psi_j^s)^dagger
        W = frechet_exp_skew(lamH[j], V[j], prob.dt, G, adjoint=True)
        for k in range(prob.M):
            g[k, j] = 2.0 * prob.dt * np.imag(np.vdot(W, prob.Hk[k]))
        lam = lam @ np.conj(U[j])               # rows: U_j^dagger lambda^s
        if j >= 1:
            lam = lam + _step_source(prob, psi[j])
    out["grad"] = g + _regularizer_grad(prob, u)
    return out


def gradient_first_order(prob, u: Optional[np.ndarray] = None) -> np.ndarray:
    """The paper's approximate gradient (eq. (7), App. A, Algorithms 1-3).

    Replaces dU_j/du_kj by (-i dt H_k) U_j, i.e. drops the non-commuting
    corrections, giving g_kj ~ 2 dt Im sum_s <lambda_{j+1}^s|H_k|psi_{j+1}^s>.
    Exact when all H_j commute; a comparison mode only.
    """
    u = prob.u if u is None else np.asarray(u, dtype=np.float64)
    out, U, lamH, V, psi = _forward(prob, u)
    N, S = prob.N, prob.S
    g = np.zeros((prob.M, N))
    lam = _costate_final(prob, psi[N], out["overlaps"], out["z"])
    for j in range(N - 1, -1, -1):
        for k in range(prob.M):
            Hpsi = psi[j + 1] @ prob.Hk[k].T
            g[k, j] = 2.0 * prob.dt * np.imag(np.sum(np.conj(lam) * Hpsi))
        lam = lam @ np.conj(U[j])
        if j >= 1:
            lam = lam + _step_source(prob, psi[j])
    return g + _regularizer_grad(prob, u)
