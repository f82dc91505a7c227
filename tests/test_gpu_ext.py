"""GPU parity of the per-step terms beyond the level penalty (Table I):
general forbidden states in C5 (a set of forbidden states summed, Sec.
II.A) and the time-optimal term C6 / C7 (the fidelity penalised at every
time step), against the FP64 oracle: cost, every c_j, psi_N and the
gradient, at the FP32 targets (FP64 chains: tight), on ragged shapes and
the paths of every padded d."""
import numpy as np
import pytest

import workloads
from test_gpu_parity import check, compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,S,N,nf,at,mode,pen,L", [
    (5, 2, 37, 2, 0.0, "coherent", True, 0),       # padded d 16, level weights and states
    (16, 4, 203, 3, 0.5, "coherent", False, 16),   # C6 (coherent) with forbidden states
    (12, 2, 131, 0, 0.8, "incoherent", False, 32), # C7 (incoherent) alone, ragged blocks
    (20, 3, 60, 1, 0.3, "incoherent", True, 8),    # padded d 32
    (40, 2, 45, 2, 0.3, "coherent", True, 0),      # padded d 48
    (64, 2, 70, 4, 0.4, "coherent", True, 0),      # 64-tiled chains
    (100, 3, 25, 2, 0.2, "incoherent", False, 4),  # padded d 112, batched derivative
    (3, 2, 1, 1, 1.0, "coherent", True, 0),        # a single step
])
def test_forbidden_states_and_time_optimal(d, S, N, nf, at, mode, pen, L):
    rng = np.random.default_rng(700 + d + N)
    p = workloads.random_problem(rng, d=d, M=3, N=N, S=S, dt=0.2, scale=1.5, fid_mode=mode,
                                 with_penalty=pen, n_forbidden=nf, alpha_time=at)
    out, ref, e = compare(f"ext_d{d}_S{S}_N{N}_nf{nf}_t{at}", p, checkpoint_every=L)
    check(p, e)


def test_time_optimal_full_basis_gate_fp64():
    # C6 on a full basis (S = d, identity columns): FP64 chains, tight
    rng = np.random.default_rng(710)
    p = workloads.random_problem(rng, d=6, M=2, N=40, S=6, dt=0.2, scale=1.5,
                                 with_penalty=False, alpha_time=0.7, n_forbidden=2)
    p.psi0 = np.eye(6, dtype=complex)
    out, ref, e = compare("ext_gate_fp64", p, precision="fp64")
    check(p, e, precision="fp64")


def test_transmon_cavity_forbidden_superpositions():
    """The transmon-cavity workload (reduced N) with forbidden cavity
    superpositions (cat-like states near the truncation edge) and the
    time-optimal term."""
    p = workloads.config3().with_steps(300)
    d = p.d
    F = np.zeros((2, d), complex)
    F[0, 28] = F[0, 30] = 1 / np.sqrt(2)          # |g,28> + |g,30>
    F[1, 32 + 29] = 1 / np.sqrt(2)
    F[1, 31] = 1j / np.sqrt(2)                     # |e,29> + i |g,31>
    p.forbidden = F
    p.alpha_time = 0.2
    out, ref, e = compare("ext_c3_N300", p, checkpoint_every=16)
    check(p, e)
