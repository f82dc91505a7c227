"""FP64 CPU oracle for the cost and exact gradient of piecewise-constant
quantum optimal control (Leung, Abdelhafez, Koch, Schuster, arXiv:1612.04929).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the only common inputs come from the seeded generators in
``workloads``.

The oracle computes the plain definition of what the method approximates:
the step propagator is the *exact* exponential of each Hermitian step
Hamiltonian (Sec. II, eq. (3); the text notes each short-time propagator can
be evaluated exactly by matrix exponentiation), obtained from LAPACK
``eigh``; the gradient is the exact adjoint with the exact Frechet
derivative of each step exponential (Daleckii-Krein formula).  The Taylor +
scaling-and-squaring approximant of Sec. III and its ``(p, n)`` selection
rule are provided separately so that tests can bound the approximation.

Every function's pins (closed forms, library routines, finite differences)
live in ``tests/test_oracle_*.py``.  Functions without an independent pin
say "parity unpinned" in their docstring; currently none.
"""
from .grape import (  # noqa: F401
    step_hamiltonians,
    step_norms,
    propagators,
    propagate,
    fidelity,
    step_penalties,
    time_fidelities,
    regularizers,
    cost,
    cost_grad,
    gradient_first_order,
    frechet_exp_skew,
    taylor_select,
    taylor_bound,
    taylor_squaring_expm,
    action_select,
    taylor_action,
    ps_products,
    taylor_select_ps,
)
