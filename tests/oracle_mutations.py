"""Planted mistakes in the FP64 oracle, one at a time, on the CPU.

Each entry replaces one fragment of ``oracle/grape.py`` (it must occur
exactly once) with a plausible slip: a wrong sign, index or operand, a
dropped term or factor, a transposed matrix, a wrong norm.  With
``QOC_ORACLE_MUTATION=<name>`` in the environment, ``tests/conftest.py``
loads the mutated source in place of ``oracle.grape`` before any test
module is collected; ``tests/test_oracle_mutations.py`` runs the oracle's
pins that way and requires each mutation to fail at least one of them.
"""
import os
import sys
import types

HERE = os.path.dirname(os.path.abspath(__file__))
GRAPE = os.path.join(os.path.dirname(HERE), "oracle", "grape.py")

MUTATIONS = {
    # Paterson-Stockmeyer count: the scalar top block multiplied anyway;
    # the batched rule on the Horner count
    "ps_top_block": ("        best = min(best, (s - 1) + q - (1 if rem == 0 else 0))\n",
                     "        best = min(best, (s - 1) + q)\n"),
    "ps_rule_horner": ("                cost = ps_products(p) + n\n", "                cost = p - 1 + n\n"),
    "ps_rule_ties": ("cost < best[0] or (cost == best[0] and p < best[1])", "cost < best[0]"),
    # action form: series term without its 1/k, (p, n) rule on matrix
    # products instead of matrix-vector products, no term-growth limit
    "action_term_factorial": ("            term = X @ term / k\n", "            term = X @ term\n"),
    "action_rule_products": ("                products = p * 2 ** n\n",
                             "                products = p - 1 + n\n"),
    "action_rule_growth": ("        if theta / 2.0 ** n > 1.0:\n            continue\n"
                           "        for p in range(2, p_max + 1):\n"
                           "            if taylor_bound(theta, p, n) <= tau:\n"
                           "                products = p * 2 ** n\n",
                           "        for p in range(2, p_max + 1):\n"
                           "            if taylor_bound(theta, p, n) <= tau:\n"
                           "                products = p * 2 ** n\n"),
    "ps_rule_growth": ("        if theta / 2.0 ** n > 1.0:\n            continue\n"
                       "        for p in range(2, p_max + 1):\n"
                       "            if taylor_bound(theta, p, n) <= tau:\n"
                       "                cost = ps_products(p) + n\n",
                       "        for p in range(2, p_max + 1):\n"
                       "            if taylor_bound(theta, p, n) <= tau:\n"
                       "                cost = ps_products(p) + n\n"),
    # exponential: sign of the phase, transposed propagator
    "expm_sign": ("phase = np.exp(-1j * prob.dt * lam)", "phase = np.exp(1j * prob.dt * lam)"),
    "expm_transpose": ("U = (V * phase[:, None, :]) @ np.conj(np.swapaxes(V, 1, 2))",
                       "U = np.swapaxes((V * phase[:, None, :]) @ np.conj(np.swapaxes(V, 1, 2)), 1, 2)"),
    # propagation with the transposed operand
    "propagate_transpose": ("psi[j + 1] = psi[j] @ U[j].T", "psi[j + 1] = psi[j] @ U[j]"),
    # fidelity: dropped 1/S, bilinear instead of sesquilinear overlap
    "fidelity_no_mean": ("z = ov.sum() / S", "z = ov.sum()"),
    "fidelity_no_conj": ("ov = np.array([np.vdot(psiT[s], psiN[s]) for s in range(S)])",
                         "ov = np.array([np.dot(psiT[s], psiN[s]) for s in range(S)])"),
    # penalty over j = 0..N-1 instead of 1..N
    "penalty_index": ('np.abs(psi[1:]) ** 2, w) / S', 'np.abs(psi[:-1]) ** 2, w) / S'),
    # regulariser: absolute instead of squared variation
    "variation_abs": ("c_var = float(np.sum(du * du))", "c_var = float(np.sum(np.abs(du)))"),
    # step norms: Frobenius instead of the 1-norm, dropped dt
    "norm_frobenius": ("return prob.dt * np.abs(H).sum(axis=1).max(axis=1)",
                       "return prob.dt * np.sqrt((np.abs(H) ** 2).sum(axis=(1, 2)))"),
    "norm_no_dt": ("return prob.dt * np.abs(H).sum(axis=1).max(axis=1)",
                   "return np.abs(H).sum(axis=1).max(axis=1)"),
    # (p, n) rule: bound without the 2^n amplification, ties to more squarings
    "bound_no_amplification": ("return 2.0 ** n * x ** (p + 1) / math.factorial(p + 1) * math.exp(x)",
                               "return x ** (p + 1) / math.factorial(p + 1) * math.exp(x)"),
    "select_ties": ("if best is None or G < best[0]:", "if best is None or G <= best[0]:"),
    # Frechet derivative: phase of the adjoint not conjugated, sinc argument
    "frechet_adjoint_phase": ("phase = np.exp(1j * half) if adjoint else np.exp(-1j * half)",
                              "phase = np.exp(-1j * half)"),
    "frechet_sinc": ("Phi = phase * np.sinc(x / np.pi)", "Phi = phase * np.sinc(x)"),
    # gradient: sign, costate through U_j instead of U_j^dagger, penalty source
    # from psi_{j+1} instead of psi_j (the penalty at j = 0 would be an
    # equivalent change: lambda_0 feeds no gradient)
    "grad_sign": ("g[k, j] = 2.0 * prob.dt * np.imag(np.vdot(W, prob.Hk[k]))",
                  "g[k, j] = -2.0 * prob.dt * np.imag(np.vdot(W, prob.Hk[k]))"),
    "costate_operand": ("lam = lam @ np.conj(U[j])               # rows: U_j^dagger lambda^s",
                        "lam = lam @ U[j]"),
    "costate_penalty_index": ("lam = lam @ np.conj(U[j])               # rows: U_j^dagger lambda^s\n        if j >= 1:\n            lam = lam + _step_source(prob, psi[j])",
                              "lam = lam @ np.conj(U[j])               # rows: U_j^dagger lambda^s\n        if j >= 1:\n            lam = lam + _step_source(prob, psi[j + 1])"),
    # final costate without the j = N step terms
    "costate_final_no_step_terms": ("return _fidelity_costate(prob, ov, z, prob.alpha_fid) + _step_source(prob, psiN)",
                                    "return _fidelity_costate(prob, ov, z, prob.alpha_fid)"),
    # forbidden states: bilinear overlap in the penalty, transposed source
    "forbidden_no_conj": ('ov = np.einsum("fm,jsm->jsf", np.conj(forbidden), psi[1:])',
                          'ov = np.einsum("fm,jsm->jsf", forbidden, psi[1:])'),
    "forbidden_source_conj": ("src = src + prob.alpha_pen / S * (ovf.T @ forb)",
                              "src = src + prob.alpha_pen / S * (ovf.T @ np.conj(forb))"),
    # time-optimal: steps 0..N-1 instead of 1..N, source without the 1/N
    "time_index": ("return np.array([fidelity(psi[j], psiT, mode)[2] for j in range(1, psi.shape[0])])",
                   "return np.array([fidelity(psi[j], psiT, mode)[2] for j in range(0, psi.shape[0] - 1)])"),
    "time_source_scale": ("src = src + _fidelity_costate(prob, ovt, zt, a_time / prob.N)",
                          "src = src + _fidelity_costate(prob, ovt, zt, a_time)"),
    "amp_grad_factor": ("g = 2.0 * prob.alpha_amp * u", "g = prob.alpha_amp * u"),
}


def mutated_source(name):
    src = open(GRAPE).read()
    old, new = MUTATIONS[name]
    count = src.count(old)
    if count != 1:
        raise RuntimeError(f"mutation {name!r}: fragment found {count} times in oracle/grape.py")
    return src.replace(old, new)


def install(name):
    """Replace oracle.grape (and the package's re-exports) by the mutated source."""
    import oracle
    mod = types.ModuleType("oracle.grape")
    mod.__file__ = GRAPE
    exec(compile(mutated_source(name), GRAPE, "exec"), mod.__dict__)
    sys.modules["oracle.grape"] = mod
    oracle.grape = mod
    for attr in dir(oracle):
        if not attr.startswith("_") and hasattr(mod, attr) and callable(getattr(oracle, attr)):
            setattr(oracle, attr, getattr(mod, attr))
