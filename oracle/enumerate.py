"""Exhaustive TE-PAI sum for tiny circuits (oracle side).

Statement 1 (unbiasedness): sum over every gate-setting multi-index l of
g_l * <O>_l equals the Trotter-circuit value, where g_l = prod of the
selected gamma_l(|theta|) (appendix "PAI & TE-PAI").  Feasible for
L_eff * N up to about 12 (3^12 settings).
"""
from __future__ import annotations

import itertools

import numpy as np

from .dense import apply_op, basis_state, expectation
from .schedule import setting_operator


def exhaustive_expectation(problem, table, observables):
    """sum_l g_l <O>_l for each observable in ``observables`` (a list)."""
    L = table.l_eff
    slots = [(j, k) for j in range(problem.trotter_steps) for k in range(L)]
    total = np.zeros(len(observables))
    for choice in itertools.product((0, 1, 2), repeat=len(slots)):
        g = 1.0
        psi = basis_state(problem.initial_bits)
        for (j, k), c in zip(slots, choice):
            row = table.rows[k]
            g *= row.gamma[c]
            if g == 0.0:
                break
            if c == 0:
                continue
            term = problem.terms[row.term]
            U = setting_operator(term.paulis, row.theta, problem.delta, c)
            psi = apply_op(psi, U, term.qubits)
        if g == 0.0:
            continue
        total += g * np.array([expectation(psi, o) for o in observables])
    return total
