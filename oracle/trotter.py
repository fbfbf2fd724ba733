"""Deterministic Trotter evolution as an MPS (oracle side; test infrastructure).

The hybrid use of the method (sec. "Implementation", the Trotter-then-TE-PAI
experiment) starts every TE-PAI sample from a state that a deep Trotter
circuit prepared.  This module prepares such a state with the same MPS
machinery as the samples: every rotation of every step is applied exactly,
R_k(theta_k) (split rotations as their sub-rotations), through the same
schedule (pair fusion, wrap-bond routing, truncation at the bond cap).
The same circuit is the deterministic comparison of sec. "Truncation" (a
problem with ``trotter`` set runs it in place of sampled circuits).
"""
from __future__ import annotations

import numpy as np

import tepai_inputs as ti

from . import pai
from .mps import MPS
from .sampler import SET_EXACT, Circuit
from .schedule import build_schedule


def product_formula_circuit(table, steps: int, sample: int = 0) -> Circuit:
    """The first ``steps`` steps of the first-order product formula (eq.
    Trotter-Suzuki): every rotation of the table, in time order, exact."""
    draws = np.arange(steps * table.l_eff, dtype=np.uint64)
    return Circuit(sample=sample, draws=draws,
                   settings=np.full(draws.size, SET_EXACT, dtype=np.uint8), sign=1)


def trotter_initial_mps(problem, steps: int, chi: int) -> ti.InitialMPS:
    """State after ``steps`` Trotter steps of ``problem``'s H, as an InitialMPS."""
    table = pai.build_table(problem)
    circ = product_formula_circuit(table, steps)
    base = problem.with_(initial_mps=None)
    ops, qubit_at = build_schedule(base, table, circ, chi)
    m = MPS(base.initial_bits, problem.svd_cutoff).run(ops)
    return ti.InitialMPS(tensors=tuple(m.A), centre=m.centre, qubit_at=tuple(qubit_at))
