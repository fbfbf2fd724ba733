"""Deterministic Trotter evolution as an MPS (oracle side; test infrastructure).

The hybrid use of the method (sec. "Implementation", the Trotter-then-TE-PAI
experiment) starts every TE-PAI sample from a state that a deep Trotter
circuit prepared.  This module prepares such a state with the same MPS
machinery as the samples: every rotation of every step is applied exactly,
R_k(theta_k) (split rotations as their sub-rotations), through the same
schedule (pair fusion, wrap-bond routing, truncation at the bond cap).
"""
from __future__ import annotations

import numpy as np

import tepai_inputs as ti

from . import pai
from .mps import MPS
from .sampler import SET_EXACT, Circuit
from .schedule import build_schedule


def trotter_initial_mps(problem, steps: int, chi: int) -> ti.InitialMPS:
    """State after ``steps`` Trotter steps of ``problem``'s H, as an InitialMPS."""
    table = pai.build_table(problem)
    L = table.l_eff
    draws = np.arange(steps * L, dtype=np.uint64)
    circ = Circuit(sample=0, draws=draws, settings=np.full(draws.size, SET_EXACT, dtype=np.uint8),
                   sign=1)
    base = problem.with_(initial_mps=None)
    ops, qubit_at = build_schedule(base, table, circ, chi)
    m = MPS(base.initial_bits, problem.svd_cutoff).run(ops)
    return ti.InitialMPS(tensors=tuple(m.A), centre=m.centre, qubit_at=tuple(qubit_at))
