"""TE-PAI circuit sampling (oracle side).

Protocol of the paper's sec. "TE-PAI" (steps 1-2) with the per-gate choice of
the appendix "PAI & TE-PAI": every rotation of the N-step Trotter circuit is
independently replaced by A = I, B = R(sign(theta) Delta) or C = R(pi) with
probabilities p_1, p_2, p_3.  The sample's sign is (-1)^(number of C
choices) (proof of Statement 2).

A sampled circuit is returned as the time-ordered list of its non-identity
gates, each encoded by its flat rotation index g = j * L_eff + k (Trotter step
j, table row k) and its setting (1 = B, 2 = C).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .philox import uniform_u64

SET_B = 1
SET_C = 2
SET_EXACT = 3     # not drawn: the exact rotation R(theta), for deterministic Trotter circuits


@dataclass(frozen=True)
class Circuit:
    sample: int
    draws: np.ndarray     # uint64 flat indices of non-identity gates, ascending
    settings: np.ndarray  # uint8, SET_B or SET_C
    sign: int             # +1 or -1

    @property
    def n_gates(self) -> int:
        return int(self.draws.size)


def choose(v63: np.ndarray, t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """Setting index 0 (A), 1 (B) or 2 (C) from the 63-bit uniform and thresholds."""
    out = np.full(v63.shape, 2, dtype=np.uint8)
    out[v63 < t2] = 1
    out[v63 < t1] = 0
    return out


def sample_circuit(problem, table, sample: int, layers=None) -> Circuit:
    """Sampled circuit of global sample index ``sample`` (first ``layers`` steps)."""
    L = table.l_eff
    J = problem.trotter_steps if layers is None else layers
    g = np.arange(J * L, dtype=np.uint64)
    u = uniform_u64(problem.seed, sample, g)
    v = u >> np.uint64(1)
    t1 = np.array([r.t1 for r in table.rows], dtype=np.uint64)
    t2 = np.array([r.t2 for r in table.rows], dtype=np.uint64)
    k = (g % np.uint64(L)).astype(np.int64)
    sel = choose(v, t1[k], t2[k])
    keep = sel != 0
    n_c = int(np.count_nonzero(sel == 2))
    return Circuit(sample=sample, draws=g[keep], settings=sel[keep],
                   sign=-1 if (n_c & 1) else 1)
