"""MPS operation schedule of one sampled circuit (oracle side).

Turns a sampled TE-PAI circuit into the sequence of operations an MPS
simulator performs.  The paper fixes the MPS method only in outline (sec.
"Resource model and cost metrics": two-site gates on a mixed-canonical MPS,
SVD re-factorisation, truncation to the chi largest singular values at each
two-site update); the following readings fill in the rest and are shared by
every path that claims parity with this oracle:

1. Gates act in time order.  A single-qubit gate is applied exactly to its
   site tensor.
2. Consecutive sampled gates on the same qubit pair, with no other gate on
   either qubit in between and within one Trotter step, are multiplied into
   one 4x4 operator and applied as ONE two-site update (one truncated SVD).  A run made only of pi
   rotations (C = -i P (x) P) is a product of local unitaries and is applied
   to the two site tensors without an SVD.  With ``problem.per_gate`` every
   run holds a single gate: each sampled two-qubit gate is its own truncated
   update (a pi rotation its own pair of local Paulis).
3. A two-qubit operator whose qubits sit on non-adjacent sites lo < hi (on a
   ring kept as a chain these are the chain's two ends) is routed with SWAPs
   and the chain is left in its new order: the end qubit nearer the
   orthogonality centre (the one at hi when the centre is at or above the
   midpoint (lo + hi) / 2) is carried past every qubit in between, one
   truncated SWAP update at a time, and the last step is the single update
   SWAP . G on the pair, which applies the operator and completes the move.
   On a ring this rotates the chain by one site (hi - lo updates in all), so
   every ring bond but one stays adjacent, and the next Trotter step goes on
   from where the centre is.
4. The orthogonality centre sits inside the two sites of every two-site
   update.  Before an update at sites (i, i+1) the centre moves to the nearer
   of i and i+1 by single-site SVD shifts that drop singular values
   <= cutoff * sigma_0 and keep the rest (no cap, no renormalisation).  An
   update leaves the centre on its right site, except the SWAP updates that
   carry a qubit down, which leave it on their left site.
5. A two-site update keeps k = min(chi, #{sigma_i > cutoff * sigma_0})
   singular values and renormalises them to unit 2-norm.

Operations are expressed on sites:
    ("local",  site, U)              2x2 unitary on the physical index
    ("update", i, G, chi, right)     4x4 operator on sites (i, i+1), index
                                     s_i * 2 + s_{i+1}; right=True leaves the
                                     centre on i+1
    ("shift",  c, +1 | -1)           move the centre from site c to c +/- 1
    ("truncate", chi)                first op of a sample that starts from a
                                     shared state with a bond above its cap
                                     chi (``MPS.truncate_to``)
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np

from .sampler import SET_B, SET_C, SET_EXACT

PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}
SWAP4 = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex)


def pauli_matrix(paulis: str) -> np.ndarray:
    m = np.ones((1, 1), dtype=complex)
    for ch in paulis:
        m = np.kron(m, PAULI[ch])
    return m


def setting_operator(paulis: str, theta: float, delta: float, setting: int) -> np.ndarray:
    """Matrix of setting B = R(sign(theta) Delta) or C = R(pi) (eq. settings).

    R(phi) = exp(-i phi P / 2) = cos(phi/2) I - i sin(phi/2) P; at phi = pi this
    is exactly -i P, which is used as such.
    """
    P = pauli_matrix(paulis)
    if setting == SET_C:
        return -1j * P
    if setting == SET_EXACT:
        return math.cos(theta / 2.0) * np.eye(P.shape[0]) - 1j * math.sin(theta / 2.0) * P
    phi = math.copysign(delta, theta) if theta != 0.0 else delta
    return math.cos(phi / 2.0) * np.eye(P.shape[0]) - 1j * math.sin(phi / 2.0) * P


def flip_pair(G: np.ndarray) -> np.ndarray:
    """A 4x4 operator with its two tensor factors exchanged."""
    return SWAP4 @ G @ SWAP4


class _Pending:
    def __init__(self, qa: int, qb: int, layer: int):
        self.qa, self.qb = qa, qb
        self.layer = layer
        self.M = np.eye(4, dtype=complex)
        self.has_b = False
        self.La = np.eye(2, dtype=complex)
        self.Lb = np.eye(2, dtype=complex)
        self.phase = 1.0 + 0.0j

    def touches(self, q: int) -> bool:
        return q == self.qa or q == self.qb

    def same_pair(self, qa: int, qb: int) -> bool:
        return {qa, qb} == {self.qa, self.qb}


def build_schedule(problem, table, circuit, chi: Optional[int] = None) -> Tuple[List[tuple], List[int]]:
    """Operation list for ``circuit`` and the final qubit-at-site map."""
    n = problem.n_qubits
    chi = problem.chi_max if chi is None else chi
    L = table.l_eff
    init = getattr(problem, "initial_mps", None)
    qubit_at = list(init.qubit_at) if init is not None else list(range(n))
    site_of = [0] * n
    for k, q in enumerate(qubit_at):
        site_of[q] = k
    ops: List[tuple] = []
    centre = [init.centre if init is not None else 0]
    if init is not None and max(t.shape[2] for t in init.tensors) > chi:
        # a shared start with a bond above this sample's cap is truncated on
        # copy, which leaves the centre on the last site
        ops.append(("truncate", chi))
        centre[0] = n - 1

    def move_centre_to(i: int):
        # the centre must end on i or i + 1
        while centre[0] < i:
            ops.append(("shift", centre[0], +1))
            centre[0] += 1
        while centre[0] > i + 1:
            ops.append(("shift", centre[0], -1))
            centre[0] -= 1

    def update(i: int, G: np.ndarray, right: bool):
        move_centre_to(i)
        ops.append(("update", i, G, chi, right))
        centre[0] = i + 1 if right else i

    def swap_sites(i: int, right: bool):
        update(i, SWAP4, right)
        a, b = qubit_at[i], qubit_at[i + 1]
        qubit_at[i], qubit_at[i + 1] = b, a
        site_of[a], site_of[b] = i + 1, i

    def flush(p: Optional[_Pending]):
        if p is None:
            return
        if not p.has_b:
            ops.append(("local", site_of[p.qa], p.phase * p.La))
            ops.append(("local", site_of[p.qb], p.Lb))
            return
        ia, ib = site_of[p.qa], site_of[p.qb]
        lo, hi = min(ia, ib), max(ia, ib)
        if hi - lo == 1:
            update(lo, p.M if ia < ib else flip_pair(p.M), right=True)
            return
        if 2 * centre[0] >= lo + hi:             # carry the upper qubit down
            for s in range(hi - 1, lo, -1):      # ends next to the other qubit
                swap_sites(s, right=False)
            at = lo
        else:                                    # carry the lower qubit up
            for s in range(lo, hi - 1):
                swap_sites(s, right=True)
            at = hi - 1
        ia, ib = site_of[p.qa], site_of[p.qb]
        G = p.M if ia < ib else flip_pair(p.M)
        update(at, SWAP4 @ G, right=True)        # gate, then the last exchange
        a, b = qubit_at[at], qubit_at[at + 1]
        qubit_at[at], qubit_at[at + 1] = b, a
        site_of[a], site_of[b] = at + 1, at

    per_gate = bool(getattr(problem, "per_gate", False))
    pending: Optional[_Pending] = None
    for g, setting in zip(circuit.draws.tolist(), circuit.settings.tolist()):
        layer = g // L
        if pending is not None and pending.layer != layer:
            flush(pending)
            pending = None
        row = table.rows[g % L]
        term = problem.terms[row.term]
        U = setting_operator(term.paulis, row.theta, problem.delta, setting)
        if len(term.qubits) == 1:
            q = term.qubits[0]
            if pending is not None and pending.touches(q):
                flush(pending)
                pending = None
            ops.append(("local", site_of[q], U))
            continue
        qa, qb = term.qubits
        if pending is not None and not pending.same_pair(qa, qb):
            flush(pending)
            pending = None
        if pending is None:
            pending = _Pending(qa, qb, layer)
        if (qa, qb) != (pending.qa, pending.qb):
            U = flip_pair(U)
            pa, pb = term.paulis[1], term.paulis[0]
        else:
            pa, pb = term.paulis[0], term.paulis[1]
        pending.M = U @ pending.M
        if setting != SET_C:
            pending.has_b = True
        else:
            pending.La = PAULI[pa] @ pending.La
            pending.Lb = PAULI[pb] @ pending.Lb
            pending.phase *= -1j
        if per_gate:
            flush(pending)
            pending = None
    flush(pending)
    return ops, qubit_at
