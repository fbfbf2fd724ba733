"""Dense state-vector references (oracle side, complex128, n <= ~14).

* ``circuit_state``    applies a sampled circuit gate by gate;
* ``trotter_state``    applies every rotation of the N-step product formula
                       (eq. Trotter-Suzuki / productFormula);
* ``exact_state``      exp(-iHT) |psi0> from an eigendecomposition of H;
* ``schedule_state``   replays an MPS operation list on the full state, doing
                       every truncation as a Schmidt cut of the whole vector
                       (the optimal rank-k approximation across that cut).

Qubit i is tensor axis i (axis 0 most significant); in ``schedule_state``
axis k is MPS site k instead.
"""
from __future__ import annotations

import math

import numpy as np

from .schedule import pauli_matrix, setting_operator
from .pai import theta_of


def basis_state(bits: str) -> np.ndarray:
    n = len(bits)
    psi = np.zeros((2,) * n, dtype=complex)
    psi[tuple(int(b) for b in bits)] = 1.0
    return psi


def apply_op(psi: np.ndarray, U: np.ndarray, axes) -> np.ndarray:
    """Apply a 2^m x 2^m matrix to the given tensor axes (in that order)."""
    m = len(axes)
    n = psi.ndim
    Ut = U.reshape((2,) * (2 * m))
    out = np.tensordot(Ut, psi, axes=(list(range(m, 2 * m)), list(axes)))
    # result axes: the m new ones first, then the untouched ones in order
    rest = [a for a in range(n) if a not in axes]
    order = list(axes) + rest
    inv = np.argsort(order)
    return np.transpose(out, inv)


def rotation(paulis: str, theta: float) -> np.ndarray:
    """R(theta) = exp(-i theta P / 2) for a Pauli string P."""
    P = pauli_matrix(paulis)
    return math.cos(theta / 2) * np.eye(P.shape[0]) - 1j * math.sin(theta / 2) * P


def circuit_state(problem, table, circuit) -> np.ndarray:
    psi = basis_state(problem.initial_bits)
    L = table.l_eff
    for g, s in zip(circuit.draws.tolist(), circuit.settings.tolist()):
        row = table.rows[g % L]
        term = problem.terms[row.term]
        U = setting_operator(term.paulis, row.theta, problem.delta, s)
        psi = apply_op(psi, U, term.qubits)
    return psi


def trotter_state(problem, layers=None) -> np.ndarray:
    """Every rotation R_k(theta_k) of the first ``layers`` Trotter steps."""
    psi = basis_state(problem.initial_bits)
    J = problem.trotter_steps if layers is None else layers
    ops = []
    for term in problem.terms:
        th = theta_of(term.coeff, problem.total_time, problem.trotter_steps)
        ops.append((rotation(term.paulis, th), term.qubits))
    for _ in range(J):
        for U, q in ops:
            psi = apply_op(psi, U, q)
    return psi


def hamiltonian(problem) -> np.ndarray:
    n = problem.n_qubits
    H = np.zeros((2 ** n, 2 ** n), dtype=complex)
    for term in problem.terms:
        full = ["I"] * n
        for p, q in zip(term.paulis, term.qubits):
            full[q] = p
        H += term.coeff * pauli_matrix("".join(full))
    return H


def exact_state(problem, t=None) -> np.ndarray:
    n = problem.n_qubits
    t = problem.total_time if t is None else t
    w, V = np.linalg.eigh(hamiltonian(problem))
    psi0 = basis_state(problem.initial_bits).reshape(-1)
    psi = V @ (np.exp(-1j * w * t) * (V.conj().T @ psi0))
    return psi.reshape((2,) * n)


def expectation(psi: np.ndarray, observable) -> float:
    """<psi|O|psi>/<psi|psi> for O = sum of weighted Pauli strings (qubit axes)."""
    nrm = np.vdot(psi, psi).real
    tot = 0.0
    for ps in observable:
        phi = psi
        for p, q in zip(ps.paulis, ps.qubits):
            phi = apply_op(phi, pauli_matrix(p), (q,))
        tot += ps.coeff * np.vdot(psi, phi).real
    return tot / nrm


def schmidt_cut(psi: np.ndarray, i: int, keep_max: int, cutoff: float,
                renormalise: bool) -> np.ndarray:
    """Best approximation of psi with at most k Schmidt values across (i | i+1)."""
    n = psi.ndim
    M = psi.reshape(2 ** (i + 1), 2 ** (n - i - 1))
    U, S, Vh = np.linalg.svd(M, full_matrices=False)
    r = int(np.count_nonzero(S > cutoff * S[0])) if S[0] > 0 else 0
    k = max(min(keep_max, r), 1)
    Sk = S[:k]
    if renormalise:
        Sk = Sk / np.linalg.norm(Sk)
    return ((U[:, :k] * Sk[None, :]) @ Vh[:k]).reshape(psi.shape)


def schedule_state(problem, ops) -> np.ndarray:
    """Replay an MPS operation list on the dense state (site axes)."""
    psi = basis_state(problem.initial_bits)
    cut = problem.svd_cutoff
    for op in ops:
        if op[0] == "local":
            psi = apply_op(psi, op[2], (op[1],))
        elif op[0] == "update":
            i, G, chi = op[1], op[2], op[3]
            psi = apply_op(psi, G, (i, i + 1))
            psi = schmidt_cut(psi, i, chi, cut, renormalise=True)
        elif op[0] == "shift":
            c, d = op[1], op[2]
            bond = c if d > 0 else c - 1
            psi = schmidt_cut(psi, bond, 1 << 30, cut, renormalise=False)
        else:
            # ("truncate", chi) only opens the schedule of a shared start,
            # which this replay (from a basis state) does not take
            raise ValueError(f"dense replay has no operation {op[0]!r}")
    return psi


def site_to_qubit_order(psi_sites: np.ndarray, qubit_at) -> np.ndarray:
    """Reorder site axes into qubit axes given qubit_at[site]."""
    order = np.argsort(np.asarray(qubit_at))
    return np.transpose(psi_sites, order)
