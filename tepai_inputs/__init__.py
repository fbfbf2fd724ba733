"""Seeded synthetic inputs for MPS TE-PAI runs.

This module only *describes problems*: Hamiltonian term lists, initial bit
strings, observables and run parameters.  It holds none of the method's
arithmetic (no rotation angles, no PAI coefficients, no sampling, no
simulation), so that both the CPU oracle and the GPU path can take their
inputs from it without sharing any of the computation.

Workloads follow the disordered spin ring of the paper's implementation
section (eq. "spinRing"): H = sum_k omega_k Z_k + J sigma_k . sigma_{k+1} on a
ring of n qubits, with the XXZ variant (J_xy, J_z) and the Neel initial state
used by the benchmark configurations.

Term order (the paper leaves the order of rotations inside one Trotter step
open): the single-site fields Z_0 .. Z_{n-1} first, then for every bond
b = 0 .. n-1 the pair (b, b+1 mod n) as XX, YY, ZZ.  Array order is time
order, so the wrap-around bond (n-1, 0) is the last one of every step.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

PAULI_CODE = {"I": 0, "X": 1, "Y": 2, "Z": 3}


@dataclass(frozen=True)
class Term:
    """One Pauli term c * P of H; ``paulis[i]`` acts on ``qubits[i]``."""

    paulis: str
    qubits: Tuple[int, ...]
    coeff: float


@dataclass(frozen=True)
class PauliString:
    """A weighted Pauli string coeff * prod_i P_i(q_i)."""

    paulis: str
    qubits: Tuple[int, ...]
    coeff: float = 1.0


# An observable is a sum of Pauli strings.
Observable = Tuple[PauliString, ...]


@dataclass(frozen=True)
class InitialMPS:
    """A shared starting state for every sample (hybrid start).

    ``tensors[k]`` is the complex site tensor at chain site k, shaped
    (chi_k, 2, chi_{k+1}) with chi_0 = chi_n = 1; ``qubit_at[k]`` is the qubit
    held at site k; sites left of ``centre`` are left-canonical, sites right
    of it right-canonical.
    """

    tensors: Tuple[np.ndarray, ...]
    centre: int
    qubit_at: Tuple[int, ...]

    def bonds(self) -> Tuple[int, ...]:
        return (1,) + tuple(int(a.shape[2]) for a in self.tensors)


@dataclass(frozen=True)
class Problem:
    """Everything that defines one TE-PAI estimation problem.

    ``trotter_steps`` is N, ``delta`` the PAI angle, ``chi_max`` the bond cap,
    ``svd_cutoff`` the relative singular-value floor below which Schmidt values
    count as zero, ``initial_bits[i]`` the computational-basis value of qubit i.
    """

    n_qubits: int
    terms: Tuple[Term, ...]
    total_time: float
    trotter_steps: int
    delta: float
    n_samples: int
    seed: int
    chi_max: int
    initial_bits: str
    observables: Tuple[Observable, ...]
    sample_offset: int = 0
    svd_cutoff: float = 1e-12
    chi_per_sample: Optional[Tuple[int, ...]] = None
    no_pi: bool = False         # biased variant without pi rotations
    trotter: bool = False       # deterministic product formula: every rotation exact
    per_gate: bool = False      # every sampled two-qubit gate its own truncated update
    initial_mps: Optional[InitialMPS] = None   # start every sample from this state
    name: str = ""

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def disorder(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Field strengths h_i ~ U[lo, hi] drawn from numpy's PCG64 at ``seed``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=n)


def spin_ring(n: int, fields: Sequence[float], j_xy: float = 1.0,
              j_z: Optional[float] = None, periodic: bool = True) -> Tuple[Term, ...]:
    """Terms of sum_i h_i Z_i + sum_b (J_xy (XX + YY) + J_z ZZ) in time order."""
    if j_z is None:
        j_z = j_xy
    terms: List[Term] = [Term("Z", (i,), float(fields[i])) for i in range(n)]
    n_bonds = n if periodic else n - 1
    for b in range(n_bonds):
        a, c = b, (b + 1) % n
        terms.append(Term("XX", (a, c), float(j_xy)))
        terms.append(Term("YY", (a, c), float(j_xy)))
        terms.append(Term("ZZ", (a, c), float(j_z)))
    return tuple(terms)


def neel(n: int) -> str:
    return "01" * (n // 2) + ("0" if n % 2 else "")


def z_all(n: int) -> Tuple[Observable, ...]:
    return tuple((PauliString("Z", (i,)),) for i in range(n))


def zz(a: int, b: int) -> Observable:
    return (PauliString("ZZ", (a, b)),)


def half_ring_zz(n: int) -> Observable:
    return tuple(PauliString("ZZ", (i, i + 1)) for i in range(n // 2))


def xyz_all(n: int) -> Tuple[Observable, ...]:
    """Every single-qubit Pauli observable: X_i, Y_i, Z_i for i = 0 .. n-1."""
    return tuple((PauliString(p, (i,)),) for i in range(n) for p in "XYZ")


def product_state(labels: str) -> InitialMPS:
    """A product state of X or Z eigenstates ('+', '-', '0', '1' per qubit) as
    a bond-1 MPS, centre on site 0, qubit k on site k."""
    r = 1.0 / np.sqrt(2.0)
    vec = {"0": (1.0, 0.0), "1": (0.0, 1.0), "+": (r, r), "-": (r, -r)}
    tensors = tuple(np.array(vec[c], dtype=np.complex128).reshape(1, 2, 1) for c in labels)
    return InitialMPS(tensors=tensors, centre=0, qubit_at=tuple(range(len(labels))))


def random_mps(n: int, chi: int, seed: int) -> InitialMPS:
    """A seeded random state with every bond at min(2^k, 2^(n-k), chi).

    Site tensors have i.i.d. complex Gaussian entries; sweeping from the last
    site to the first, each is replaced by the row-orthonormal factor of its
    (chi_k, 2 chi_{k+1}) matrix and the triangular rest is pushed into its
    left neighbour, so every site right of site 0 is right-canonical and the
    norm sits in site 0, which is scaled to 1.  Qubit k is on site k.
    """
    rng = np.random.default_rng(seed)
    bonds = [min(2 ** k, 2 ** (n - k), chi) for k in range(n + 1)]
    ts = [rng.standard_normal((bonds[k], 2, bonds[k + 1]))
          + 1j * rng.standard_normal((bonds[k], 2, bonds[k + 1])) for k in range(n)]
    for k in range(n - 1, 0, -1):
        q, r = np.linalg.qr(ts[k].reshape(bonds[k], -1).conj().T)
        ts[k] = q.conj().T.reshape(bonds[k], 2, bonds[k + 1])
        ts[k - 1] = np.tensordot(ts[k - 1], r.conj().T, axes=(2, 0))
    ts[0] = ts[0] / np.linalg.norm(ts[0])
    return InitialMPS(tensors=tuple(ts), centre=0, qubit_at=tuple(range(n)))


def plus_with_minus(n: int) -> str:
    """|+ ... + - + ... +> with the single '-' on qubit n // 2."""
    return "+" * (n // 2) + "-" + "+" * (n - n // 2 - 1)


def trotter_steps_for(T: float, n_ref: int = 20, dt_ref: float = 0.1) -> int:
    """N(T) = N_dT (T / dT)^2, the constant-accuracy step count of the
    first-order reference (eq. trotter-baseline-scaling, N_dT = 20, dT = 0.1)."""
    return int(round(n_ref * (T / dt_ref) ** 2))


# ---------------------------------------------------------------------------
# The benchmark configurations (disordered Heisenberg / XXZ rings).
# ---------------------------------------------------------------------------

def config(k: int, **overrides) -> Problem:
    """Configuration k = 1..5 of the benchmark set, seeded with k."""
    if k == 1:
        n = 8
        h = disorder(n, -1.0, 1.0, seed=1)
        p = Problem(n_qubits=n, terms=spin_ring(n, h), total_time=1.0,
                    trotter_steps=100, delta=np.pi / 64, n_samples=200, seed=1,
                    chi_max=16, initial_bits="01010101",
                    observables=((PauliString("Z", (0,)),),),
                    name="heisenberg_ring_n8_chi16")
    elif k == 2:
        n = 32
        h = disorder(n, -1.0, 1.0, seed=2)
        p = Problem(n_qubits=n, terms=spin_ring(n, h), total_time=2.0,
                    trotter_steps=400, delta=np.pi / 128, n_samples=10_000, seed=2,
                    chi_max=64, initial_bits=neel(n),
                    observables=z_all(n) + (zz(0, 16),),
                    name="heisenberg_ring_n32_chi64")
    elif k in (3, 4):
        n = 64
        h = disorder(n, -2.0, 2.0, seed=k)
        chi = 128
        ns = 100_000 if k == 3 else 20_000
        cps = tuple((32, 64, 128)[s % 3] for s in range(ns)) if k == 3 else None
        p = Problem(n_qubits=n, terms=spin_ring(n, h, j_xy=1.0, j_z=0.5),
                    total_time=3.0, trotter_steps=800, delta=np.pi / 256,
                    n_samples=ns, seed=k, chi_max=chi, chi_per_sample=cps,
                    initial_bits=neel(n), observables=z_all(n) + (zz(0, 32),),
                    name=f"xxz_ring_n64_chi128_cfg{k}")
    elif k == 5:
        n = 100
        h = disorder(n, -1.0, 1.0, seed=5)
        p = Problem(n_qubits=n, terms=spin_ring(n, h), total_time=2.0,
                    trotter_steps=1024, delta=np.pi / 512, n_samples=4096, seed=5,
                    chi_max=64, initial_bits=neel(n),
                    observables=z_all(n) + (half_ring_zz(n),),
                    name="heisenberg_ring_n100_tepai_segment")
    else:
        raise ValueError(f"no configuration {k}")
    return p.with_(**overrides) if overrides else p


def truncation_workload(chi: int, *, trotter: bool = False, n: int = 20, J: float = 1.0,
                        T: float = 1.0, n_samples: int = 100, seed: int = 7,
                        **overrides) -> Problem:
    """The truncation-robustness experiment (sec. "Truncation" and its figure):
    an n = 20 spin ring (eq. spinRing) with J = 1 and omega_k ~ U[-1, 1], evolved
    to T = 1 with Delta = pi / 2^12 and N_s = 100 TE-PAI circuits, or with the
    deterministic product formula (``trotter``), at bond cap ``chi``; the
    start is |+ ... + - + ... +> and the observables are X, Y and Z of every
    qubit.  N = N(T) of the first-order reference rule."""
    fields = disorder(n, -1.0, 1.0, seed=seed)
    p = Problem(n_qubits=n, terms=spin_ring(n, fields, j_xy=J, j_z=J), total_time=T,
                trotter_steps=trotter_steps_for(T), delta=np.pi / 2 ** 12,
                n_samples=1 if trotter else n_samples, seed=seed, chi_max=chi,
                initial_bits="0" * n, observables=xyz_all(n), trotter=trotter,
                initial_mps=product_state(plus_with_minus(n)),
                name=f"ring_n{n}_J{J:g}_T{T:g}_{'trotter' if trotter else 'tepai'}_chi{chi}")
    return p.with_(**overrides) if overrides else p


def small_ring(n: int, seed: int, *, T: float = 0.5, N: int = 20,
               delta: float = np.pi / 16, chi: int = 16, n_samples: int = 8,
               j_xy: float = 1.0, j_z: Optional[float] = None,
               h: float = 1.0, periodic: bool = True,
               observables: Optional[Tuple[Observable, ...]] = None) -> Problem:
    """A small disordered ring for parity tests (seeded, Neel start)."""
    fields = disorder(n, -h, h, seed=seed)
    obs = observables if observables is not None else z_all(n) + (zz(0, n // 2),)
    return Problem(n_qubits=n, terms=spin_ring(n, fields, j_xy, j_z, periodic),
                   total_time=T, trotter_steps=N, delta=delta,
                   n_samples=n_samples, seed=seed, chi_max=chi,
                   initial_bits=neel(n), observables=obs,
                   name=f"ring_n{n}_chi{chi}_seed{seed}")
