"""The whole TE-PAI estimator on the CPU (oracle side).

For each sample: sample the circuit, build its MPS schedule, run the MPS,
read out <O> for every observable; then weight and reduce (protocol steps
1-3 of the paper's sec. "TE-PAI"; estimator of Statement 2).  A problem with
``trotter`` set runs the deterministic product formula instead, every sample
the same circuit with weight 1.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import pai
from .estimator import estimate, weights
from .mps import MPS, Stats
from .sampler import sample_circuit
from .schedule import PAULI, build_schedule
from .trotter import product_formula_circuit


@dataclass
class SampleResult:
    sample: int
    sign: int
    n_gates: int
    values: np.ndarray
    stats: Stats
    bonds: List[int]


@dataclass
class RunResult:
    samples: List[SampleResult]
    log_g1: float
    weights: np.ndarray
    values: np.ndarray
    mean: np.ndarray
    std_err: np.ndarray
    config_var: np.ndarray


def chi_of(problem, s: int) -> int:
    if problem.chi_per_sample is not None:
        return int(problem.chi_per_sample[s])
    return problem.chi_max


def observable_value(mps: MPS, qubit_at, observable) -> float:
    site_of = {q: k for k, q in enumerate(qubit_at)}
    tot = 0.0
    for ps in observable:
        ops = [None] * mps.n
        for p, q in zip(ps.paulis, ps.qubits):
            k = site_of[q]
            ops[k] = PAULI[p] if ops[k] is None else PAULI[p] @ ops[k]
        tot += ps.coeff * mps.expectation(ops).real
    return tot


def run_sample(problem, table, s: int, layers: Optional[int] = None,
               perturb=None) -> SampleResult:
    """One sample; ``perturb = (seed, scale)`` perturbs every factorisation at
    the level of an SVD backward error (see ``mps.MPS``)."""
    if getattr(problem, "trotter", False):
        steps = problem.trotter_steps if layers is None else layers
        circ = product_formula_circuit(table, steps, s)
    else:
        circ = sample_circuit(problem, table, s, layers)
    ops, qubit_at = build_schedule(problem, table, circ, chi_of(problem, s))
    init = getattr(problem, "initial_mps", None)
    mps = (MPS.from_initial(init, problem.svd_cutoff, perturb) if init is not None
           else MPS(problem.initial_bits, problem.svd_cutoff, perturb)).run(ops)
    vals = np.array([observable_value(mps, qubit_at, o) for o in problem.observables])
    return SampleResult(sample=s, sign=circ.sign, n_gates=circ.n_gates, values=vals,
                        stats=mps.stats, bonds=mps.bonds())


def run(problem, samples: Optional[Sequence[int]] = None,
        layers: Optional[int] = None) -> RunResult:
    table = pai.build_table(problem)
    if samples is None:
        samples = range(problem.sample_offset, problem.sample_offset + problem.n_samples)
    res = [run_sample(problem, table, s, layers) for s in samples]
    lg = table.log_g1(layers)
    w = weights([r.sign for r in res], lg)
    vals = np.stack([r.values for r in res]) if res else np.zeros((0, len(problem.observables)))
    mean, se, cv = estimate(vals, w)
    return RunResult(samples=res, log_g1=lg, weights=w, values=vals, mean=mean,
                     std_err=se, config_var=cv)
