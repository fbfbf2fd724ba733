"""Pins of the oracle's biased variant without pi rotations.

Appendix "Proof of Statement 3": gamma~ = (1 - lambda, lambda) with
lambda = |theta| / Delta, ||gamma~||_1 = 1, all signs +1, ||g||_1 = 1, and a
per-gate bias R~(theta) - R(theta) = |theta| (Delta - |theta|) / 2 R''(0)
+ O(Delta^3).  The references here are independent of the oracle's
sampler and MPS: the Taylor expansion of the rotation channel, the binomial
closed form of a single commuting term, and a density-matrix evolution
under the two-point channels.
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai, sampler
from oracle.enumerate import exhaustive_expectation
from oracle.run import run

PAULI = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]], complex),
         "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.diag([1.0, -1.0]).astype(complex)}


def pauli_matrix(s):
    m = np.eye(1)
    for c in s:
        m = np.kron(m, PAULI[c])
    return m


def rot(paulis, th):
    P = pauli_matrix(paulis)
    return math.cos(th / 2) * np.eye(P.shape[0]) - 1j * math.sin(th / 2) * P


def superop(U):
    return np.kron(U, U.conj())


def test_no_pi_table():
    p = ti.config(4).with_(no_pi=True)
    t = pai.build_table(p)
    assert t.log_g1_step == 0.0 and t.n_split_terms > 0
    for r in t.rows:
        lam = abs(r.theta) / p.delta
        assert r.gamma == (1.0 - lam, lam, 0.0)
        assert 0.0 <= lam <= 1.0 and r.norm1 == 1.0
        assert r.t1 == pai.to_threshold(1.0 - lam) and r.t2 == pai.T_ONE
    for s in range(4):
        c = sampler.sample_circuit(p, t, s, layers=3)
        assert c.sign == 1 and not np.any(c.settings == sampler.SET_C)


@pytest.mark.parametrize("paulis", ["X", "ZZ", "XY"])
def test_no_pi_bias_is_second_order(paulis):
    d2 = 4 ** len(paulis)
    P = pauli_matrix(paulis)
    R2 = -0.5 * np.eye(d2) + 0.5 * np.kron(P, P.conj())     # d^2/dtheta^2 of U (x) conj(U) at 0
    ratios = []
    for delta in (0.2, 0.1, 0.05, 0.025):
        worst = 0.0
        for th in np.linspace(-delta, delta, 9):
            g = pai.gammas_no_pi(abs(th), delta)
            B = rot(paulis, math.copysign(delta, th) if th != 0 else delta)
            diff = g[0] * np.eye(d2) + g[1] * superop(B) - superop(rot(paulis, th))
            pred = abs(th) * (delta - abs(th)) / 2.0 * R2
            worst = max(worst, float(np.max(np.abs(diff - pred))))
            # the leading term itself is not negligible
            if 0 < abs(th) < delta:
                assert np.max(np.abs(diff)) > 0.1 * np.max(np.abs(pred))
        ratios.append(worst / delta ** 3)
    assert max(ratios) < 0.1                # the remainder is third order


def single_term(no_pi=True, N=50, ns=2000):
    return ti.Problem(n_qubits=2, terms=(ti.Term("XX", (0, 1), 0.8),), total_time=1.0,
                      trotter_steps=N, delta=math.pi / 16, n_samples=ns, seed=5,
                      chi_max=4, initial_bits="00", no_pi=no_pi,
                      observables=((ti.PauliString("Z", (0,)),),))


def test_no_pi_single_term_closed_form_and_bias():
    """H = c X0 X1 on |00>: each sample gives cos(b Delta), b ~ Binomial(N, lambda)."""
    p = single_term()
    t = pai.build_table(p)
    lam = t.rows[0].gamma[1]
    theta = 2 * 0.8 * p.total_time / p.trotter_steps
    assert abs(lam - theta / p.delta) < 1e-15
    z = (1 - lam + lam * np.exp(1j * p.delta)) ** p.trotter_steps
    e_biased = z.real
    # the exact evolution gives e^{i N theta}; the per-gate factor has modulus
    # sqrt(1 - 2 lam (1 - lam) (1 - cos D)) = 1 - theta (D - theta) / 2 + O(D^4):
    # the second-order bias of the two-point formula
    pred = p.trotter_steps * theta * (p.delta - theta) / 2
    assert abs((1 - abs(z)) - pred) < 0.1 * pred
    assert abs(abs(z) - (1 - 2 * lam * (1 - lam) * (1 - math.cos(p.delta))) ** (p.trotter_steps / 2)) < 1e-14
    r = run(p)
    assert np.all(r.weights == 1.0)
    for sr in r.samples[:50]:
        c = sampler.sample_circuit(p, t, sr.sample)
        b = int(np.count_nonzero(c.settings == sampler.SET_B))
        assert abs(sr.values[0] - math.cos(b * p.delta)) < 1e-12
    assert abs(r.mean[0] - e_biased) < 5 * r.std_err[0]
    var = 0.5 * (1 + ((1 - lam + lam * np.exp(2j * p.delta)) ** p.trotter_steps).real) - e_biased ** 2
    assert 0.7 < r.std_err[0] ** 2 * p.n_samples / var < 1.3


def full_unitary(n, paulis, qubits, angle):
    """exp(-i angle P / 2) on the n-qubit register (qubit 0 most significant)."""
    P = full_pauli(n, ti.PauliString(paulis, tuple(qubits)))
    return math.cos(angle / 2) * np.eye(2 ** n) - 1j * math.sin(angle / 2) * P


def test_no_pi_exhaustive_sum_equals_channel_evolution():
    """sum_l g~_l <O>_l = Tr[O rho_T], rho_T from the two-point channels gate by gate."""
    terms = (ti.Term("XX", (0, 1), 0.9), ti.Term("YZ", (0, 1), -0.6),
             ti.Term("Z", (0,), 0.7), ti.Term("X", (1,), -0.5))
    p = ti.Problem(n_qubits=2, terms=terms, total_time=0.35, trotter_steps=2,
                   delta=math.pi / 4, n_samples=1, seed=1, chi_max=4, no_pi=True,
                   initial_bits="01", observables=((ti.PauliString("Z", (0,)),),
                                                   (ti.PauliString("YX", (0, 1)),)))
    t = pai.build_table(p)
    got = exhaustive_expectation(p, t, list(p.observables))
    psi0 = np.zeros(4, complex)
    psi0[int(p.initial_bits, 2)] = 1.0
    rho = np.outer(psi0, psi0.conj())
    for _ in range(p.trotter_steps):
        for term in p.terms:
            th = 2 * term.coeff * p.total_time / p.trotter_steps
            lam = abs(th) / p.delta
            B = full_unitary(2, term.paulis, term.qubits, math.copysign(p.delta, th))
            rho = (1 - lam) * rho + lam * B @ rho @ B.conj().T
    for o, obs in enumerate(p.observables):
        O = sum(ps.coeff * full_pauli(2, ps) for ps in obs)
        assert abs(got[o] - np.trace(O @ rho).real) < 1e-13


def full_pauli(n, ps):
    ops = ["I"] * n
    for q, c in zip(ps.qubits, ps.paulis):
        ops[q] = c
    return pauli_matrix("".join(ops))
