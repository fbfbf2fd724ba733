"""Pins of the deterministic product-formula mode (the comparison circuit of
sec. "Truncation"): every rotation of every step applied exactly.

References: the dense state vector of the same first-order circuit (eq.
Trotter-Suzuki), the exact evolution e^{-iHT} (first-order convergence in N),
the closed form of a field-only Hamiltonian, and the truncation bound of a
truncate-and-renormalise trajectory.
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import dense, pai
from oracle.pai import T_ONE
from oracle.run import run
from oracle.sampler import sample_circuit


def dense_product(labels):
    init = ti.product_state(labels)
    v = np.ones((1, 1), complex)
    for A in init.tensors:
        v = np.einsum("xa,asb->xsb", v, A).reshape(-1, A.shape[2])
    return v.reshape((2,) * len(labels))


def dense_trotter_from(psi, problem, steps):
    for _ in range(steps):
        for term in problem.terms:
            th = 2.0 * term.coeff * problem.total_time / problem.trotter_steps
            psi = dense.apply_op(psi, dense.rotation(term.paulis, th), term.qubits)
    return psi


def small(n=6, N=12, chi=64, T=0.6, labels=None, **kw):
    labels = labels or ti.plus_with_minus(n)
    p = ti.truncation_workload(chi, trotter=True, n=n, T=T, trotter_steps=N, **kw)
    return p.with_(initial_mps=ti.product_state(labels)), labels


def test_trotter_table():
    p, _ = small(n=6, N=3)          # J = 1 rotations: theta = 2 T / N = 0.4 > Delta, split
    t = pai.build_table(p)
    ref = pai.build_table(p.with_(trotter=False))
    assert t.l_eff == ref.l_eff > len(p.terms)
    assert t.log_g1_step == 0.0
    for r, q in zip(t.rows, ref.rows):
        assert (r.term, r.theta) == (q.term, q.theta)
        assert r.gamma == (0.0, 1.0, 0.0) and r.norm1 == 1.0
        assert (r.t1, r.t2) == (0, T_ONE)
    # the sampler then keeps every rotation, with setting B and sign +1
    c = sample_circuit(p, t, 5, 2)
    assert c.n_gates == 2 * t.l_eff and set(c.settings.tolist()) == {1} and c.sign == 1


@pytest.mark.parametrize("layers", [1, 5, 12])
def test_trotter_equals_dense_product_formula_when_exact(layers):
    p, labels = small()
    r = run(p.with_(n_samples=2), layers=layers)
    psi = dense_trotter_from(dense_product(labels), p, layers)
    ref = np.array([dense.expectation(psi, o) for o in p.observables])
    assert np.max(np.abs(r.values - ref[None, :])) < 1e-12
    assert np.all(r.weights == 1.0) and r.log_g1 == 0.0
    assert np.array_equal(r.values[0], r.values[1])
    assert all(s.n_gates == layers * pai.build_table(p).l_eff for s in r.samples)


def test_trotter_converges_to_exact_evolution_at_first_order():
    n = 5
    errs = []
    for N in (8, 16, 32):
        p, labels = small(n=n, N=N, T=0.5)
        vals = run(p).values[0]
        w, V = np.linalg.eigh(dense.hamiltonian(p))
        psi0 = dense_product(labels).reshape(-1)
        psi = (V @ (np.exp(-1j * w * p.total_time) * (V.conj().T @ psi0))).reshape((2,) * n)
        ref = np.array([dense.expectation(psi, o) for o in p.observables])
        errs.append(np.max(np.abs(vals - ref)))
    assert errs[0] > 1e-3                                   # the formula is not exact
    for a, b in zip(errs, errs[1:]):
        assert 1.6 < a / b < 2.4                            # error ~ 1 / N


def test_field_only_closed_form_at_chi_one():
    # H = sum omega_i Z_i commutes term by term: the product formula is exact
    # and the state stays a product, so chi = 1 loses nothing.
    n, T = 4, 0.9
    om = ti.disorder(n, -1.0, 1.0, seed=11)
    terms = tuple(ti.Term("Z", (i,), float(om[i])) for i in range(n))
    p, _ = small(n=n, N=7, chi=1, T=T, labels="+" * n)
    p = p.with_(terms=terms)
    v = run(p).values[0].reshape(n, 3)
    assert np.allclose(v[:, 0], np.cos(2 * om * T), atol=1e-13)
    assert np.allclose(v[:, 1], np.sin(2 * om * T), atol=1e-13)
    assert np.allclose(v[:, 2], 0.0, atol=1e-13)


def test_truncated_trotter_within_discarded_weight_bound():
    p, labels = small(n=6, N=10, chi=2, T=0.8)
    r = run(p)
    s = r.samples[0]
    assert s.stats.discarded > 1e-6                         # chi = 2 truncates
    assert max(s.bonds) <= 2
    psi = dense_trotter_from(dense_product(labels), p, p.trotter_steps)
    ref = np.array([dense.expectation(psi, o) for o in p.observables])
    # each truncate-and-renormalise step moves psi by <= sqrt(2 eps_m);
    # sum_m sqrt(2 eps_m) <= sqrt(2 M sum_m eps_m) (Cauchy-Schwarz)
    bound = 2.0 * math.sqrt(2.0 * s.stats.updates * s.stats.discarded)
    err = np.max(np.abs(r.values[0] - ref))
    assert err <= bound
    assert err > 1e-4                                       # and the error is real


def test_workload_shape():
    p = ti.truncation_workload(16)
    assert (p.n_qubits, p.total_time, p.trotter_steps, p.n_samples) == (20, 1.0, 2000, 100)
    assert p.delta == math.pi / 2 ** 12 and len(p.observables) == 60
    assert ti.plus_with_minus(20)[10] == "-" and ti.plus_with_minus(20).count("-") == 1
    q = ti.truncation_workload(2, trotter=True)
    assert q.trotter and q.n_samples == 1 and q.chi_max == 2
