"""Pins of the hybrid start: every sample begins from a shared Trotter state.

The method's hybrid use (sec. "Implementation", Trotter-then-TE-PAI) evolves
with a deep Trotter circuit to t0 and continues with TE-PAI.  References: the
dense state vector of the same Trotter circuit, the dense evolution of each
sampled continuation, and the full dense Trotter evolution to t0 + T (the
TE-PAI segment is unbiased, Statement 1).
"""
import math

import numpy as np

import tepai_inputs as ti
from oracle import dense, pai, sampler
from oracle.run import run, run_sample
from oracle.schedule import setting_operator
from oracle.trotter import trotter_initial_mps


def hybrid(n=6, T0=0.4, N0=8, T=0.3, N=6, chi=8, ns=6, seed=3):
    pre = ti.small_ring(n, seed=seed, T=T0, N=N0, delta=math.pi / 16, chi=chi, n_samples=1)
    init = trotter_initial_mps(pre, N0, chi)
    seg = pre.with_(total_time=T, trotter_steps=N, n_samples=ns, initial_mps=init)
    return pre, init, seg


def dense_of(init):
    v = np.ones((1, 1), complex)
    for A in init.tensors:
        v = np.einsum("xa,asb->xsb", v, A).reshape(-1, A.shape[2])
    return dense.site_to_qubit_order(v.reshape((2,) * len(init.tensors)), init.qubit_at)


def test_trotter_mps_equals_dense_trotter_in_exact_regime():
    pre, init, _ = hybrid()
    assert sorted(init.qubit_at) == list(range(pre.n_qubits))
    assert init.qubit_at != tuple(range(pre.n_qubits))       # the wrap bond rotated the chain
    psi, ref = dense_of(init), dense.trotter_state(pre)
    fid = abs(np.vdot(ref, psi)) / (np.linalg.norm(ref) * np.linalg.norm(psi))
    assert abs(fid - 1.0) < 1e-12
    # mixed-canonical about the centre
    for k, A in enumerate(init.tensors):
        cl, _, cr = A.shape
        if k < init.centre:
            M = A.reshape(cl * 2, cr)
            assert np.allclose(M.conj().T @ M, np.eye(cr), atol=1e-12)
        elif k > init.centre:
            M = A.reshape(cl, 2 * cr)
            assert np.allclose(M @ M.conj().T, np.eye(cl), atol=1e-12)


def test_hybrid_samples_equal_dense_continuations():
    pre, init, seg = hybrid()
    t = pai.build_table(seg)
    psi0 = dense.trotter_state(pre)
    for s in range(seg.n_samples):
        r = run_sample(seg, t, s)
        c = sampler.sample_circuit(seg, t, s)
        psi = psi0
        for g, st in zip(c.draws.tolist(), c.settings.tolist()):
            row = t.rows[g % t.l_eff]
            term = seg.terms[row.term]
            psi = dense.apply_op(psi, setting_operator(term.paulis, row.theta, seg.delta, st),
                                 term.qubits)
        for o, obs in enumerate(seg.observables):
            assert abs(r.values[o] - dense.expectation(psi, obs)) < 1e-11


def test_hybrid_estimator_is_unbiased_for_the_whole_evolution():
    pre, init, seg = hybrid(ns=1500, seed=6)
    psi = dense.trotter_state(pre)
    for _ in range(seg.trotter_steps):
        for term in seg.terms:
            th = 2 * term.coeff * seg.total_time / seg.trotter_steps
            psi = dense.apply_op(psi, dense.rotation(term.paulis, th), term.qubits)
    r = run(seg)
    for o, obs in enumerate(seg.observables):
        assert abs(r.mean[o] - dense.expectation(psi, obs)) < 5 * r.std_err[o]
