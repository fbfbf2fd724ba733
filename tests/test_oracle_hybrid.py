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


# ------------------------------------------------ truncation on copy
def centred(init, c):
    """The same state with its orthogonality centre moved to site c."""
    from oracle.mps import MPS
    m = MPS.from_initial(init)
    while m.centre < c:
        m.shift(m.centre, +1)
    return ti.InitialMPS(tensors=tuple(m.A), centre=c, qubit_at=init.qubit_at)


def dense_truncation_sweep(psi, n, chi, cutoff=1e-12):
    """The definition written out on the state vector: the optimal rank-k cut
    (k = min(chi, #{sigma > cutoff sigma_0}), renormalised) after site 0,
    then after site 1 of the state that cut left, and so on."""
    for c in range(n - 1):
        U, S, Vh = np.linalg.svd(psi.reshape(2 ** (c + 1), -1), full_matrices=False)
        k = min(chi, max(int(np.count_nonzero(S > cutoff * S[0])), 1))
        psi = ((U[:, :k] * (S[:k] / np.linalg.norm(S[:k]))) @ Vh[:k]).reshape(-1)
    return psi


def test_truncation_on_copy_equals_the_dense_sweep():
    from oracle.mps import MPS
    init = centred(ti.random_mps(7, 8, seed=5), 3)
    m0 = MPS.from_initial(init)
    psi0 = m0.to_dense()
    assert max(m0.bonds()) == 8
    for chi in (1, 2, 3, 5):
        m = MPS.from_initial(init)
        m.truncate_to(chi)
        assert max(m.bonds()) <= chi and m.centre == 6
        ref = dense_truncation_sweep(psi0, 7, chi)
        assert np.max(np.abs(m.to_dense() - ref)) <= 1e-12, chi
        assert abs(np.linalg.norm(m.to_dense()) - 1.0) <= 1e-13
        for A in m.A[:-1]:      # sites left of the centre are left-canonical
            X = A.reshape(-1, A.shape[2])
            assert np.allclose(X.conj().T @ X, np.eye(X.shape[1]), atol=1e-12)
        assert m.stats.shifts == 3 + 6     # exact shifts to site 0, then the sweep


def test_truncation_on_copy_only_below_the_largest_bond():
    # a sample whose cap holds the shared state starts from it unchanged;
    # one with a smaller cap starts with the truncation sweep
    init = centred(ti.random_mps(7, 8, seed=5), 3)
    p = ti.small_ring(7, seed=2, T=0.2, N=2, delta=math.pi / 16, chi=8, n_samples=3,
                      periodic=False).with_(initial_mps=init, chi_per_sample=(8, 4, 2))
    t = pai.build_table(p)
    from oracle.schedule import build_schedule
    for s, chi in enumerate((8, 4, 2)):
        ops, _ = build_schedule(p, t, sampler.sample_circuit(p, t, s), chi)
        assert (ops[0] == ("truncate", chi)) == (chi < 8)
        r = run_sample(p, t, s)
        assert max(r.bonds) <= chi
