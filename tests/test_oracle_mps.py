"""Pins of the oracle's MPS simulator and schedule.

* exact regime: MPS result equals the dense state vector of the same sampled
  circuit (including the SWAP-routed wrap bond);
* truncated regime: MPS equals the dense replay of the same operation list,
  where every truncation is a Schmidt cut of the whole state (Eckart-Young);
* invariants: norm, canonical isometries, truncation error bound;
* diagonal Hamiltonians leave a product state a product state.
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import dense, pai, sampler, schedule
from oracle.mps import MPS
from oracle.run import observable_value, run_sample


def mps_for(p, t, s, chi=None):
    c = sampler.sample_circuit(p, t, s)
    ops, qubit_at = schedule.build_schedule(p, t, c, chi)
    m = MPS(p.initial_bits, p.svd_cutoff).run(ops)
    return c, ops, qubit_at, m


def qubit_state(m, qubit_at):
    return dense.site_to_qubit_order(m.to_dense().reshape((2,) * m.n), qubit_at)


@pytest.mark.parametrize("s", [0, 1, 5, 11])
def test_exact_regime_matches_dense_circuit_cfg1(s):
    p = ti.config(1)
    t = pai.build_table(p)
    c, ops, qa, m = mps_for(p, t, s)
    assert sorted(qa) == list(range(p.n_qubits))
    psi_m = qubit_state(m, qa).reshape(-1)
    psi_c = dense.circuit_state(p, t, c).reshape(-1)
    assert abs(abs(np.vdot(psi_m, psi_c)) - 1.0) < 1e-12
    # same phase too: the schedule applies exactly the sampled operators
    assert np.max(np.abs(psi_m - psi_c)) < 1e-12
    for obs in p.observables:
        assert abs(observable_value(m, qa, obs) - dense.expectation(psi_c.reshape((2,) * 8), obs)) < 1e-12


def test_exact_regime_open_chain_and_general_pairs():
    # open chain with mixed two-qubit Pauli pairs (non-commuting on one bond)
    n = 6
    h = ti.disorder(n, -1, 1, seed=9)
    terms = list(ti.spin_ring(n, h, periodic=False))
    terms += [ti.Term("XY", (2, 3), 0.7), ti.Term("ZX", (4, 3), -0.4),
              ti.Term("YZ", (5, 0), 0.3)]
    p = ti.Problem(n_qubits=n, terms=tuple(terms), total_time=0.6, trotter_steps=8,
                   delta=math.pi / 8, n_samples=4, seed=21, chi_max=8,
                   initial_bits="011010", observables=ti.z_all(n))
    t = pai.build_table(p)
    for s in range(4):
        c, ops, qa, m = mps_for(p, t, s)
        psi_m = qubit_state(m, qa).reshape(-1)
        psi_c = dense.circuit_state(p, t, c).reshape(-1)
        assert np.max(np.abs(psi_m - psi_c)) < 1e-12


@pytest.mark.parametrize("chi", [2, 3, 5])
def test_truncated_updates_are_schmidt_cuts(chi):
    """Every operation equals the dense Schmidt cut of the state it starts from."""
    p = ti.small_ring(10, seed=4, T=0.8, N=16, delta=math.pi / 16, chi=chi)
    t = pai.build_table(p)
    for s in range(2):
        c = sampler.sample_circuit(p, t, s)
        ops, qa = schedule.build_schedule(p, t, c, chi)
        m = MPS(p.initial_bits, p.svd_cutoff)
        worst = 0.0
        for op in ops:
            before = m.to_dense().reshape((2,) * p.n_qubits)
            m.run([op])
            if op[0] == "local":
                ref = dense.apply_op(before, op[2], (op[1],))
            elif op[0] == "update":
                ref = dense.apply_op(before, op[2], (op[1], op[1] + 1))
                ref = dense.schmidt_cut(ref, op[1], op[3], p.svd_cutoff, True)
            else:
                bond = op[1] if op[2] > 0 else op[1] - 1
                ref = dense.schmidt_cut(before, bond, 1 << 30, p.svd_cutoff, False)
            worst = max(worst, float(np.max(np.abs(m.to_dense() - ref.reshape(-1)))))
        assert m.stats.discarded > 0          # truncation really happens
        assert max(m.bonds()) <= chi
        # rounding moves a truncated subspace by ~ eps / gap (Wedin's bound)
        assert worst < 1e-12 + 1e-14 / m.stats.min_gap


def test_truncated_trajectory_matches_dense_replay():
    # a well-conditioned case (Schmidt gaps at the cut >= 3e-4): the whole
    # truncated trajectory agrees with the dense replay of the same schedule
    p = ti.small_ring(10, seed=4, T=0.4, N=12, delta=math.pi / 16, chi=4)
    t = pai.build_table(p)
    for s in range(4):
        c, ops, qa, m = mps_for(p, t, s)
        assert m.stats.discarded > 1e-2 and m.stats.min_gap > 3e-4
        ref = dense.schedule_state(p, ops).reshape(-1)
        assert np.max(np.abs(m.to_dense() - ref)) < 1e-12


def test_invariants_norm_isometry_and_truncation_bound():
    p = ti.small_ring(10, seed=6, T=0.8, N=16, delta=math.pi / 16, chi=4)
    t = pai.build_table(p)
    c, ops, qa, m = mps_for(p, t, 2)
    assert abs(np.linalg.norm(m.to_dense()) - 1) < 1e-13
    for k, A in enumerate(m.A):
        cl, _, cr = A.shape
        if k < m.centre:
            M = A.reshape(cl * 2, cr)
            assert np.max(np.abs(M.conj().T @ M - np.eye(cr))) < 1e-13
        elif k > m.centre:
            M = A.reshape(cl, 2 * cr)
            assert np.max(np.abs(M @ M.conj().T - np.eye(cl))) < 1e-13
    # |<O>_chi - <O>_exact| <= 2 ||O|| sum_m sqrt(2 eps_m)
    psi_c = dense.circuit_state(p, t, c)
    eps_total = 0.0
    m2 = MPS(p.initial_bits, p.svd_cutoff)
    bound = 0.0
    for op in ops:
        before = m2.stats.discarded
        m2.run([op])
        bound += 2 * math.sqrt(2 * max(m2.stats.discarded - before, 0.0))
    for obs in p.observables:
        err = abs(observable_value(m, qa, obs) - dense.expectation(psi_c, obs))
        assert err <= bound + 1e-12


def test_unitarity_without_truncation():
    # with chi large enough nothing is discarded and the norm before
    # renormalisation stays 1 (the update is unitary)
    p = ti.small_ring(6, seed=8, T=0.5, N=10, delta=math.pi / 16, chi=64)
    t = pai.build_table(p)
    c, ops, qa, m = mps_for(p, t, 0)
    assert m.stats.discarded < 1e-20


def test_diagonal_hamiltonian_keeps_product_state():
    n = 6
    terms = tuple([ti.Term("Z", (i,), 0.3 * (i + 1)) for i in range(n)] +
                  [ti.Term("ZZ", (i, (i + 1) % n), 0.5) for i in range(n)])
    p = ti.Problem(n_qubits=n, terms=terms, total_time=1.0, trotter_steps=20,
                   delta=math.pi / 16, n_samples=6, seed=5, chi_max=8,
                   initial_bits="010011", observables=ti.z_all(n))
    t = pai.build_table(p)
    for s in range(6):
        r = run_sample(p, t, s)
        assert max(r.bonds) == 1
        z = np.array([1 - 2 * int(b) for b in p.initial_bits], dtype=float)
        assert np.max(np.abs(r.values - z)) < 1e-13


def test_fused_runs_reduce_updates_but_not_the_state():
    # one update per maximal same-bond run: at most one update per bond per
    # Trotter step outside SWAP routes
    p = ti.config(1)
    t = pai.build_table(p)
    c, ops, qa, m = mps_for(p, t, 3)
    n_two_site = sum(1 for g in c.draws.tolist()
                     if len(p.terms[t.rows[g % t.l_eff].term].qubits) == 2)
    gate_updates = sum(1 for o in ops if o[0] == "update" and not np.allclose(o[2], schedule.SWAP4))
    assert gate_updates < n_two_site


def test_transfer_contraction_on_random_state_matches_dense():
    # an entangled state with no structure: every bond at its maximum (or the
    # cap) and every Schmidt spectrum generic, so a dropped term, a swapped
    # index or a missing conjugate in the contraction shows
    n = 9
    init = ti.random_mps(n, 12, seed=4)
    assert init.bonds() == (1, 2, 4, 8, 12, 12, 8, 4, 2, 1)
    for k, A in enumerate(init.tensors[1:], start=1):
        M = A.reshape(A.shape[0], -1)
        assert np.allclose(M @ M.conj().T, np.eye(A.shape[0]), atol=1e-13)
    m = MPS.from_initial(init)
    psi = m.to_dense()
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13
    psi = psi.reshape((2,) * n)
    obs = ti.xyz_all(n) + (ti.zz(0, 5), ti.half_ring_zz(n),
                           (ti.PauliString("XY", (2, 7), 0.3), ti.PauliString("ZZ", (1, 8), -1.1)))
    qa = tuple(range(n))
    for o in obs:
        assert abs(observable_value(m, qa, o) - dense.expectation(psi, o)) < 1e-13
