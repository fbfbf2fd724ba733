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


# ---------------------------------------------------------------- accounting
@pytest.mark.parametrize("chi", [1, 2, 16, 128, 256])
def test_nominal_update_flops_uniform_chi_is_704_chi_cubed(chi):
    """At uniform bond chi the per-update count is 32 chi^3 for the
    (2chi x chi)(chi x 2chi) complex contraction plus the Golub-Reinsch SVD
    of the 2chi x 2chi result, 4 (4 + 8 + 9) (2chi)^3 = 672 chi^3."""
    from oracle.mps import nominal_update_flops, svd_flops
    assert nominal_update_flops(chi, chi, chi) == 704.0 * chi ** 3
    assert svd_flops(2 * chi, 2 * chi) == 672.0 * chi ** 3
    # thin SVD of a tall matrix: 4 (4 m^2 n + 8 m n^2 + 9 n^3), either orientation
    assert svd_flops(6, 2) == svd_flops(2, 6) == 4 * (4 * 36 * 2 + 8 * 6 * 4 + 9 * 8)


def test_sum_chi3_and_flops_follow_the_update_log():
    """The counters add chi_mid^3 and the nominal count of every update, in
    the order the updates run (replayed here from the operation list)."""
    from oracle.mps import nominal_update_flops
    p = ti.small_ring(8, seed=4, T=0.4, N=6, delta=math.pi / 16, chi=4, n_samples=1)
    t = pai.build_table(p)
    c = sampler.sample_circuit(p, t, 0)
    ops, _ = schedule.build_schedule(p, t, c)
    m = MPS(p.initial_bits, p.svd_cutoff)
    chi3, flops, n = 0.0, 0.0, 0
    for op in ops:
        if op[0] == "update":
            i = op[1]
            cl, cm, cr = m.A[i].shape[0], m.A[i].shape[2], m.A[i + 1].shape[2]
            chi3 += float(cm) ** 3
            flops += nominal_update_flops(cl, cm, cr)
            n += 1
        m.run([op])
    assert n == m.stats.updates > 0
    assert m.stats.sum_chi3 == chi3 and m.stats.nominal_flops == flops


# ------------------------------------------------------------- near-ties
def _unitary(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _truncated_state(M, k):
    U, S, Vh = np.linalg.svd(M, full_matrices=False)
    psi = (U[:, :k] * S[:k]) @ Vh[:k]
    return psi.reshape(-1) / np.linalg.norm(S[:k])


@pytest.mark.parametrize("s_cut", [0.3, 1e-3])
@pytest.mark.parametrize("gap", [1e-4, 1e-6, 1e-8, 1e-10])
def test_cut_sensitivity_bounds_truncations_of_nearby_matrices(s_cut, gap):
    """Two matrices eta sigma_0 apart (two SVDs with backward error eta) give
    truncated states whose expectation values, over every observable of unit
    norm, differ by at most the cut's bound B (with eps = eta) plus the
    direct effect of the perturbation, 4 eta / |sigma_kept|; and when the gap
    is far below eta the straddling pair is mixed and B is attained to within
    a small factor (so B scales with sigma_{k-1}, not with the gap alone)."""
    from oracle.mps import cut_sensitivity
    rng = np.random.default_rng(17)
    R, C, k, eta = 24, 20, 8, 1e-6
    head = np.geomspace(1.0, 3 * s_cut, k - 1)
    tail = np.geomspace(0.5 * s_cut, 1e-3 * s_cut, C - k - 1)
    sig = np.concatenate([head, [s_cut, s_cut - gap * 1.0], tail])
    assert np.all(np.diff(sig) <= 0)
    M = (_unitary(R, rng)[:, :C] * sig) @ _unitary(C, rng)
    E = rng.standard_normal((R, C)) + 1j * rng.standard_normal((R, C))
    E *= eta * sig[0] / np.linalg.norm(E, 2)
    a, b = _truncated_state(M, k), _truncated_state(M + E, k)
    worst = 2.0 * math.sqrt(max(0.0, 1.0 - abs(np.vdot(a, b)) ** 2))   # max over |O| <= 1
    S = np.linalg.svd(M, compute_uv=False)
    B = cut_sensitivity(S, k, R, C, eps=eta)
    kept = np.linalg.norm(S[:k])
    assert worst <= B + 4 * eta / kept, (worst, B)
    if gap < 1e-2 * eta:
        assert worst >= B / 30, (worst, B)


def test_nonfinite_tensor_flags_the_sample():
    """A non-finite entry (forced into an oracle tensor) flags the sample and
    makes its values NaN instead of stopping the run."""
    from oracle.mps import NONFINITE
    p = ti.small_ring(6, seed=2, T=0.3, N=4, delta=math.pi / 16, chi=4, n_samples=1)
    t = pai.build_table(p)
    c = sampler.sample_circuit(p, t, 0)
    ops, qa = schedule.build_schedule(p, t, c)
    m = MPS(p.initial_bits, p.svd_cutoff)
    m.A[2] = m.A[2].copy()
    m.A[2][0, 0, 0] = np.nan
    m.run(ops)
    assert m.stats.flags & NONFINITE
    assert math.isnan(observable_value(m, qa, p.observables[0]))


def test_rounding_sensitivity_run():
    """The perturbed oracle run (a random backward error of u sqrt(R C) |M|
    added before every factorisation) moves a well-conditioned trajectory by
    rounding-level amounts, scales with the perturbation, and separates a
    trajectory whose cap cut falls inside an exactly degenerate pair."""
    # exact regime (no cap cut): the change stays at the rounding level
    p = ti.config(1)
    t = pai.build_table(p)
    r = run_sample(p, t, 3)
    d64 = np.max(np.abs(run_sample(p, t, 3, perturb=(1, 1.0)).values - r.values))
    d32 = np.max(np.abs(run_sample(p, t, 3, perturb=(1, 2.0 ** 29)).values - r.values))
    assert 0 < d64 < 1e-12
    assert 1e-9 < d32 < 1e-4 and d32 > 1e5 * d64
    # cap 2 with a doubly degenerate spectrum at the cut (the kept vector is
    # not unique): a rounding-level perturbation moves the values at O(1e-2)
    q = ti.small_ring(10, seed=7, T=0.4, N=10, delta=math.pi / 16, chi=8, n_samples=6)
    q = q.with_(chi_per_sample=(2, 4, 8, 3, 8, 5))
    tq = pai.build_table(q)
    rq = run_sample(q, tq, 0)
    assert rq.stats.ties > 0
    assert np.max(np.abs(run_sample(q, tq, 0, perturb=(1, 1.0)).values - rq.values)) > 1e-6


# ------------------------------------------------------------ per-gate mode
def test_per_gate_mode_exact_regime_matches_dense_and_fused():
    """One truncated update per sampled gate changes only where the
    truncations happen: at full bond dimension the state equals the dense
    state of the same sampled circuit, and the fused schedule's."""
    p = ti.config(1).with_(per_gate=True)
    t = pai.build_table(p)
    for s in (0, 4):
        c, ops, qa, m = mps_for(p, t, s)
        psi_m = qubit_state(m, qa).reshape(-1)
        psi_c = dense.circuit_state(p, t, c).reshape(-1)
        assert np.max(np.abs(psi_m - psi_c)) < 1e-12
        _, ops_f, qa_f, m_f = mps_for(p.with_(per_gate=False), t, s)
        assert np.max(np.abs(qubit_state(m_f, qa_f).reshape(-1) - psi_m)) < 1e-12


def test_per_gate_update_count_is_one_per_b_gate_plus_routing():
    """Every sampled B setting on a qubit pair is one two-site update; the
    wrap pair adds hi - lo - 1 SWAP updates when its qubits are not adjacent;
    C settings on pairs cost no update."""
    p = ti.small_ring(8, seed=6, T=0.5, N=8, delta=math.pi / 16, chi=4, n_samples=1)
    pg = p.with_(per_gate=True)
    t = pai.build_table(p)
    c = sampler.sample_circuit(p, t, 0)
    ops_g, _ = schedule.build_schedule(pg, t, c)
    ops_f, _ = schedule.build_schedule(p, t, c)
    n_b2 = sum(1 for g, st in zip(c.draws.tolist(), c.settings.tolist())
               if st == sampler.SET_B and len(p.terms[t.rows[g % t.l_eff].term].qubits) == 2)
    swaps = sum(1 for op in ops_g if op[0] == "update" and np.allclose(op[2], schedule.SWAP4))
    n_upd = sum(1 for op in ops_g if op[0] == "update")
    assert n_upd == n_b2 + swaps
    assert n_upd > sum(1 for op in ops_f if op[0] == "update")
