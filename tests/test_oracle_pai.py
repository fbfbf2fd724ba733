"""Pins of the oracle's RNG, PAI coefficients, table and sampler.

Each test checks the oracle against something other than itself: published
known-answer vectors, the channel identity the PAI coefficients are derived
from, closed forms and limits stated in the paper, and exact statistics.
"""
import math
import os

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai, sampler
from oracle.philox import philox4x32_10, uniform_u64
from oracle.schedule import pauli_matrix, setting_operator

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = philox4x32_10(tuple(w[0:4]), tuple(w[4:6]))
        assert [int(o) for o in out] == w[6:10]


def test_uniform_u64_uses_declared_counter_layout():
    # counter = (g_lo, g_hi, sample, stream), key = (seed_lo, seed_hi)
    seed, s, g = 0x123456789ABCDEF0, 77, (5 << 32) | 9
    x = philox4x32_10((9, 5, 77, 1), (0x9ABCDEF0, 0x12345678))
    want = (int(x[1]) << 32) | int(x[0])
    assert int(uniform_u64(seed, s, np.array([g], dtype=np.uint64))[0]) == want


def superop(U):
    """Superoperator of rho -> U rho U^dag acting on row-major vec(rho)."""
    return np.kron(U, U.conj())


def rot(paulis, th):
    P = pauli_matrix(paulis)
    return math.cos(th / 2) * np.eye(P.shape[0]) - 1j * math.sin(th / 2) * P


@pytest.mark.parametrize("paulis", ["X", "Z", "XX", "YY", "ZZ", "XY"])
@pytest.mark.parametrize("delta", [math.pi / 512, math.pi / 64, 0.3, 1.0, 2.5])
def test_channel_identity(paulis, delta):
    """R(theta) = gamma1 A + gamma2 B + gamma3 C as channels (appendix PAI)."""
    for th in np.linspace(-delta, delta, 13):
        g = pai.gammas(abs(th), delta)
        A = np.eye(2 ** len(paulis))
        B = rot(paulis, math.copysign(delta, th) if th != 0 else delta)
        C = rot(paulis, math.pi)
        lhs = superop(rot(paulis, th))
        rhs = g[0] * superop(A) + g[1] * superop(B) + g[2] * superop(C)
        assert np.max(np.abs(lhs - rhs)) < 1e-13
        # the settings used by the simulators are the same channels
        Bs = setting_operator(paulis, th, delta, sampler.SET_B)
        Cs = setting_operator(paulis, th, delta, sampler.SET_C)
        rhs2 = g[0] * superop(A) + g[1] * superop(Bs) + g[2] * superop(Cs)
        assert np.max(np.abs(lhs - rhs2)) < 1e-13


def test_channel_identity_is_not_a_unitary_identity():
    # the decomposition holds for superoperators only; the same combination of
    # unitaries misses R(theta) (so a test on unitaries would be wrong)
    d, th = math.pi / 64, 0.01
    g = pai.gammas(th, d)
    U = g[0] * np.eye(2) + g[1] * rot("X", d) + g[2] * rot("X", math.pi)
    assert np.max(np.abs(U - rot("X", th))) > 1e-6


def test_gamma_special_cases_and_signs():
    for d in [math.pi / 256, 0.1, 1.3, 3.0]:
        assert np.allclose(pai.gammas(0.0, d), (1.0, 0.0, 0.0), atol=1e-15)
        assert np.allclose(pai.gammas(d, d), (0.0, 1.0, 0.0), atol=1e-14)
        for th in np.linspace(0, d, 17):
            g1, g2, g3 = pai.gammas(th, d)
            assert abs(g1 + g2 + g3 - 1.0) < 1e-14
            assert g1 >= -1e-15 and g2 >= -1e-15 and g3 <= 1e-15
            assert abs((abs(g1) + abs(g2) + abs(g3)) - (1 - 2 * g3)) < 1e-14


def test_thresholds_are_exact_floors():
    p = ti.config(4)
    t = pai.build_table(p)
    for r in t.rows:
        assert r.t1 == (pai.T_ONE if r.p[0] >= 1 else math.floor(r.p[0] * 2 ** 63))
        assert r.t1 <= r.t2 <= pai.T_ONE
        assert abs(sum(r.p) - 1) < 1e-15


def test_splitting_reproduces_rotation():
    p = ti.config(4)
    t = pai.build_table(p)
    assert t.n_split_terms > 0
    by_term = {}
    for r in t.rows:
        by_term.setdefault(r.term, []).append(r.theta)
    for k, thetas in by_term.items():
        full = pai.theta_of(p.terms[k].coeff, p.total_time, p.trotter_steps)
        assert all(abs(x) <= p.delta for x in thetas)
        assert len(thetas) == (1 if abs(full) <= p.delta else math.ceil(abs(full) / p.delta))
        U = np.eye(2 ** len(p.terms[k].paulis))
        for x in thetas:
            U = rot(p.terms[k].paulis, x) @ U
        assert np.max(np.abs(U - rot(p.terms[k].paulis, full))) < 1e-14
    # rows follow term order (time order)
    assert [r.term for r in t.rows] == sorted(r.term for r in t.rows)


def c1_norm(p):
    return sum(abs(t.coeff) for t in p.terms)


def test_g1_limit_eq_overhead():
    """||g||_1 -> exp(2 tan(Delta/2) ||c||_1 T) as N -> infinity (eq. overhead)."""
    p = ti.config(2)
    want = 2 * math.tan(p.delta / 2) * c1_norm(p) * p.total_time
    vals, errs = [], []
    for N in (10 ** 4, 10 ** 5, 10 ** 6):
        t = pai.build_table(p.with_(trotter_steps=N))
        vals.append(t.log_g1())
        errs.append(abs(t.log_g1() - want) / want)
    assert errs[2] < 2e-4
    assert 9 < errs[0] / errs[1] < 11 and 9 < errs[1] / errs[2] < 11   # O(1/N)
    richardson = (10 * vals[2] - vals[1]) / 9                         # O(1/N^2)
    assert abs(richardson - want) / want < 1e-7


def test_nu_limit_eq_tepai_gates():
    """E[nu] -> csc(Delta)(3 - cos Delta) ||c||_1 T (eq. tepai-gates)."""
    p = ti.config(2)
    want = (3 - math.cos(p.delta)) / math.sin(p.delta) * c1_norm(p) * p.total_time
    means = []
    for N in (10 ** 5, 10 ** 6):
        t = pai.build_table(p.with_(trotter_steps=N))
        means.append(N * sum(r.p[1] + r.p[2] for r in t.rows))
    richardson = (10 * means[1] - means[0]) / 9
    assert abs(means[1] - want) / want < 1e-3
    assert abs(richardson - want) / want < 1e-7


def test_sampler_counts_match_probabilities():
    """Per-row choice counts vs p_l (chi-square) and E[nu], Var[nu] (exact)."""
    p = ti.small_ring(8, seed=3, T=1.0, N=60, delta=math.pi / 32)
    t = pai.build_table(p)
    L = t.l_eff
    counts = np.zeros((L, 3))
    nus = []
    ns = 300
    for s in range(ns):
        c = sampler.sample_circuit(p, t, s)
        nus.append(c.n_gates)
        k = (c.draws % np.uint64(L)).astype(int)
        for sel in (1, 2):
            np.add.at(counts[:, sel], k[c.settings == sel], 1)
        # sign = (-1)^(#C)
        assert c.sign == (-1) ** int(np.count_nonzero(c.settings == 2))
        assert np.all(np.diff(c.draws.astype(np.int64)) > 0)
    trials = ns * p.trotter_steps
    counts[:, 0] = trials - counts[:, 1] - counts[:, 2]
    P = np.array([r.p for r in t.rows])
    exp = trials * P
    mask = exp > 5
    chi2 = float(np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask]))
    dof = int(mask.sum()) - L
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    q = np.array([r.p[1] + r.p[2] for r in t.rows])
    mean = p.trotter_steps * q.sum()
    var = p.trotter_steps * float(np.sum(q * (1 - q)))
    assert abs(np.mean(nus) - mean) < 5 * math.sqrt(var / ns)
    assert 0.6 < np.var(nus, ddof=1) / var < 1.5


def test_sampler_is_deterministic_and_prefix_consistent():
    p = ti.config(1)
    t = pai.build_table(p)
    a = sampler.sample_circuit(p, t, 17)
    b = sampler.sample_circuit(p, t, 17)
    assert np.array_equal(a.draws, b.draws) and np.array_equal(a.settings, b.settings)
    pre = sampler.sample_circuit(p, t, 17, layers=40)
    n = pre.n_gates
    assert np.array_equal(a.draws[:n], pre.draws)
    assert a.draws[n] >= 40 * t.l_eff
