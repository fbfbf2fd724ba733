"""Pins of the oracle's estimator: unbiasedness, closed forms, statistics."""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import dense, pai, sampler
from oracle.enumerate import exhaustive_expectation
from oracle.estimator import estimate, weights
from oracle.run import run


def single_term_problem(c=0.8, T=1.0, N=50, delta=math.pi / 16, ns=400, seed=3):
    return ti.Problem(n_qubits=2, terms=(ti.Term("XX", (0, 1), c),), total_time=T,
                      trotter_steps=N, delta=delta, n_samples=ns, seed=seed,
                      chi_max=4, initial_bits="00",
                      observables=((ti.PauliString("Z", (0,)),),))


def test_single_term_closed_form():
    """H = c X0 X1 on |00>: <Z0> = cos(2cT) and E[x] = Re[(g1 - g3 + g2 e^{iD})^N]."""
    p = single_term_problem()
    t = pai.build_table(p)
    g1, g2, g3 = t.rows[0].gamma
    z = (g1 - g3 + g2 * np.exp(1j * p.delta)) ** p.trotter_steps
    assert abs(z.real - math.cos(2 * 0.8 * p.total_time)) < 1e-13
    r = run(p)
    # per sample: x = ||g||_1 cos(b Delta), b = number of B settings
    for sr, w in zip(r.samples, r.weights):
        c = sampler.sample_circuit(p, t, sr.sample)
        b = int(np.count_nonzero(c.settings == 1))
        assert abs(w * sr.values[0] - math.exp(r.log_g1) * math.cos(b * p.delta)) < 1e-12
    assert abs(r.mean[0] - math.cos(1.6)) < 5 * r.std_err[0]
    # exact variance of x
    p1, p2, p3 = t.rows[0].p
    ex2 = math.exp(2 * r.log_g1) * 0.5 * (1 + ((p1 + p3) + p2 * np.exp(2j * p.delta)) ** p.trotter_steps).real
    var = ex2 - math.cos(1.6) ** 2
    assert 0.7 < r.std_err[0] ** 2 * p.n_samples / var < 1.3


def test_deterministic_limit_all_B():
    """theta_k = Delta for every k: every sample is the full Trotter circuit."""
    n = 4
    delta = math.pi / 16
    T, N = 1.0, 8
    c = delta * N / (2 * T)         # theta = 2 c T / N = Delta
    terms = tuple([ti.Term("Z", (i,), c) for i in range(n)] +
                  [ti.Term(pp, (i, (i + 1) % n), c) for i in range(n) for pp in ("XX", "YY", "ZZ")])
    p = ti.Problem(n_qubits=n, terms=terms, total_time=T, trotter_steps=N, delta=delta,
                   n_samples=5, seed=2, chi_max=16, initial_bits="0110",
                   observables=ti.z_all(n))
    t = pai.build_table(p)
    assert all(abs(r.p[1] - 1) < 1e-12 for r in t.rows)
    r = run(p)
    assert np.allclose(r.weights, 1.0, atol=1e-12)
    assert np.all(r.std_err < 1e-12)
    psi = dense.trotter_state(p)
    for o, obs in enumerate(p.observables):
        assert abs(r.mean[o] - dense.expectation(psi, obs)) < 1e-12


@pytest.mark.parametrize("case", ["open2", "ring3"])
def test_exhaustive_sum_equals_trotter(case):
    """Statement 1: sum_l g_l <O>_l = <O>_Trotter (exact, all 3^(L N) settings)."""
    if case == "open2":
        terms = (ti.Term("XX", (0, 1), 0.9), ti.Term("YZ", (0, 1), -0.6),
                 ti.Term("Z", (0,), 0.7), ti.Term("X", (1,), -0.5))
        p = ti.Problem(n_qubits=2, terms=terms, total_time=0.35, trotter_steps=2,
                       delta=math.pi / 4, n_samples=1, seed=1, chi_max=4,
                       initial_bits="01", observables=((ti.PauliString("Z", (0,)),),
                                                       (ti.PauliString("YX", (0, 1)),)))
    else:
        terms = (ti.Term("XX", (0, 1), 1.0), ti.Term("ZZ", (1, 2), 0.6),
                 ti.Term("YY", (2, 0), -0.8), ti.Term("Z", (1,), 0.5))
        p = ti.Problem(n_qubits=3, terms=terms, total_time=0.2, trotter_steps=2,
                       delta=math.pi / 6, n_samples=1, seed=1, chi_max=8,
                       initial_bits="010", observables=((ti.PauliString("Z", (2,)),),))
    t = pai.build_table(p)
    psi = dense.trotter_state(p)
    got = exhaustive_expectation(p, t, list(p.observables))
    for o, obs in enumerate(p.observables):
        assert abs(got[o] - dense.expectation(psi, obs)) < 1e-13


def test_identity_observable_weights_unbiased():
    """E[w_s] = 1 (Sigma gamma = 1) with Var = ||g||_1^2 - 1."""
    p = ti.small_ring(6, seed=7, T=1.0, N=40, delta=math.pi / 32, n_samples=4000)
    t = pai.build_table(p)
    signs = [sampler.sample_circuit(p, t, s).sign for s in range(p.n_samples)]
    w = weights(signs, t.log_g1())
    g1 = math.exp(t.log_g1())
    se = math.sqrt((g1 ** 2 - 1) / p.n_samples)
    assert abs(w.mean() - 1) < 5 * se


def test_estimate_formulae():
    vals = np.array([[0.5, 1.0], [0.25, -1.0], [-0.5, 0.0]])
    w = np.array([2.0, -2.0, 2.0])
    mean, se, cv = estimate(vals, w)
    x = vals * w[:, None]
    assert np.allclose(mean, x.mean(0))
    assert np.allclose(se, x.std(0, ddof=1) / math.sqrt(3))
    assert np.allclose(cv, x.var(0, ddof=1) / 4)


def test_configuration_variance_closed_form():
    """Statement 2's configuration variance against its exact value.

    For H = c X0 X1 on |00> the signed per-circuit value is v = cos(b Delta)
    with b ~ Binomial(N, p_B) (a pi setting flips both the sign of g_l and
    <Z0>), so Var[v] = (1 + Re[(p_A + p_pi + p_B e^{2i Delta})^N]) / 2
    - (cos(2cT) / ||g||_1)^2.  At T = 2, Delta = pi/4 the weight is
    ||g||_1 = 3.35, so dividing the sample variance by ||g||_1 instead of its
    square, or not centring it, is off by far more than the 10% allowed for
    2000 samples (the relative spread of the estimate is ~2%).
    """
    p = single_term_problem(T=2.0, delta=math.pi / 4, ns=2000, seed=1)
    t = pai.build_table(p)
    p1, p2, p3 = t.rows[0].p
    g1 = math.exp(t.log_g1())
    assert g1 > 3
    mean_v = math.cos(2 * 0.8 * p.total_time) / g1
    ev2 = 0.5 * (1 + (((p1 + p3) + p2 * np.exp(2j * p.delta)) ** p.trotter_steps).real)
    exact = ev2 - mean_v ** 2
    r = run(p)
    assert abs(r.config_var[0] / exact - 1) < 0.1, (r.config_var, exact)
    # eq. config_var: Var[x] = ||g||_1^2 Var[v], so N_s SE^2 = ||g||_1^2 cv
    assert abs(p.n_samples * r.std_err[0] ** 2 - g1 ** 2 * r.config_var[0]) < 1e-12 * g1 ** 2


def test_configuration_variance_bound():
    """Var[v] <= 1 for |v| <= 1 (Statement 2); the unbiased sample form
    reaches N_s/(N_s - 1) exactly when half the values are +1, half -1."""
    rng = np.random.default_rng(5)
    for ns in (2, 3, 10, 101):
        g1 = 7.5
        vals = rng.uniform(-1, 1, size=(ns, 3))
        w = g1 * rng.choice([-1.0, 1.0], size=ns)
        _, _, cv = estimate(vals, w)
        assert np.all(cv <= ns / (ns - 1) + 1e-12)
    ns = 10
    vals = np.array([[1.0], [-1.0]] * (ns // 2))
    _, _, cv = estimate(vals, np.full(ns, 4.0))
    assert abs(cv[0] - ns / (ns - 1)) < 1e-12


def test_cfg1_estimate_agrees_with_dense_trotter():
    """cfg1 (n=8, chi=16 exact, 200 samples) lands within 4 SE of the Trotter value."""
    p = ti.config(1)
    t = pai.build_table(p)
    vals, signs = [], []
    for s in range(p.n_samples):
        c = sampler.sample_circuit(p, t, s)
        psi = dense.circuit_state(p, t, c)
        vals.append([dense.expectation(psi, o) for o in p.observables])
        signs.append(c.sign)
    w = weights(signs, t.log_g1())
    mean, se, _ = estimate(np.array(vals), w)
    ref = dense.expectation(dense.trotter_state(p), p.observables[0])
    z = abs(mean[0] - ref) / se[0]
    assert z < 4, (mean, ref, se, z)


def test_trotter_error_bound_context():
    """Dense Trotter vs exp(-iHT) within the first-order bound (Statement 4)."""
    p = ti.small_ring(6, seed=1, T=0.5, N=40)
    psi_t = dense.trotter_state(p).reshape(-1)
    psi_e = dense.exact_state(p).reshape(-1)
    # crude bound N * (T/N)^2 / 2 * sum_{a<b} ||[c_a h_a, c_b h_b]|| <= ... use 2|c_a||c_b|
    cs = [abs(t.coeff) for t in p.terms]
    norm_T = sum(2 * cs[a] * sum(cs[a + 1:]) for a in range(len(cs)))
    bound = p.trotter_steps * (p.total_time / p.trotter_steps) ** 2 / 2 * norm_T
    assert np.linalg.norm(psi_t - psi_e) <= bound
