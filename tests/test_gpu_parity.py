"""HIP MPS path vs the CPU oracle, sample by sample (FP64).

Tolerance: 1e-10 per sample value in FP64, the bar the method's FP64 path is
held to; weights must agree in sign exactly and in magnitude to 1e-14
relative; gate counts, signs and the schedule's update counts must be
identical.  A truncation at the bond cap amplifies rounding by about
1/gap, gap g = (sigma_{k-1} - sigma_k) / sigma_0 at the cut.  The HIP path's
one-sided Jacobi skips a column pair once its off-diagonal product is below
tau * |x||y|, tau = 1e-15 sqrt(R) for R <= 2 chi rows, so the pair of singular
vectors straddling the cut is only fixed to an angle of about tau / (2 g)
(Wedin's sin-theta theorem, with the QR and the projection adding a few units
of u = 2^-53), and an observable of norm 1 moves by at most twice that.  A
sample whose oracle trajectory has a smallest gap g is therefore held to
max(1e-10, (tau + 4u) / g), and a tie-flagged sample (g <= 1e-10: the
truncated state is not unique) is excluded from the value check (its
circuit, sign and weight still are).
"""
import math

import numpy as np
import pytest
import torch

import tepai_inputs as ti
from oracle import pai
from oracle.run import chi_of, run_sample
from oracle.estimator import estimate
from paper_2604_13144_amd import _lib as L

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def gpu_batch(handle, p, first, count, windows):
    """Run samples [first, first+count) through the batch API; returns values, weights, stats."""
    ps = L.ProblemStruct(p)
    dev = torch.device("cuda", 0)
    b = L.Batch(handle, ps, first, count)
    for w in windows:
        b.evolve(w)
    v = torch.empty(count * ps.n_obs, dtype=torch.float64, device=dev)
    w = torch.empty(count, dtype=torch.float64, device=dev)
    b.observe(v, w)
    st = b.stats()
    torch.cuda.synchronize()
    vals = v.cpu().numpy().reshape(count, ps.n_obs)
    return vals, w.cpu().numpy(), st


def compare(p, samples, vals, wts, st, first, layers=None, tol=TOL):
    t = pai.build_table(p)
    lg = t.log_g1(layers)
    worst = 0.0
    for i, s in enumerate(samples):
        r = run_sample(p, t, p.sample_offset + first + i, layers)
        assert int(st["n_gates"][i]) == r.n_gates
        assert int(st["sign"][i]) == r.sign
        assert int(st["updates"][i]) == r.stats.updates
        assert wts[i] * r.sign > 0
        assert abs(abs(wts[i]) - math.exp(lg)) <= 1e-14 * math.exp(lg)
        if r.stats.ties:
            assert int(st["ties"][i]) > 0 or st["min_gap"][i] < 1e-9
            continue
        err = float(np.max(np.abs(vals[i] - r.values)))
        worst = max(worst, err)
        assert err <= value_tol(r, tol, chi_of(p, p.sample_offset + first + i)), \
            (s, err, r.stats.min_gap)
    return worst


U_ROUND = 2.0 ** -53


def value_tol(r, tol=TOL, cap=None):
    """Per-sample bound for oracle result r; cap is the sample's bond cap (the
    matrices factorised have at most 2 cap rows), else its largest final bond."""
    tau = 1e-15 * math.sqrt(2 * (cap if cap is not None else max(r.bonds)))
    return max(tol, (tau + 4.0 * U_ROUND) / r.stats.min_gap)


def test_cfg1_exact_regime(handle):
    p = ti.config(1)
    print("parity: cfg1 n=8 chi=16, 40 samples", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, 40, [p.trotter_steps])
    worst = compare(p, range(40), vals, wts, st, 0)
    print("cfg1 worst per-sample error", worst)


def test_cfg1_full_estimator_via_run(handle):
    p = ti.config(1)
    print("parity: cfg1 tepai_run 200 samples", flush=True)
    out = L.tepai_run(handle, L.ProblemStruct(p))
    mean, se, cv = estimate(out["values"], out["weights"])
    assert np.allclose(out["mean"], mean, rtol=0, atol=1e-13)
    assert np.allclose(out["std_err"], se, rtol=1e-12, atol=0)
    # spot-check a few samples against the oracle
    t = pai.build_table(p)
    for s in (0, 57, 199):
        r = run_sample(p, t, s)
        assert np.max(np.abs(out["values"][s] - r.values)) <= TOL


@pytest.mark.parametrize("chi", [3, 6])
def test_truncated_small_ring(handle, chi):
    p = ti.small_ring(12, seed=11, T=0.4, N=10, delta=math.pi / 16, chi=chi, n_samples=6)
    print(f"parity: ring n=12 chi={chi}", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, 6, [p.trotter_steps])
    assert max(st["max_bond"]) <= chi
    worst = compare(p, range(6), vals, wts, st, 0)
    print("truncated worst", worst)


def test_several_tiles_and_ragged_columns(handle):
    # chi = 40: two-site matrices up to 80 x 80 (2 x 64 rows per lane span, ragged)
    p = ti.small_ring(14, seed=5, T=0.6, N=12, delta=math.pi / 24, chi=40, n_samples=3,
                      j_z=0.7)
    print("parity: ring n=14 chi=40", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, 3, [5, 7])
    assert max(st["max_bond"]) > 32
    compare(p, range(3), vals, wts, st, 0)


def test_metric_shape_prefix(handle):
    # the n=64 XXZ ring of the benchmark at chi=128, first 3 Trotter steps
    p = ti.config(4).with_(n_samples=4)
    print("parity: xxz n=64 chi=128 prefix 3 steps", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, 4, [1, 2])
    compare(p, range(4), vals, wts, st, 0, layers=3)


def test_windows_equal_single_launch_and_determinism(handle):
    p = ti.small_ring(10, seed=2, T=0.5, N=12, delta=math.pi / 16, chi=8, n_samples=4)
    a = gpu_batch(handle, p, 0, 4, [12])
    b = gpu_batch(handle, p, 0, 4, [3, 4, 5])
    c = gpu_batch(handle, p, 0, 4, [12])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0])


def test_edge_cases(handle):
    # two-qubit open chain: one bond, runs on a single pair
    terms = (ti.Term("XX", (0, 1), 0.9), ti.Term("ZZ", (0, 1), 0.4), ti.Term("Z", (1,), 0.3))
    p = ti.Problem(n_qubits=2, terms=terms, total_time=1.0, trotter_steps=30,
                   delta=math.pi / 8, n_samples=5, seed=9, chi_max=2, initial_bits="10",
                   observables=((ti.PauliString("Z", (0,)),), (ti.PauliString("XY", (0, 1)),)))
    vals, wts, st = gpu_batch(handle, p, 0, 5, [30])
    compare(p, range(5), vals, wts, st, 0)
    # chi = 1: every update truncates to a product state
    p1 = ti.small_ring(6, seed=3, T=0.3, N=6, delta=math.pi / 16, chi=1, n_samples=3)
    vals, wts, st = gpu_batch(handle, p1, 0, 3, [6])
    assert max(st["max_bond"]) == 1
    compare(p1, range(3), vals, wts, st, 0)
    # a single sample: the standard error is undefined
    out = L.tepai_run(handle, L.ProblemStruct(p.with_(n_samples=1)))
    assert np.all(np.isnan(out["std_err"]))


def test_no_pi_variant(handle):
    # biased variant without pi rotations: weights exactly 1, same MPS path
    p = ti.small_ring(10, seed=4, T=0.5, N=12, delta=math.pi / 16, chi=8, n_samples=6)
    p = p.with_(no_pi=True)
    print("parity: no-pi ring n=10 chi=8", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, 6, [5, 7])
    assert np.all(wts == 1.0) and np.all(st["sign"] == 1)
    compare(p, range(6), vals, wts, st, 0)


def test_heterogeneous_chi_per_sample(handle):
    p = ti.small_ring(10, seed=7, T=0.4, N=10, delta=math.pi / 16, chi=8, n_samples=6)
    p = p.with_(chi_per_sample=(2, 4, 8, 3, 8, 5))
    vals, wts, st = gpu_batch(handle, p, 0, 6, [10])
    assert all(int(m) <= c for m, c in zip(st["max_bond"], p.chi_per_sample))
    t = pai.build_table(p)
    for i in range(6):
        r = run_sample(p, t, i)
        if not r.stats.ties:
            assert np.max(np.abs(vals[i] - r.values)) <= value_tol(r, cap=p.chi_per_sample[i])


def test_time_series_checkpoints(handle):
    # one batch read out after 4, 8 and 12 Trotter steps: each read-out is the
    # TE-PAI estimate at time jT/N (prefix samples, weight sign_j ||g||_1(j))
    p = ti.small_ring(10, seed=8, T=0.6, N=12, delta=math.pi / 16, chi=8, n_samples=5)
    ps = L.ProblemStruct(p)
    dev = torch.device("cuda", 0)
    b = L.Batch(handle, ps, 0, 5)
    v = torch.empty(5 * ps.n_obs, dtype=torch.float64, device=dev)
    w = torch.empty(5, dtype=torch.float64, device=dev)
    mean = torch.empty(ps.n_obs, dtype=torch.float64, device=dev)
    se = torch.empty(ps.n_obs, dtype=torch.float64, device=dev)
    t = pai.build_table(p)
    for j in (4, 8, 12):
        b.evolve(4)
        b.observe(v, w)
        L.tepai_reduce(handle, 5, ps.n_obs, v, w, mean, se)
        torch.cuda.synchronize()
        vals = v.cpu().numpy().reshape(5, ps.n_obs)
        res = [run_sample(p, t, s, j) for s in range(5)]
        for s, r in enumerate(res):
            assert float(w[s]) * r.sign > 0
            assert abs(abs(float(w[s])) - math.exp(t.log_g1(j))) <= 1e-14 * math.exp(t.log_g1(j))
            if not r.stats.ties:
                assert np.max(np.abs(vals[s] - r.values)) <= value_tol(r, cap=p.chi_max)
        ws = np.array([r.sign * math.exp(t.log_g1(j)) for r in res])
        m, _, _ = estimate(np.array([r.values for r in res]), ws)
        assert np.max(np.abs(mean.cpu().numpy() - m)) <= 1e-9
