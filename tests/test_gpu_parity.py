"""HIP MPS path vs the CPU oracle, sample by sample (FP64).

The bars are those of ``tests/parity.py``: circuits, signs and counts
identical (sum of chi^3 and nominal flops too), weights to 1e-14 relative,
values to 1e-10 plus the oracle trajectory's near-tie bound; samples with a
tie (a cap cut whose own bound exceeds 1e-10) are left out of the value
check.
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

import parity

pytestmark = pytest.mark.gpu

TOL = parity.TOL


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


def compare(p, samples, vals, wts, st, first, layers=None):
    """Every slot against the oracle with the FP64 bars; returns the worst
    value error (and prints how many samples were held to 1e-10 outright)."""
    t = pai.build_table(p)
    lg = t.log_g1(layers)
    worst, strict = 0.0, 0
    for i, s in enumerate(samples):
        o = parity.OracleSample(p, t, p.sample_offset + first + i, layers)
        parity.check_counts(st, i, o)
        parity.check_weight(wts[i], o, lg)
        strict += parity.fp64_value_ok(vals[i], o, f"sample {s}: ")
        worst = max(worst, float(np.max(np.abs(vals[i] - o.r.values))))
    print(f"  {strict} of {len(samples)} samples held to 1e-10 outright, worst {worst:.1e}",
          flush=True)
    return worst


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
        assert parity.fp64_value_ok(out["values"][s], parity.OracleSample(p, t, s), f"sample {s}: ")


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
    compare(p, range(6), vals, wts, st, 0)


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
        res = [parity.OracleSample(p, t, s, j) for s in range(5)]
        for s, o in enumerate(res):
            parity.check_weight(float(w[s]), o, t.log_g1(j))
            parity.fp64_value_ok(vals[s], o, f"step {j} sample {s}: ")
        ws = np.array([o.r.sign * math.exp(t.log_g1(j)) for o in res])
        m, _, _ = estimate(np.array([o.r.values for o in res]), ws)
        assert np.max(np.abs(mean.cpu().numpy() - m)) <= 1e-9


@pytest.mark.parametrize("precision", [L.TEPAI_FP64, L.TEPAI_FP32_MIXED])
def test_per_gate_mode(handle, precision):
    # TEPAI_PER_GATE: one truncated update per sampled two-qubit gate, on a
    # truncated ring (chi = 4) whose runs of same-pair gates would otherwise fuse
    p = ti.small_ring(10, seed=12, T=0.5, N=10, delta=math.pi / 16, chi=4, n_samples=5)
    p = p.with_(per_gate=True)
    print(f"parity: per-gate ring n=10 chi=4, precision {precision}", flush=True)
    ps = L.ProblemStruct(p, precision=precision)
    dev = torch.device("cuda", 0)
    b = L.Batch(handle, ps, 0, 5)
    b.evolve(4)
    b.evolve(6)
    v = torch.empty(5 * ps.n_obs, dtype=torch.float64, device=dev)
    w = torch.empty(5, dtype=torch.float64, device=dev)
    b.observe(v, w)
    st = b.stats()
    torch.cuda.synchronize()
    vals = v.cpu().numpy().reshape(5, ps.n_obs)
    t = pai.build_table(p)
    fused = L.tepai_run(handle, L.ProblemStruct(p.with_(per_gate=False), precision=precision))
    assert np.all(st["updates"] > fused["stats"]["updates"])
    for i in range(5):
        o = parity.OracleSample(p, t, i, mixed=precision == L.TEPAI_FP32_MIXED,
                                fp64=precision == L.TEPAI_FP64)
        parity.check_counts(st, i, o, fp64=precision == L.TEPAI_FP64)
        if precision == L.TEPAI_FP64:
            parity.fp64_value_ok(vals[i], o, f"sample {i}: ")
        else:
            parity.mixed_value_ok(vals[i], o, f"sample {i}: ")
