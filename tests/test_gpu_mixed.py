"""Mixed-precision path (TEPAI_FP32_MIXED) vs the FP64 oracle and the FP64 path.

The mixed path stores site tensors as complex64 and runs the contractions on
FP32 matrix cores; the QR, Jacobi, truncation, renormalisation, weights and
the estimator stay FP64.  Bar: 1e-4 per sample value against the oracle
plus ten times the trajectory's sensitivity to FP32-sized rounding
(``tests/parity.py``); weights and sampled circuits identical to the FP64
path.
"""
import math

import numpy as np
import pytest
import torch

import tepai_inputs as ti
from oracle import pai
from oracle.run import run_sample
from paper_2604_13144_amd import _lib as L

import parity

pytestmark = pytest.mark.gpu

TOL_MIXED = parity.TOL_MIXED


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def run_batch(handle, p, count, windows, precision):
    ps = L.ProblemStruct(p, precision=precision)
    dev = torch.device("cuda", 0)
    b = L.Batch(handle, ps, 0, count)
    for w in windows:
        b.evolve(w)
    v = torch.empty(count * ps.n_obs, dtype=torch.float64, device=dev)
    w = torch.empty(count, dtype=torch.float64, device=dev)
    b.observe(v, w)
    st = b.stats()
    torch.cuda.synchronize()
    return v.cpu().numpy().reshape(count, ps.n_obs), w.cpu().numpy(), st


def against_oracle(p, vals, st, layers=None):
    t = pai.build_table(p)
    worst = 0.0
    for i in range(vals.shape[0]):
        o = parity.OracleSample(p, t, i, layers, mixed=True, fp64=False)
        parity.check_counts(st, i, o, fp64=False)
        worst = max(worst, parity.mixed_value_ok(vals[i], o, f"sample {i}: "))
    return worst


def test_mixed_cfg1_exact_regime(handle):
    p = ti.config(1)
    print("mixed: cfg1 n=8 chi=16, 40 samples", flush=True)
    vals, wts, st = run_batch(handle, p, 40, [p.trotter_steps], L.TEPAI_FP32_MIXED)
    _, w64, _ = run_batch(handle, p, 40, [p.trotter_steps], L.TEPAI_FP64)
    assert np.array_equal(wts, w64)
    print("mixed cfg1 worst", against_oracle(p, vals, st))


@pytest.mark.parametrize("chi", [3, 6])
def test_mixed_truncated_small_ring(handle, chi):
    p = ti.small_ring(12, seed=11, T=0.4, N=10, delta=math.pi / 16, chi=chi, n_samples=6)
    print(f"mixed: ring n=12 chi={chi}", flush=True)
    vals, _, st = run_batch(handle, p, 6, [p.trotter_steps], L.TEPAI_FP32_MIXED)
    assert max(st["max_bond"]) <= chi
    print("mixed truncated worst", against_oracle(p, vals, st))


def test_mixed_several_tiles(handle):
    p = ti.small_ring(14, seed=5, T=0.6, N=12, delta=math.pi / 24, chi=40, n_samples=3, j_z=0.7)
    print("mixed: ring n=14 chi=40", flush=True)
    vals, _, st = run_batch(handle, p, 3, [5, 7], L.TEPAI_FP32_MIXED)
    print("mixed tiles worst", against_oracle(p, vals, st))


def test_mixed_metric_shape_prefix(handle):
    p = ti.config(4).with_(n_samples=4)
    print("mixed: xxz n=64 chi=128 prefix 3 steps", flush=True)
    vals, _, st = run_batch(handle, p, 4, [1, 2], L.TEPAI_FP32_MIXED)
    print("mixed prefix worst", against_oracle(p, vals, st, layers=3))


def test_mixed_matches_fp64_path_at_saturation(handle):
    # the benchmark workload past the point where the bond reaches chi = 128:
    # the FP64 path stands in for the oracle (it matches it to 1e-10)
    p = ti.config(4).with_(n_samples=4)
    print("mixed vs fp64: xxz n=64 chi=128, 32 steps", flush=True)
    vm, wm, sm = run_batch(handle, p, 4, [16, 16], L.TEPAI_FP32_MIXED)
    vd, wd, sd = run_batch(handle, p, 4, [16, 16], L.TEPAI_FP64)
    assert np.array_equal(wm, wd)
    assert np.array_equal(sm["n_gates"], sd["n_gates"])
    assert max(sd["max_bond"]) == 128
    err = float(np.max(np.abs(vm - vd)))
    print("mixed vs fp64 worst", err, "sweeps/factorisation",
          sm["jacobi_sweeps"].sum() / (sm["updates"].sum() + sm["shifts"].sum()),
          sd["jacobi_sweeps"].sum() / (sd["updates"].sum() + sd["shifts"].sum()))
    assert err <= TOL_MIXED


def test_mixed_estimator_agrees_with_fp64(handle):
    p = ti.config(1)
    o64 = L.tepai_run(handle, L.ProblemStruct(p))
    o32 = L.tepai_run(handle, L.ProblemStruct(p, precision=L.TEPAI_FP32_MIXED))
    assert np.array_equal(o64["weights"], o32["weights"])
    assert np.max(np.abs(o64["mean"] - o32["mean"])) <= TOL_MIXED
