"""Deterministic product formula on the GPU (TEPAI_TROTTER), the comparison
circuit of sec. "Truncation": per-value parity with the oracle (FP64 1e-10
with the gap rule, mixed 1e-4), weights exactly 1, every rotation present;
then both methods at the experiment's own shape (n = 20 ring, chi = 2 and
16) over a prefix of its 2000 steps.
"""
import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai
from paper_2604_13144_amd import _lib as L

from test_gpu_parity import compare, gpu_batch
from test_gpu_mixed import against_oracle, run_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def trotter_small(n=10, N=20, chi=4, T=0.5, ns=2):
    return ti.truncation_workload(chi, trotter=True, n=n, T=T, trotter_steps=N).with_(n_samples=ns)


@pytest.mark.parametrize("chi", [2, 4, 32])
def test_trotter_fp64(handle, chi):
    p = trotter_small(chi=chi)
    L_eff = pai.build_table(p).l_eff
    print(f"trotter fp64: ring n=10 chi={chi} N=20 from |+..-..+>", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, p.n_samples, [7, 13])
    assert np.all(wts == 1.0) and np.all(st["sign"] == 1)
    assert np.all(st["n_gates"] == p.trotter_steps * L_eff)
    assert np.array_equal(vals[0], vals[1])                  # one deterministic circuit
    assert max(st["max_bond"]) <= chi
    compare(p, range(p.n_samples), vals, wts, st, 0)


def test_trotter_sampler_keeps_every_rotation(handle):
    p = trotter_small()
    L_eff = pai.build_table(p).l_eff
    off, words, signs = L.tepai_sample_circuits(handle, L.ProblemStruct(p), 0, 2, 5)
    w = words.astype(np.uint64)
    for i in range(2):
        seg = w[off[i]:off[i + 1]]
        assert np.array_equal(seg >> np.uint64(2), np.arange(5 * L_eff, dtype=np.uint64))
        assert np.all((seg & np.uint64(3)) == 1)          # TEPAI_SET_B: the exact rotation
    assert np.all(signs == 1)


def test_trotter_mixed(handle):
    p = trotter_small(chi=6)
    print("trotter mixed: ring n=10 chi=6", flush=True)
    vals, _, st = run_batch(handle, p, p.n_samples, [p.trotter_steps], L.TEPAI_FP32_MIXED)
    print("trotter mixed worst", against_oracle(p, vals, st))


@pytest.mark.parametrize("chi", [2, 16])
@pytest.mark.parametrize("trotter", [True, False])
def test_truncation_workload_prefix(handle, chi, trotter):
    # the experiment's n = 20 ring at its real step size, first 30 of 2000 steps
    p = ti.truncation_workload(chi, trotter=trotter)
    p = p.with_(n_samples=1 if trotter else 3)
    print(f"truncation workload prefix: trotter={trotter} chi={chi} 30 steps", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, p.n_samples, [10, 20])
    assert max(st["max_bond"]) <= chi
    compare(p, range(p.n_samples), vals, wts, st, 0, layers=30)


@pytest.mark.parametrize("trotter", [True, False])
def test_truncation_workload_prefix_per_gate(handle, trotter):
    # the same experiment with one truncated update per gate (TEPAI_PER_GATE)
    p = ti.truncation_workload(2, trotter=trotter, per_gate=True)
    p = p.with_(n_samples=1 if trotter else 3)
    print(f"truncation workload prefix, per gate: trotter={trotter} chi=2 30 steps", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, p.n_samples, [10, 20])
    compare(p, range(p.n_samples), vals, wts, st, 0, layers=30)


def test_truncation_workload_full_length_chi2(handle):
    # all 2000 steps of the experiment at chi = 2 (77.9k truncated updates per
    # circuit): the product formula and two TE-PAI circuits against the oracle
    # (a sample with a tie at a cut is checked for its counts and flag only)
    for trotter, ns in ((True, 1), (False, 2)):
        p = ti.truncation_workload(2, trotter=trotter).with_(n_samples=ns)
        print(f"truncation workload full length: trotter={trotter} chi=2", flush=True)
        vals, wts, st = gpu_batch(handle, p, 0, ns, [p.trotter_steps])
        assert int(st["updates"][0]) > 70_000
        compare(p, range(ns), vals, wts, st, 0)
