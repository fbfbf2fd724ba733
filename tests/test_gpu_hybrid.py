"""Hybrid start on the GPU: every sample begins from a shared Trotter MPS.

The shared state is the oracle's deterministic Trotter evolution (same
schedule, routing and truncation as the samples); the TE-PAI segment then
runs on the GPU and is compared per sample with the oracle (FP64: 1e-10 with
the gap rule; mixed: 1e-4).
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle.trotter import trotter_initial_mps
from paper_2604_13144_amd import _lib as L

from test_gpu_parity import compare, gpu_batch
from test_gpu_mixed import TOL_MIXED, against_oracle, run_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def hybrid_problem(n=12, chi=10, N0=10, T0=0.8, seed=9, ns=5):
    pre = ti.small_ring(n, seed=seed, T=T0, N=N0, delta=math.pi / 16, chi=chi, n_samples=1)
    init = trotter_initial_mps(pre, N0, chi)
    return pre.with_(total_time=0.3, trotter_steps=6, n_samples=ns, initial_mps=init), init


def test_hybrid_fp64(handle):
    p, init = hybrid_problem()
    assert max(init.bonds()) == 10 and init.qubit_at != tuple(range(12))
    print("hybrid fp64: ring n=12 chi=10 from a 10-step Trotter state", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, p.n_samples, [2, 4])
    assert max(st["max_bond"]) == 10
    compare(p, range(p.n_samples), vals, wts, st, 0)


def test_hybrid_mixed(handle):
    p, _ = hybrid_problem(seed=10)
    print("hybrid mixed: ring n=12 chi=10", flush=True)
    vals, _, st = run_batch(handle, p, p.n_samples, [6], L.TEPAI_FP32_MIXED)
    print("hybrid mixed worst", against_oracle(p, vals, st))
