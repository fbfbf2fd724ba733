"""The largest bond cap (chi = 256) on the GPU against the oracle.

A seeded random MPS on an n = 18 ring starts with its three middle bonds at
256, so the first two-site updates factorise 512 x 512 matrices (the widest
row class of the kernels) and truncate back to 256; one Trotter step of the
disordered Heisenberg ring then runs through the bond-cap cuts, the
wrap-bond routing and the read-out at that size.  FP64 values are held to
the near-tie rule of the FP64 parity tests, the mixed path to 1e-4.
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from paper_2604_13144_amd import _lib as L

from test_gpu_parity import compare, gpu_batch
from test_gpu_mixed import against_oracle, run_batch

pytestmark = pytest.mark.gpu

N_SAMPLES = 3


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def chi256_problem(seed):
    p = ti.small_ring(18, seed=seed, T=0.05, N=1, delta=math.pi / 16, chi=256,
                      n_samples=N_SAMPLES)
    return p.with_(initial_mps=ti.random_mps(18, 256, seed=3))


def test_chi256_fp64(handle):
    p = chi256_problem(21)
    print("chi256 fp64: ring n=18 from a random chi=256 MPS", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, N_SAMPLES, [1])
    assert max(st["max_bond"]) == 256
    assert int(np.max(st["nonconverged"])) == 0
    print("chi256 fp64 worst", compare(p, range(N_SAMPLES), vals, wts, st, 0), flush=True)


def test_chi256_mixed(handle):
    p = chi256_problem(22)
    print("chi256 mixed: ring n=18 from a random chi=256 MPS", flush=True)
    vals, _, st = run_batch(handle, p, N_SAMPLES, [1], L.TEPAI_FP32_MIXED)
    assert max(st["max_bond"]) == 256
    print("chi256 mixed worst", against_oracle(p, vals, st), flush=True)
