"""The other benchmark configurations' shapes on the GPU, against the oracle.

* The plain batched FP64 configuration: the n = 32 disordered Heisenberg
  ring at chi = 64 (Neel start, <Z_i> for all i and <Z_0 Z_16>), its first
  24 Trotter steps, by which every sample cuts at the cap.
* The combined long-time configuration: the n = 100 Heisenberg ring, a
  10-step product-formula state at cap 16 (prepared by the oracle) shared by
  TE-PAI samples with caps 64, 32 and 16, their first 3 Trotter steps of the
  N = 1024, Delta = pi/512 segment, <Z_i> for all i and the half-ring sum of
  Z_i Z_{i+1}.

Both precisions are compared with one oracle pass per sample with the bars
of ``tests/parity.py``; every test checks at least one sample by value.
"""
import pytest

import tepai_inputs as ti
from oracle.trotter import trotter_initial_mps
from paper_2604_13144_amd import _lib as L

from test_gpu_batching import check_both_precisions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def test_plain_batched_ring_n32_chi64_prefix(handle):
    p = ti.config(2).with_(n_samples=3)
    print("config shape: heisenberg n=32 chi=64, 24 steps", flush=True)
    assert check_both_precisions(handle, p, 24, [10, 14]) >= 1


def test_long_time_ring_n100_shared_start_prefix(handle):
    p5 = ti.config(5)
    pre = p5.with_(total_time=0.05, trotter_steps=10, chi_max=16, n_samples=1)
    init = trotter_initial_mps(pre, 10, 16)
    assert max(init.bonds()) == 16
    p = p5.with_(n_samples=3, chi_per_sample=(64, 32, 16), initial_mps=init)
    print("config shape: heisenberg n=100 from a shared Trotter state, caps 64/32/16, 3 steps",
          flush=True)
    assert check_both_precisions(handle, p, 3, [1, 2]) >= 1
