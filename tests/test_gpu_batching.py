"""Per-sample bond caps at the batching workload's shape, against the oracle.

The n = 64 XXZ ring with caps (32, 64, 128) by sample index mod 3: six
samples run in one launch (the library starts them by decreasing cap, so
the launch order is a real permutation here) for 16 Trotter steps, by which
the cap-32 and cap-64 samples cut at their caps.  Both precisions are
checked against one oracle pass with the bars of ``tests/parity.py``.
"""
import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai
from oracle.run import run_sample
from paper_2604_13144_amd import _lib as L

import parity
from test_gpu_parity import gpu_batch
from test_gpu_mixed import run_batch

pytestmark = pytest.mark.gpu

STEPS = 16
COUNT = 6


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def check_both_precisions(handle, p, steps, windows):
    """Run p's samples in one FP64 and one mixed batch and compare each with
    the oracle; returns the number of samples held to 1e-10 outright."""
    count = p.n_samples
    caps = p.chi_per_sample or (p.chi_max,) * count
    v64, w64, s64 = gpu_batch(handle, p, 0, count, windows)
    vmx, wmx, smx = run_batch(handle, p, count, [steps], L.TEPAI_FP32_MIXED)
    assert np.array_equal(w64, wmx)
    t = pai.build_table(p)
    lg = t.log_g1(steps)
    strict = 0
    for s in range(count):
        o = parity.OracleSample(p, t, s, steps, mixed=True)
        r = o.r
        parity.check_counts(s64, s, o)
        parity.check_counts(smx, s, o, fp64=False)
        for st in (s64, smx):
            assert int(st["max_bond"][s]) <= caps[s]
        parity.check_weight(w64[s], o, lg)
        print(f"sample {s} cap {caps[s]}: max bond {max(r.bonds)}, ties {r.stats.ties}, "
              f"s64 {o.s64:.1e}, s32 {o.s32:.1e}, min gap {r.stats.min_gap:.2e}", flush=True)
        emx = parity.mixed_value_ok(vmx[s], o, f"mixed sample {s}: ")
        strict += parity.fp64_value_ok(v64[s], o, f"fp64 sample {s}: ")
        print(f"  fp64 err {float(np.max(np.abs(v64[s] - r.values))):.2e}, mixed err {emx:.2e}",
              flush=True)
    return strict


def test_batching_caps_32_64_128(handle):
    p = ti.config(3)
    p = p.with_(n_samples=COUNT, chi_per_sample=p.chi_per_sample[:COUNT])
    assert p.chi_per_sample == (32, 64, 128, 32, 64, 128)
    print("batching: xxz n=64, caps 32/64/128, 16 steps, fp64 and mixed", flush=True)
    assert check_both_precisions(handle, p, STEPS, [STEPS // 2, STEPS // 2]) >= 1
