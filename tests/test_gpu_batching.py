"""Per-sample bond caps at the batching workload's shape, against the oracle.

The n = 64 XXZ ring with caps (32, 64, 128) by sample index mod 3: six
samples run in one launch (the library starts them by decreasing cap, so
the launch order is a real permutation here) for 16 Trotter steps, by which
the cap-32 and cap-64 samples cut at their caps.  Both precisions are
checked against one oracle pass: circuits, signs, weights and update counts
exactly, values to 1e-10 in FP64 (near-tie rule) and 1e-4 mixed.  Samples
whose cuts fall among numerically zero singular values are tie-flagged (the
kept state is not unique there); their values are held to the sum of the
two trajectories' truncation bounds instead.
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai
from oracle.run import run_sample
from paper_2604_13144_amd import _lib as L

from test_gpu_parity import gpu_batch, value_tol
from test_gpu_mixed import TOL_MIXED, run_batch

pytestmark = pytest.mark.gpu

STEPS = 16
COUNT = 6


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def check_both_precisions(handle, p, steps, windows):
    """Run p's samples in one FP64 and one mixed batch and compare each with
    one oracle pass; returns the number of samples compared by value."""
    count = p.n_samples
    caps = p.chi_per_sample or (p.chi_max,) * count
    v64, w64, s64 = gpu_batch(handle, p, 0, count, windows)
    vmx, wmx, smx = run_batch(handle, p, count, [steps], L.TEPAI_FP32_MIXED)
    assert np.array_equal(w64, wmx)
    t = pai.build_table(p)
    lg = t.log_g1(steps)
    compared = 0
    for s in range(count):
        r = run_sample(p, t, s, steps)
        for st in (s64, smx):
            assert int(st["n_gates"][s]) == r.n_gates
            assert int(st["sign"][s]) == r.sign
            assert int(st["updates"][s]) == r.stats.updates
            assert int(st["max_bond"][s]) <= caps[s]
        assert w64[s] * r.sign > 0
        assert abs(abs(w64[s]) - math.exp(lg)) <= 1e-14 * math.exp(lg)
        print(f"sample {s} cap {caps[s]}: max bond {max(r.bonds)}, ties {r.stats.ties}, "
              f"min gap {r.stats.min_gap:.2e}", flush=True)
        e64 = float(np.max(np.abs(v64[s] - r.values)))
        emx = float(np.max(np.abs(vmx[s] - r.values)))
        if r.stats.ties:
            # the kept state is not unique, but each trajectory stays within
            # 2 sum_m sqrt(2 eps_m) of the untruncated one (eps_m: weight
            # discarded at update m), so the two differ by at most the sum
            def drift(upd, eps_max):
                return 2.0 * upd * math.sqrt(2.0 * eps_max)
            bound = drift(r.stats.updates, r.stats.max_discarded)
            b64 = bound + drift(int(s64["updates"][s]), float(s64["max_discarded"][s]))
            bmx = bound + drift(int(smx["updates"][s]), float(smx["max_discarded"][s]))
            print(f"  tie-flagged: fp64 err {e64:.2e} (bound {b64:.1e}), "
                  f"mixed err {emx:.2e} (bound {bmx:.1e})", flush=True)
            assert e64 <= 1e-10 + b64, (s, e64, b64)
            assert emx <= TOL_MIXED + bmx, (s, emx, bmx)
            continue
        print(f"  fp64 err {e64:.2e}, mixed err {emx:.2e}", flush=True)
        assert e64 <= value_tol(r, cap=caps[s]), (s, e64)
        assert emx <= TOL_MIXED, (s, emx)
        compared += 1
    return compared


def test_batching_caps_32_64_128(handle):
    p = ti.config(3)
    p = p.with_(n_samples=COUNT, chi_per_sample=p.chi_per_sample[:COUNT])
    assert p.chi_per_sample == (32, 64, 128, 32, 64, 128)
    print("batching: xxz n=64, caps 32/64/128, 16 steps, fp64 and mixed", flush=True)
    assert check_both_precisions(handle, p, STEPS, [STEPS // 2, STEPS // 2]) >= 2
