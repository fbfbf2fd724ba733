"""Failure handling on the GPU, forced from the host (every kernel exits normally).

* A shared starting state with a non-finite entry in its orthogonality
  centre: every sample meets a NaN at its first factorisation.  The kernels order columns with NaN-safe keys,
  so the run completes; each sample's TEPAI_SAMPLE_NONFINITE flag is set,
  tepai_run returns TEPAI_ENUMERIC and still writes every output, and the
  oracle flags the same samples.
* tepai_sample_circuits with a gate capacity but no gate buffer is rejected
  before any device work.
"""
import ctypes as C
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai
from oracle.mps import NONFINITE
from oracle.run import run_sample
from oracle.trotter import trotter_initial_mps
from paper_2604_13144_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


@pytest.mark.parametrize("precision", [L.TEPAI_FP64, L.TEPAI_FP32_MIXED])
def test_nonfinite_start_is_flagged_not_fatal(handle, precision):
    pre = ti.small_ring(6, seed=3, T=0.4, N=6, chi=4, n_samples=1)
    init = trotter_initial_mps(pre, 6, 4)
    # NaN in the orthogonality centre: the first factorisation (a shift or an
    # update, both include the centre) meets it, and the read-out divides by
    # the centre's norm
    bad = [a.copy() for a in init.tensors]
    bad[init.centre][0, 1, 0] = np.nan
    p = pre.with_(n_samples=4, trotter_steps=3, total_time=0.2,
                  initial_mps=ti.InitialMPS(tuple(bad), init.centre, init.qubit_at))
    print(f"failure: NaN in the shared start, precision {precision}", flush=True)
    with pytest.raises(L.TepaiError) as e:
        L.tepai_run(handle, L.ProblemStruct(p, precision=precision))
    assert e.value.status == L.TEPAI_ENUMERIC
    out = e.value.result
    assert np.all(out["stats"]["flags"] & L.TEPAI_SAMPLE_NONFINITE)
    assert np.all(np.isnan(out["values"]))
    assert np.all(np.abs(out["weights"]) > 0)          # weights do not depend on the state
    t = pai.build_table(p)
    r = run_sample(p, t, 0)
    assert r.stats.flags & NONFINITE and np.all(np.isnan(r.values))
    # the handle stays usable: a clean problem runs normally afterwards
    ok = L.tepai_run(handle, L.ProblemStruct(pre.with_(n_samples=2), precision=precision))
    assert np.all(ok["stats"]["flags"] == 0) and np.all(np.isfinite(ok["mean"]))


def test_sample_circuits_rejects_missing_gate_buffer(handle):
    p = ti.config(1).with_(n_samples=2)
    ps = L.ProblemStruct(p)
    offsets = np.zeros(3, np.uint64)
    signs = np.zeros(2, np.int8)
    st = L.load().tepai_sample_circuits(handle.h, ps.ref(), 0, 2, 0, 1000,
                                        offsets.ctypes.data_as(C.c_void_p), None,
                                        signs.ctypes.data_as(C.c_void_p))
    assert st == -1
