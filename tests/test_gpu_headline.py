"""Both GPU paths against stored oracle results at the benchmark's own regime.

``tests/golden/headline_xxz_ring_n64.json`` holds what the CPU oracle (and
only the oracle: ``tests/golden/make_headline_fixtures.py``) computes for
the n = 64 XXZ ring after 40 Trotter steps: samples 0-3 at bond cap 128
(every middle bond at the cap, 256 x 256 factorisations, the regime the
throughput metric is quoted on) and samples 0-2 of the per-sample caps
32 / 64 / 128.  The GPU runs the same samples through the batch API and is
held to the bars of ``tests/parity.py``: FP64 counts identical (gates,
updates, shifts, sum of chi^3, nominal flops), values within 1e-10 plus ten
times the stored rounding sensitivity of the sample's trajectory; mixed
values within 1e-4 plus ten times its FP32-sized sensitivity.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import tepai_inputs as ti
from paper_2604_13144_amd import _lib as L

import parity

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "headline_xxz_ring_n64.json")


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def fixture_cases(name):
    doc = json.load(open(FIXTURE))
    return [r for r in doc["samples"] if r["case"] == name]


def problem(cfg, count):
    p = ti.config(cfg)
    if cfg == 3:
        return p.with_(n_samples=count, chi_per_sample=p.chi_per_sample[:count])
    return p.with_(n_samples=count)


class Ref:
    """An oracle sample (parity.OracleSample's fields) rebuilt from the stored record."""

    def __init__(self, d):
        self.r = type("R", (), {})()
        self.r.values = np.array(d["values"])
        self.r.sign = d["sign"]
        self.r.n_gates = d["n_gates"]
        self.r.stats = type("S", (), {})()
        for k in ("updates", "shifts", "sum_chi3", "nominal_flops", "ties", "min_gap"):
            setattr(self.r.stats, k, d[k])
        self.s64, self.s32, self.stable = d["s64"], d["s32"], d["work_stable"]


def run(handle, p, count, layers, precision):
    ps = L.ProblemStruct(p, precision=precision)
    dev = torch.device("cuda", 0)
    b = L.Batch(handle, ps, 0, count)
    for _ in range(layers // 20):
        b.evolve(20)
    b.evolve(layers % 20)
    v = torch.empty(count * ps.n_obs, dtype=torch.float64, device=dev)
    w = torch.empty(count, dtype=torch.float64, device=dev)
    b.observe(v, w)
    st = b.stats()
    torch.cuda.synchronize()
    return v.cpu().numpy().reshape(count, ps.n_obs), w.cpu().numpy(), st


@pytest.mark.parametrize("name,cfg", [("precision_chi128", 4), ("batching_caps", 3)])
def test_headline_regime_against_stored_oracle(handle, name, cfg):
    cases = fixture_cases(name)
    count = len(cases)
    assert [c["sample"] for c in cases] == list(range(count))
    layers = cases[0]["layers"]
    p = problem(cfg, count)
    print(f"headline: {name}, {count} samples, {layers} steps, fp64 then mixed", flush=True)
    v64, w64, s64 = run(handle, p, count, layers, L.TEPAI_FP64)
    vmx, wmx, smx = run(handle, p, count, layers, L.TEPAI_FP32_MIXED)
    assert np.array_equal(w64, wmx)
    strict = 0
    for i, d in enumerate(cases):
        o = Ref(d)
        parity.check_counts(s64, i, o)
        parity.check_counts(smx, i, o, fp64=False)
        parity.check_weight(w64[i], o, d["log_g1"])
        assert max(d["bonds"]) <= int(s64["max_bond"][i]) <= d["chi"]
        emx = parity.mixed_value_ok(vmx[i], o, f"mixed sample {i}: ")
        ok = parity.fp64_value_ok(v64[i], o, f"fp64 sample {i}: ")
        strict += ok
        print(f"  sample {i} cap {d['chi']}: max bond {max(d['bonds'])}, fp64 err "
              f"{float(np.max(np.abs(v64[i] - o.r.values))):.2e} (s64 {d['s64']:.1e}), "
              f"mixed err {emx:.2e} (s32 {d['s32']:.1e}), ties oracle/gpu "
              f"{d['ties']}/{int(s64['ties'][i])}, sum chi^3 {d['sum_chi3']:.4e}", flush=True)
    assert strict >= 1
