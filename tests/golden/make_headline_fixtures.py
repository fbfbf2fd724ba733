"""Write the oracle's per-sample results at the benchmark's own regime.

Runs only the CPU oracle (``oracle/``) on seeded synthetic inputs
(``tepai_inputs``) and stores, per sample, what the GPU paths are compared
with in ``tests/test_gpu_headline.py``:

* the n = 64 XXZ ring of the precision configuration (chi = 128, seed 4):
  samples 0-3 after 40 Trotter steps, by which every middle bond of the
  FP64 trajectory sits at the cap of 128 and each update factorises a
  256 x 256 matrix (sec. "Resource model and cost metrics": two-site update,
  SVD, truncation to the chi largest singular values);
* the same ring with per-sample caps 32 / 64 / 128 of the batching
  configuration (seed 3): samples 0-2 after 40 Trotter steps, each cutting
  at its own cap.

Per sample: the observable values (<Z_i> for every i, then <Z_0 Z_32>),
sign, gate count, update and shift counts, sum of chi^3 and the nominal flop
count over all updates (eq. Wsample's cost model), discarded weight, the
near-tie record (smallest gap, ties), the final bonds, and the trajectory's
rounding sensitivity: the largest change of the values when the oracle runs
the sample again with every factorised matrix perturbed by a backward error
of FP64 size (s64) or of FP32 size (s32), and whether the FP64-perturbed run
reproduces the work counts.

Usage: python tests/golden/make_headline_fixtures.py [--jobs 8]
(about ten minutes on seven cores).  Output: tests/golden/headline_xxz_ring_n64.json
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "headline_xxz_ring_n64.json")
LAYERS = 40
CASES = [("precision_chi128", 4, s) for s in range(4)] + [("batching_caps", 3, s) for s in range(3)]


def problem(cfg: int):
    import tepai_inputs as ti
    p = ti.config(cfg)
    if cfg == 3:
        return p.with_(n_samples=3, chi_per_sample=p.chi_per_sample[:3])
    return p.with_(n_samples=4)


def one(case):
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import pai
    from oracle.run import chi_of, run_sample
    name, cfg, s = case
    p = problem(cfg)
    t = pai.build_table(p)
    t0 = time.time()
    r = run_sample(p, t, s, LAYERS)
    # rounding sensitivity: the same sample with every factorised matrix
    # perturbed by a backward error of FP64 size, then of FP32 size (the
    # seeds are those of tests/parity.py)
    rp = run_sample(p, t, s, LAYERS, perturb=(7919 + s, 1.0))
    rq = run_sample(p, t, s, LAYERS, perturb=(104729 + s, 2.0 ** 29))
    st = r.stats
    s64 = float(np.max(np.abs(rp.values - r.values)))
    s32 = float(np.max(np.abs(rq.values - r.values)))
    stable = bool(rp.stats.sum_chi3 == st.sum_chi3 and rp.stats.nominal_flops == st.nominal_flops)
    print(f"{name} sample {s}: {time.time() - t0:.0f} s, updates {st.updates}, "
          f"max bond {max(r.bonds)}, ties {st.ties}, s64 {s64:.1e}, s32 {s32:.1e}", flush=True)
    return {"case": name, "config": cfg, "sample": s, "chi": chi_of(p, s), "layers": LAYERS,
            "values": [float(v) for v in r.values], "sign": int(r.sign),
            "n_gates": int(r.n_gates), "updates": int(st.updates), "shifts": int(st.shifts),
            "sum_chi3": float(st.sum_chi3), "nominal_flops": float(st.nominal_flops),
            "discarded": float(st.discarded), "max_discarded": float(st.max_discarded),
            "min_gap": float(st.min_gap), "ties": int(st.ties),
            "s64": s64, "s32": s32, "work_stable": stable,
            "bonds": [int(b) for b in r.bonds], "log_g1": float(t.log_g1(LAYERS))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    with mp.get_context("spawn").Pool(a.jobs) as pool:
        rows = pool.map(one, CASES)
    doc = {"generator": "tests/golden/make_headline_fixtures.py (oracle only)",
           "workload": "n=64 XXZ ring J_xy=1 J_z=0.5 h~U[-2,2], T=3, N=800, Delta=pi/256, "
                       "Neel start; <Z_i> for all i, <Z_0 Z_32>",
           "svd_cutoff": 1e-12, "samples": rows}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main()
