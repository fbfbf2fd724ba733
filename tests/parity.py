"""Shared parity rules of the GPU tests (imported by tests/test_gpu_*.py).

Bars (per sample, per observable, against the CPU oracle on the same seeded
inputs):

* circuits, signs, gate, update and shift counts: identical;
* weights: sign identical, magnitude within 1e-14 relative;
* FP64 values: within 1e-10 plus ten times the sample's rounding
  sensitivity s64, the largest change of its values when the oracle runs
  the sample again with every factorised matrix perturbed by a random
  backward error of FP64 size (u sqrt(R C) |M|, ``oracle.mps.MPS``).  Near
  ties at bond-cap cuts make some truncated trajectories sensitive (a cut
  between nearly equal singular values lets rounding pick the kept vector,
  and later cuts amplify earlier rounding differences by sigma_{k-1} / gap);
  two FP64 computations of such a sample legitimately differ by about s64.
  A sample with s64 <= 1e-11 is held to 1e-10 outright ("strict");
* FP64 sum of chi^3 and nominal flop count: identical whenever the perturbed
  oracle run reproduces them (the bond dimensions are then fixed by the
  trajectory, not by rounding);
* mixed-path values: within 1e-4 plus ten times the sensitivity s32 to a
  perturbation of FP32 size (2^29 times larger).
"""
import math

import numpy as np

from oracle.run import run_sample

TOL = 1e-10
TOL_MIXED = 1e-4
SENS_FACTOR = 10.0
STRICT_SENS = 1e-11
FP32_SCALE = 2.0 ** 29        # 2^-24 / 2^-53


class OracleSample:
    """The oracle's result for one sample plus its rounding sensitivity."""

    def __init__(self, p, t, s, layers=None, mixed=False, fp64=True):
        self.p = p
        self.r = run_sample(p, t, s, layers)
        self.s64, self.stable = 0.0, True
        if fp64:
            rp = run_sample(p, t, s, layers, perturb=(7919 + s, 1.0))
            self.s64 = float(np.max(np.abs(rp.values - self.r.values)))
            self.stable = (rp.stats.sum_chi3 == self.r.stats.sum_chi3
                           and rp.stats.nominal_flops == self.r.stats.nominal_flops)
        self.s32 = None
        if mixed:
            rq = run_sample(p, t, s, layers, perturb=(104729 + s, FP32_SCALE))
            self.s32 = float(np.max(np.abs(rq.values - self.r.values)))


def check_counts(st, i, o, fp64=True):
    """GPU counters of slot i against oracle sample o."""
    r = o.r
    assert int(st["n_gates"][i]) == r.n_gates
    assert int(st["sign"][i]) == r.sign
    assert int(st["updates"][i]) == r.stats.updates, (i, int(st["updates"][i]), r.stats.updates)
    assert int(st["shifts"][i]) == r.stats.shifts, (i, int(st["shifts"][i]), r.stats.shifts)
    if fp64 and o.stable:
        assert math.isclose(float(st["sum_chi3"][i]), r.stats.sum_chi3, rel_tol=1e-12, abs_tol=0.0), \
            (i, float(st["sum_chi3"][i]), r.stats.sum_chi3)
        assert math.isclose(float(st["nominal_flops"][i]), r.stats.nominal_flops,
                            rel_tol=1e-12, abs_tol=0.0), \
            (i, float(st["nominal_flops"][i]), r.stats.nominal_flops)


def check_weight(w, o, log_g1):
    assert w * o.r.sign > 0
    assert abs(abs(w) - math.exp(log_g1)) <= 1e-14 * math.exp(log_g1)


def fp64_value_ok(vals, o, label=""):
    """Asserts the FP64 bar; returns True when the sample was held to 1e-10
    outright (its trajectory is not sensitive to rounding)."""
    tol = TOL + SENS_FACTOR * o.s64
    err = float(np.max(np.abs(np.asarray(vals) - o.r.values)))
    assert err <= tol, (label, err, tol, o.s64)
    strict = o.s64 <= STRICT_SENS
    if not strict:
        print(f"  {label}sensitive trajectory: s64 {o.s64:.1e}, err {err:.1e}, "
              f"ties {o.r.stats.ties}", flush=True)
    return strict


def mixed_value_ok(vals, o, label=""):
    tol = TOL_MIXED + SENS_FACTOR * o.s32
    err = float(np.max(np.abs(np.asarray(vals) - o.r.values)))
    assert err <= tol, (label, err, tol, o.s32)
    return err
