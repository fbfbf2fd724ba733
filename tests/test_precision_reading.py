"""Why the reduced-precision path contracts in FP32 and not BF16.

The oracle's trajectory is replayed with the operands of every two-site
contraction and centre shift rounded to a narrower format (round to nearest
even) and the site tensors stored as complex64, the arithmetic itself kept
exact: a CPU model of matrix-core contractions with FP32 accumulation.  With
FP32 operands (24-bit significand) the per-sample values stay well inside the
1e-4 bar that reduced precision is held to; with BF16 operands (8-bit
significand, unit roundoff 2^-8) they leave it by orders of magnitude within
a few hundred updates, so a BF16 contraction path cannot meet that bar.
"""
import math

import numpy as np

import tepai_inputs as ti
from oracle import pai
from oracle.mps import MPS
from oracle.run import chi_of, observable_value
from oracle.sampler import sample_circuit
from oracle.schedule import build_schedule


def as_c64(x):
    return x.astype(np.complex64).astype(np.complex128)


def bf16(x):
    """Round float values to the nearest bfloat16 (ties to even)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def as_bf16(x):
    return bf16(x.real) + 1j * bf16(x.imag)


def rounded_mps(round_operands):
    class Rounded(MPS):
        def update(self, i, G, chi, right):
            self.A[i], self.A[i + 1] = round_operands(self.A[i]), round_operands(self.A[i + 1])
            super().update(i, G, chi, right)
            self.A[i], self.A[i + 1] = as_c64(self.A[i]), as_c64(self.A[i + 1])

        def shift(self, c, d):
            self.A[c], self.A[c + d] = round_operands(self.A[c]), round_operands(self.A[c + d])
            super().shift(c, d)
            self.A[c], self.A[c + d] = as_c64(self.A[c]), as_c64(self.A[c + d])
    return Rounded


def sample_values(cls, p, t, s):
    circ = sample_circuit(p, t, s)
    ops, qa = build_schedule(p, t, circ, chi_of(p, s))
    m = cls(p.initial_bits, p.svd_cutoff).run(ops)
    return np.array([observable_value(m, qa, o) for o in p.observables]), m.stats.updates


def test_bf16_contractions_miss_the_reduced_precision_bar():
    # truncated ring: chi = 40 cuts, ~300 two-site updates per sample
    p = ti.small_ring(14, seed=5, T=0.6, N=12, delta=math.pi / 24, chi=40, n_samples=2,
                      j_z=0.7)
    t = pai.build_table(p)
    for s in range(2):
        v64, updates = sample_values(MPS, p, t, s)
        v32, _ = sample_values(rounded_mps(as_c64), p, t, s)
        vbf, _ = sample_values(rounded_mps(as_bf16), p, t, s)
        e32 = float(np.max(np.abs(v32 - v64)))
        ebf = float(np.max(np.abs(vbf - v64)))
        assert updates > 250
        assert e32 < 1e-5, e32
        assert ebf > 1e-3, ebf


def test_bf16_rounding_is_round_to_nearest_even():
    # exactly representable values stay; halfway cases go to the even neighbour
    assert bf16(np.float32(1.0)) == 1.0 and bf16(np.float32(-0.5)) == -0.5
    one_ulp = 2.0 ** -7                                 # spacing of bf16 in [1, 2)
    assert bf16(np.float32(1.0 + one_ulp / 2)) == 1.0   # tie, 1.0 is even
    assert bf16(np.float32(1.0 + 1.5 * one_ulp)) == 1.0 + 2 * one_ulp
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    r = bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))   # unit roundoff 2^-8
