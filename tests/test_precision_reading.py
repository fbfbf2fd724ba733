"""Why the reduced-precision path contracts in FP32 and not BF16.

The oracle's trajectory is replayed with the operands of every two-site
contraction and centre shift rounded to a narrower format (round to nearest
even) and the site tensors stored as complex64, the arithmetic itself kept
exact: a CPU model of matrix-core contractions with FP32 accumulation.  With
FP32 operands (24-bit significand) the per-sample values stay well inside the
1e-4 bar that reduced precision is held to; with BF16 operands (8-bit
significand, unit roundoff 2^-8) they leave it by orders of magnitude within
a few hundred updates, so a BF16 contraction path cannot meet that bar.

Split BF16 products (each operand written as a sum of BF16 parts, the
product as the sum of the partial products that matter) recover precision at
the cost of more matrix-core passes: two parts (three products) carry about
16 significand bits and land about a hundred times above the FP32 model's
error, three parts (six products) reach FP32's level.
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


def split_bf16(x, terms):
    """x as a sum of `terms` bfloat16 numbers per component (hi, then the
    rounded remainders): the operand split of a multi-term BF16 product."""
    parts, rest = [], np.asarray(x, dtype=np.complex128)
    for _ in range(terms):
        h = as_bf16(rest)
        parts.append(h)
        rest = rest - h
    return parts


def split_products(terms):
    """Index pairs (i, j) of the partial products a_i b_j a split matrix
    product keeps: those of order at most 2^-8 (terms - 1) relative to a b
    (part i is about 2^-8 i of its operand), i.e. i + j < terms."""
    return [(i, j) for i in range(terms) for j in range(terms) if i + j < terms]


def split_bf16_mps(terms):
    """The mixed path with every contraction done as a split BF16 product.

    The two-site contraction A_i A_{i+1} keeps the partial products of
    `split_products`; they are summed exactly by contracting the
    concatenation [A_i parts ...] along the shared bond with the matching
    [A_{i+1} parts ...] (the oracle's update then sees a bond of
    len(products) times the width, which changes only its work counters).
    The centre-shift products take both operands as the sum of their parts,
    which differs from dropping the small cross terms by the same order.
    Site tensors are stored as complex64 between operations."""
    pairs = split_products(terms)

    class SplitBF16(MPS):
        def update(self, i, G, chi, right):
            pa = split_bf16(self.A[i], terms)
            pb = split_bf16(self.A[i + 1], terms)
            self.A[i] = np.concatenate([pa[a] for a, _ in pairs], axis=2)
            self.A[i + 1] = np.concatenate([pb[b] for _, b in pairs], axis=0)
            super().update(i, G, chi, right)
            self.A[i], self.A[i + 1] = as_c64(self.A[i]), as_c64(self.A[i + 1])

        def shift(self, c, d):
            self.A[c] = sum(split_bf16(self.A[c], terms))
            self.A[c + d] = sum(split_bf16(self.A[c + d], terms))
            super().shift(c, d)
            self.A[c], self.A[c + d] = as_c64(self.A[c]), as_c64(self.A[c + d])
    return SplitBF16


def test_split_product_model_is_exact_on_a_matrix_product():
    # the concatenation trick sums exactly the kept partial products
    rng = np.random.default_rng(1)
    a = rng.standard_normal((3, 2, 5)) + 1j * rng.standard_normal((3, 2, 5))
    b = rng.standard_normal((5, 2, 4)) + 1j * rng.standard_normal((5, 2, 4))
    for terms in (1, 2, 3):
        pairs = split_products(terms)
        pa, pb = split_bf16(a, terms), split_bf16(b, terms)
        cat = np.einsum("asb,btc->astc", np.concatenate([pa[i] for i, _ in pairs], axis=2),
                        np.concatenate([pb[j] for _, j in pairs], axis=0))
        direct = sum(np.einsum("asb,btc->astc", pa[i], pb[j]) for i, j in pairs)
        assert np.allclose(cat, direct, rtol=0, atol=1e-13)
        exact = np.einsum("asb,btc->astc", a, b)
        rel = np.max(np.abs(cat - exact)) / np.max(np.abs(exact))
        # each kept term carries 8 more bits: about 2^-8 terms relative error
        assert rel < 8 * 2.0 ** (-8 * terms), (terms, rel)


def test_split_bf16_products_against_the_reduced_precision_bar():
    # the same truncated ring as above (chi = 40 cuts, ~300 updates a sample):
    # a two-term split (three BF16 products per complex product component)
    # carries ~16 significand bits and lands near the 1e-4 bar after only a
    # few hundred updates, with the error growing with the update count; a
    # three-term split (six products) is at FP32's level
    p = ti.small_ring(14, seed=5, T=0.6, N=12, delta=math.pi / 24, chi=40, n_samples=2,
                      j_z=0.7)
    t = pai.build_table(p)
    for s in range(2):
        v64, updates = sample_values(MPS, p, t, s)
        v32, _ = sample_values(rounded_mps(as_c64), p, t, s)
        e32 = float(np.max(np.abs(v32 - v64)))
        e2 = float(np.max(np.abs(sample_values(split_bf16_mps(2), p, t, s)[0] - v64)))
        e3 = float(np.max(np.abs(sample_values(split_bf16_mps(3), p, t, s)[0] - v64)))
        print(f"sample {s}: {updates} updates, fp32 {e32:.1e}, bf16x2 {e2:.1e}, bf16x3 {e3:.1e}")
        assert e3 < 10 * max(e32, 1e-7), (e3, e32)
        assert e2 > 10 * e3, (e2, e3)
