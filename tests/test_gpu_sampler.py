"""GPU sampler vs the oracle: sampled circuits must be bit-identical."""
import numpy as np
import pytest

import tepai_inputs as ti
from oracle import pai, sampler
from paper_2604_13144_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def check_bit_exact(handle, p, samples, layers=0):
    ps = L.ProblemStruct(p)
    t = pai.build_table(p)
    first, count = samples[0], len(samples)
    print(f"sampler parity: {p.name} samples {first}..{first + count - 1} layers {layers}", flush=True)
    off, words, signs = L.tepai_sample_circuits(handle, ps, first, count, layers)
    for i, s in enumerate(samples):
        c = sampler.sample_circuit(p, t, p.sample_offset + s, layers or None)
        w = words[off[i]:off[i + 1]].astype(np.uint64)
        assert np.array_equal(w >> np.uint64(2), c.draws), f"sample {s}"
        assert np.array_equal((w & np.uint64(3)).astype(np.uint8), c.settings), f"sample {s}"
        assert int(signs[i]) == c.sign


def test_sampler_cfg1_all_samples(handle):
    p = ti.config(1)
    check_bit_exact(handle, p, list(range(p.n_samples)))


def test_sampler_cfg2_subset(handle):
    check_bit_exact(handle, ti.config(2), list(range(0, 48)))


def test_sampler_cfg4_subset_and_prefix(handle):
    p = ti.config(4)
    check_bit_exact(handle, p, list(range(100, 108)))
    check_bit_exact(handle, p, list(range(5, 9)), layers=37)


def test_sampler_no_pi_variant(handle):
    p = ti.config(4).with_(no_pi=True)
    check_bit_exact(handle, p, list(range(0, 8)))
    _, words, signs = L.tepai_sample_circuits(handle, L.ProblemStruct(p), 0, 8, 0)
    assert np.all(signs == 1) and not np.any((words.astype(np.uint64) & np.uint64(3)) == 2)


def test_sampler_offset_and_seed(handle):
    p = ti.config(2).with_(sample_offset=123_456, seed=0xDEADBEEFCAFEF00D, n_samples=64)
    check_bit_exact(handle, p, list(range(0, 16)))
