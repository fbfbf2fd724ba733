"""Captured read-out steps (HIP graph) against the same steps launched one
by one: each replay advances every sample by the captured number of Trotter
steps and leaves the time-series estimate at the new time (sec.
"Deterministic Expectation Values"); the graph holds the same kernels on the
same state, so every replay's per-sample values, weights and estimate must
equal the eagerly launched step's bitwise.  Replays alternate with eager
work and synchronisations of the program's own, and every replay is checked.
"""
import math

import numpy as np
import pytest
import torch

import tepai_inputs as ti
from paper_2604_13144_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def buffers(count, n_obs):
    dev = torch.device("cuda", 0)
    return (torch.full((count * n_obs,), float("nan"), dtype=torch.float64, device=dev),
            torch.full((count,), float("nan"), dtype=torch.float64, device=dev),
            torch.full((n_obs,), float("nan"), dtype=torch.float64, device=dev),
            torch.full((n_obs,), float("nan"), dtype=torch.float64, device=dev))


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_eager_steps(handle, precision):
    p = ti.small_ring(12, seed=11, T=0.5, N=12, delta=math.pi / 16, chi=8, n_samples=6)
    ps = L.ProblemStruct(p, precision=precision)
    n_obs, count, J = ps.n_obs, 6, 3
    print(f"graph: ring n=12 chi=8, 6 samples, 4 replays of {J} steps, precision {precision}",
          flush=True)
    stream = torch.cuda.Stream()
    eager = L.Batch(handle, ps, 0, count, stream=stream)
    graphed = L.Batch(handle, ps, 0, count, stream=stream)
    ev, gv = buffers(count, n_obs), buffers(count, n_obs)
    g = graphed.capture_step(J, *gv)
    for rep in range(4):
        eager.evolve(J)
        eager.observe(ev[0], ev[1])
        L.tepai_reduce(handle, count, n_obs, ev[0], ev[1], ev[2], ev[3], stream)
        g.launch()
        stream.synchronize()
        # eager work of the program's own between replays
        scratch = torch.ones(1024, dtype=torch.float64, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(scratch) == 1024.0
        for a, b in zip(ev, gv):
            assert torch.equal(a, b), rep
        st = graphed.stats()
        assert np.all(st["layer"] == J * (rep + 1))
    with pytest.raises(L.TepaiError) as e:
        g.launch()            # steps 12..15 would pass N = 12: refused on the host
    assert e.value.status == -2
    g.close()


def test_capture_rejects_the_null_stream(handle):
    p = ti.small_ring(8, seed=3, T=0.3, N=6, delta=math.pi / 16, chi=4, n_samples=2)
    ps = L.ProblemStruct(p)
    b = L.Batch(handle, ps, 0, 2, stream=torch.cuda.default_stream())
    with pytest.raises(L.TepaiError) as e:
        b.capture_step(2, *buffers(2, ps.n_obs))
    assert e.value.status == -1
