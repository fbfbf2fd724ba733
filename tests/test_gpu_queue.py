"""The work-queue evolve kernel (TEPAI_WORK_QUEUE) against one workgroup per
slot.

Scheduling does not enter a sample's arithmetic: either way one workgroup
evolves a slot with the same per-slot code, only which workgroup and when
differ, so values, weights, every counter and the site tensors must agree
bitwise.  The batches hold more samples than the chip has CUs (256), so each
workgroup of the queue takes several slots, with mixed bond caps (slots go
out by decreasing cap); a batch smaller than the grid checks the clamp.
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


def mixed_caps(count, seed=5):
    caps = tuple((4, 8, 16)[s % 3] for s in range(count))
    return ti.small_ring(8, seed=seed, T=0.4, N=10, delta=math.pi / 16, chi=16,
                         n_samples=count).with_(chi_per_sample=caps)


def run_batch(handle, p, precision, work_queue, parts=(4, 6)):
    ps = L.ProblemStruct(p, precision=precision, work_queue=work_queue)
    count = int(ps.struct.n_samples)
    b = L.Batch(handle, ps, 0, count)
    for J in parts:
        b.evolve(J)
    dev = torch.device("cuda", 0)
    v = torch.full((count * ps.n_obs,), float("nan"), dtype=torch.float64, device=dev)
    w = torch.full((count,), float("nan"), dtype=torch.float64, device=dev)
    b.observe(v, w)
    torch.cuda.synchronize()
    slots = sorted({0, 1, 2, count // 2, count - 1})
    return dict(values=v.cpu().numpy(), weights=w.cpu().numpy(), stats=b.stats(),
                mps={s: b.read_mps(s) for s in slots})


def assert_identical(a, b):
    assert np.array_equal(a["values"], b["values"])
    assert np.array_equal(a["weights"], b["weights"])
    for f in a["stats"].dtype.names:
        assert np.array_equal(a["stats"][f], b["stats"][f]), f
    for s, m in a["mps"].items():
        o = b["mps"][s]
        assert m.centre == o.centre and m.qubit_at == o.qubit_at, s
        for x, y in zip(m.tensors, o.tensors):
            assert x.shape == y.shape and np.array_equal(x, y), s


@pytest.mark.parametrize("precision", [0, 1])
def test_queue_equals_one_workgroup_per_slot(handle, precision):
    p = mixed_caps(600)
    print(f"queue: ring n=8, 600 samples, caps 4/8/16, 10 steps, precision {precision}",
          flush=True)
    plain = run_batch(handle, p, precision, False)
    queued = run_batch(handle, p, precision, True)
    assert_identical(plain, queued)
    st = queued["stats"]
    assert np.all(st["layer"] == 10)
    caps = np.array(p.chi_per_sample)
    assert np.all(st["max_bond"] <= caps)
    assert st["max_bond"][caps == 16].max() > 8     # the caps bind


def test_queue_with_fewer_slots_than_cus(handle):
    p = mixed_caps(7, seed=9)
    print("queue: ring n=8, 7 samples (grid clamped to the slot count)", flush=True)
    assert_identical(run_batch(handle, p, 0, False, parts=(10,)),
                     run_batch(handle, p, 0, True, parts=(10,)))


def test_queue_through_the_synchronous_estimators(handle):
    # tepai_run (batches of up to 1024) and tepai_run_noalloc (the fixed array)
    p = mixed_caps(300, seed=13)
    print("queue: tepai_run / tepai_run_noalloc, 300 samples", flush=True)
    ref = L.tepai_run(handle, L.ProblemStruct(p))
    got = L.tepai_run(handle, L.ProblemStruct(p, work_queue=True))
    for k in ("mean", "std_err", "weights", "values"):
        assert np.array_equal(ref[k], got[k]), k
    for f in ref["stats"].dtype.names:
        assert np.array_equal(ref["stats"][f], got["stats"][f]), f
    ps = L.ProblemStruct(p, work_queue=True)
    dev = torch.device("cuda", 0)
    ns, no = int(ps.struct.n_samples), ps.n_obs
    out = [torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
           for k in (no, no, ns, ns * no)]
    torch.cuda.synchronize()
    L.tepai_run_noalloc(handle, ps, *out)
    torch.cuda.synchronize()
    assert np.array_equal(out[0].cpu().numpy(), ref["mean"])
    assert np.array_equal(out[2].cpu().numpy(), ref["weights"])
    assert np.array_equal(out[3].cpu().numpy().reshape(ns, no), ref["values"])


def test_queue_in_a_captured_step(handle):
    # the counter is reset by a kernel inside the graph on every replay
    p = mixed_caps(300, seed=17)
    ps_q = L.ProblemStruct(p, work_queue=True)
    ps_p = L.ProblemStruct(p)
    count, n_obs, J = 300, ps_q.n_obs, 2
    print("queue: captured step, 300 samples, 4 replays of 2 steps", flush=True)
    stream = torch.cuda.Stream()
    dev = torch.device("cuda", 0)

    def bufs():
        return [torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
                for k in (count * n_obs, count, n_obs, n_obs)]

    eager = L.Batch(handle, ps_p, 0, count, stream=stream)
    graphed = L.Batch(handle, ps_q, 0, count, stream=stream)
    ev, gv = bufs(), bufs()
    g = graphed.capture_step(J, *gv)
    for rep in range(4):
        eager.evolve(J)
        eager.observe(ev[0], ev[1])
        L.tepai_reduce(handle, count, n_obs, ev[0], ev[1], ev[2], ev[3], stream)
        g.launch()
        stream.synchronize()
        scratch = torch.ones(1024, dtype=torch.float64, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(scratch) == 1024.0
        for a, b in zip(ev, gv):
            assert torch.equal(a, b), rep
    g.close()
