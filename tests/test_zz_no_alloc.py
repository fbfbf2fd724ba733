"""tepai_run_noalloc (the estimator in the library's fixed device array)
against tepai_run, which allocates its own workspace.

Both run the same kernels on the same samples, so per-sample values, weights
and the estimate must agree to the FP64 bar (1e-10; in practice bitwise) and
every counter exactly.  Two calls in a row, the second on a smaller problem,
check that nothing the first call left in the shared array leaks into the
second; a problem whose single sample does not fit is rejected up front.
"""
import math

import numpy as np
import pytest
import torch

import tepai_inputs as ti
from paper_2604_13144_amd import _lib as L

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def run_noalloc(handle, p, precision=0):
    ps = L.ProblemStruct(p, precision=precision)
    dev = torch.device("cuda", 0)
    ns, no = int(ps.struct.n_samples), int(ps.struct.n_obs)
    d_mean = torch.full((no,), float("nan"), dtype=torch.float64, device=dev)
    d_se = torch.full((no,), float("nan"), dtype=torch.float64, device=dev)
    d_w = torch.full((ns,), float("nan"), dtype=torch.float64, device=dev)
    d_v = torch.full((ns * no,), float("nan"), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    stats = L.tepai_run_noalloc(handle, ps, d_mean, d_se, d_w, d_v)
    torch.cuda.synchronize()
    return dict(mean=d_mean.cpu().numpy(), std_err=d_se.cpu().numpy(),
                weights=d_w.cpu().numpy(), values=d_v.cpu().numpy().reshape(ns, no),
                stats=stats)


def check_same(a, b):
    assert np.array_equal(a["weights"], b["weights"])
    assert np.max(np.abs(a["values"] - b["values"])) <= TOL
    assert np.max(np.abs(a["mean"] - b["mean"])) <= TOL
    ok = np.isfinite(b["std_err"])
    assert np.array_equal(ok, np.isfinite(a["std_err"]))
    assert np.all(np.abs(a["std_err"][ok] - b["std_err"][ok]) <= TOL)
    for f in ("n_gates", "updates", "shifts", "jacobi_sweeps", "sign", "max_bond", "flags"):
        assert np.array_equal(a["stats"][f], b["stats"][f]), f


def test_noalloc_matches_run_on_two_calls(handle):
    big = ti.small_ring(12, seed=11, T=0.4, N=10, delta=math.pi / 16, chi=16, n_samples=40)
    small = ti.small_ring(8, seed=3, T=0.3, N=6, delta=math.pi / 16, chi=4, n_samples=5)
    print("no-alloc: ring n=12 chi=16 40 samples, then ring n=8 chi=4 5 samples", flush=True)
    first = run_noalloc(handle, big)
    second = run_noalloc(handle, small)
    check_same(first, L.tepai_run(handle, L.ProblemStruct(big)))
    check_same(second, L.tepai_run(handle, L.ProblemStruct(small)))
    assert max(first["stats"]["max_bond"]) > 4


def test_noalloc_mixed_path_and_truncated_shared_start(handle):
    # the mixed path, from a shared chi = 16 start that the cap-4 and cap-8
    # samples truncate on copy (the start kernel runs in the fixed array too)
    from oracle.mps import MPS
    init = ti.random_mps(12, 16, seed=9)
    m = MPS.from_initial(init)
    while m.centre < 5:
        m.shift(m.centre, +1)
    init = ti.InitialMPS(tensors=tuple(m.A), centre=5, qubit_at=init.qubit_at)
    p = ti.small_ring(12, seed=4, T=0.3, N=6, delta=math.pi / 16, chi=16, n_samples=6)
    p = p.with_(initial_mps=init, chi_per_sample=(4, 8, 16, 4, 8, 16))
    print("no-alloc: mixed path, shared chi=16 start, caps 4/8/16", flush=True)
    a = run_noalloc(handle, p, precision=1)
    check_same(a, L.tepai_run(handle, L.ProblemStruct(p, precision=1)))
    assert list(a["stats"]["max_bond"]) == [4, 8, 16, 4, 8, 16]


def test_noalloc_batches_through_the_array(handle):
    # one sample of the n=64, chi=128 ring needs ~35 MiB: 16 samples take
    # several passes through the 256 MiB array (first 2 Trotter steps)
    p = ti.config(4).with_(n_samples=16, trotter_steps=2, total_time=3.0 * 2 / 800)
    ps = L.ProblemStruct(p)
    assert L.tepai_workspace_size(handle, ps, 16) > L.NOALLOC_BYTES
    print("no-alloc: xxz n=64 chi=128, 16 samples, 2 steps", flush=True)
    a = run_noalloc(handle, p)
    check_same(a, L.tepai_run(handle, ps))


def test_noalloc_rejects_a_sample_beyond_the_array(handle):
    # n = 200 at chi = 256: 200 site slots of 2 chi^2 complex doubles each
    p = ti.small_ring(200, seed=1, T=0.1, N=2, delta=math.pi / 16, chi=256, n_samples=2)
    ps = L.ProblemStruct(p)
    assert L.tepai_workspace_size(handle, ps, 1) > L.NOALLOC_BYTES
    dev = torch.device("cuda", 0)
    no = int(ps.struct.n_obs)
    bufs = [torch.zeros(k, dtype=torch.float64, device=dev) for k in (no, no, 2, 2 * no)]
    with pytest.raises(L.TepaiError) as e:
        L.tepai_run_noalloc(handle, ps, *bufs)
    assert e.value.status == -3    # TEPAI_ENOMEM
