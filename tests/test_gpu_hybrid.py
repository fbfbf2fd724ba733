"""Hybrid start on the GPU: every sample begins from a shared Trotter MPS.

The shared state is the oracle's deterministic Trotter evolution (same
schedule, routing and truncation as the samples); the TE-PAI segment then
runs on the GPU and is compared per sample with the oracle (FP64: 1e-10 with
the gap rule; mixed: 1e-4).
"""
import math

import numpy as np
import pytest

import tepai_inputs as ti
from oracle.trotter import trotter_initial_mps
from paper_2604_13144_amd import _lib as L

from test_gpu_parity import compare, gpu_batch
from test_gpu_mixed import TOL_MIXED, against_oracle, run_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return L.Handle(0)


def hybrid_problem(n=12, chi=10, N0=10, T0=0.8, seed=9, ns=5):
    pre = ti.small_ring(n, seed=seed, T=T0, N=N0, delta=math.pi / 16, chi=chi, n_samples=1)
    init = trotter_initial_mps(pre, N0, chi)
    return pre.with_(total_time=0.3, trotter_steps=6, n_samples=ns, initial_mps=init), init


def test_hybrid_fp64(handle):
    p, init = hybrid_problem()
    assert max(init.bonds()) == 10 and init.qubit_at != tuple(range(12))
    print("hybrid fp64: ring n=12 chi=10 from a 10-step Trotter state", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, p.n_samples, [2, 4])
    assert max(st["max_bond"]) == 10
    compare(p, range(p.n_samples), vals, wts, st, 0)


def test_hybrid_mixed(handle):
    p, _ = hybrid_problem(seed=10)
    print("hybrid mixed: ring n=12 chi=10", flush=True)
    vals, _, st = run_batch(handle, p, p.n_samples, [6], L.TEPAI_FP32_MIXED)
    print("hybrid mixed worst", against_oracle(p, vals, st))


# --- the whole hybrid on the GPU: TEPAI_TROTTER batch to t0, read its MPS,
# --- start the TE-PAI samples from it (the oracle prepares its own start)

def canonical_ok(m, tol):
    for k, A in enumerate(m.tensors):
        cl, _, cr = A.shape
        if k < m.centre:
            M = A.reshape(cl * 2, cr)
            assert np.allclose(M.conj().T @ M, np.eye(cr), atol=tol)
        elif k > m.centre:
            M = A.reshape(cl, 2 * cr)
            assert np.allclose(M @ M.conj().T, np.eye(cl), atol=tol)


def gpu_trotter_state(handle, pre, steps, precision=L.TEPAI_FP64):
    b = L.Batch(handle, L.ProblemStruct(pre.with_(trotter=True, n_samples=1), precision=precision), 0, 1)
    b.evolve(steps)
    m = b.read_mps(0)
    b.close()
    return m


def test_read_mps_initial_product_state(handle):
    p = ti.small_ring(6, seed=1, n_samples=2)
    b = L.Batch(handle, L.ProblemStruct(p), 0, 2)
    m = b.read_mps(1)
    assert m.bonds() == (1,) * 7 and m.qubit_at == tuple(range(6)) and m.centre == 0
    for k, A in enumerate(m.tensors):
        e = np.zeros((1, 2, 1), complex)
        e[0, int(p.initial_bits[k]), 0] = 1.0
        assert np.array_equal(A, e)
    with pytest.raises(L.TepaiError) as err:
        b.read_mps(2)
    assert err.value.status == -2


@pytest.mark.parametrize("precision,tol", [(L.TEPAI_FP64, 1e-10), (L.TEPAI_FP32_MIXED, 1e-5)])
def test_read_mps_of_gpu_trotter_equals_oracle_state(handle, precision, tol):
    from test_oracle_hybrid import dense_of
    pre = ti.small_ring(12, seed=9, T=0.8, N=10, delta=math.pi / 16, chi=10, n_samples=1)
    print(f"read_mps: GPU Trotter n=12 chi=10, 10 steps, precision {precision}", flush=True)
    m = gpu_trotter_state(handle, pre, 10, precision)
    ref = trotter_initial_mps(pre, 10, 10)
    assert m.qubit_at == ref.qubit_at and m.centre == ref.centre
    if precision == L.TEPAI_FP64:
        assert m.bonds() == ref.bonds() and max(m.bonds()) == 10
    else:       # the mixed path's 1e-7 singular-value floor may keep fewer
        assert all(a <= b for a, b in zip(m.bonds(), ref.bonds()))
    canonical_ok(m, 1e-12 if precision == L.TEPAI_FP64 else 1e-5)
    a, r = dense_of(m), dense_of(ref)
    assert abs(np.linalg.norm(a) - 1.0) < tol
    assert 1.0 - abs(np.vdot(r, a)) < tol


def test_gpu_only_hybrid_matches_oracle_hybrid(handle):
    pre = ti.small_ring(12, seed=9, T=0.8, N=10, delta=math.pi / 16, chi=10, n_samples=1)
    print("hybrid on the GPU: Trotter to t0, read_mps, TE-PAI segment", flush=True)
    m = gpu_trotter_state(handle, pre, 10)
    seg = pre.with_(total_time=0.3, trotter_steps=6, n_samples=5)
    vals, wts, st = gpu_batch(handle, seg.with_(initial_mps=m), 0, 5, [6])
    # the oracle runs the same segment from its own Trotter state
    compare(seg.with_(initial_mps=trotter_initial_mps(pre, 10, 10)), range(5), vals, wts, st, 0)


# --- truncation on copy: a shared start whose bonds exceed some samples' caps

def centred_random_start(n, chi, seed, centre):
    from oracle.mps import MPS
    init = ti.random_mps(n, chi, seed)
    m = MPS.from_initial(init)
    while m.centre < centre:
        m.shift(m.centre, +1)
    return ti.InitialMPS(tensors=tuple(m.A), centre=centre, qubit_at=init.qubit_at)


def truncated_start_problem():
    # bonds up to 16 around the middle of a 12-site chain; caps 4, 8, 16, 6, 2:
    # four of the five samples truncate their copy before the first step
    init = centred_random_start(12, 16, seed=9, centre=5)
    p = ti.small_ring(12, seed=4, T=0.3, N=6, delta=math.pi / 16, chi=16, n_samples=5)
    return p.with_(initial_mps=init, chi_per_sample=(4, 8, 16, 6, 2)), init


def test_truncation_on_copy_fp64(handle):
    p, init = truncated_start_problem()
    assert max(init.bonds()) == 16
    print("truncation on copy fp64: random chi=16 start, caps 4/8/16/6/2", flush=True)
    vals, wts, st = gpu_batch(handle, p, 0, p.n_samples, [1, 5])
    assert all(int(m) <= c for m, c in zip(st["max_bond"], p.chi_per_sample))
    compare(p, range(p.n_samples), vals, wts, st, 0)


def test_truncation_on_copy_state_before_any_step(handle):
    # right after batch creation a truncated slot holds the oracle's truncated
    # copy, centre on the last site; the cap-16 slot holds the start unchanged
    from oracle.mps import MPS
    p, init = truncated_start_problem()
    b = L.Batch(handle, L.ProblemStruct(p), 0, p.n_samples)
    for slot, cap in enumerate(p.chi_per_sample):
        g = b.read_mps(slot)
        ref = MPS.from_initial(init, p.svd_cutoff)
        if cap < 16:
            ref.truncate_to(cap)
        assert g.centre == ref.centre and g.bonds() == tuple(ref.bonds())
        dg = MPS.from_initial(g).to_dense()
        assert np.max(np.abs(dg - ref.to_dense())) <= 1e-12, slot
    st = b.stats()
    assert list(st["shifts"]) == [5 + 11 if c < 16 else 0 for c in p.chi_per_sample]
    assert list(st["max_bond"]) == [min(c, 16) for c in p.chi_per_sample]
    b.close()


def test_truncation_on_copy_mixed(handle):
    p, _ = truncated_start_problem()
    print("truncation on copy mixed: random chi=16 start, caps 4/8/16/6/2", flush=True)
    vals, _, st = run_batch(handle, p, p.n_samples, [6], L.TEPAI_FP32_MIXED)
    print("truncation on copy mixed worst", against_oracle(p, vals, st))
