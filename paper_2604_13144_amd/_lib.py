"""ctypes binding of libtepai (argument marshalling only).

Every function mirrors one entry point of include/tepai.h and has the same
name.  Device buffers and streams come from PyTorch; all computation happens
in the HIP library.  Importing this module fails loudly when libtepai.so has
not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtepai.so")

TEPAI_OK = 0
STATUS_NAMES = {0: "TEPAI_OK", -1: "TEPAI_EINVAL", -2: "TEPAI_ERANGE", -3: "TEPAI_ENOMEM",
                -4: "TEPAI_EDEVICE", -5: "TEPAI_ENUMERIC"}
PAULI_CODE = {"X": 1, "Y": 2, "Z": 3}
TEPAI_FP64 = 0
TEPAI_FP32_MIXED = 1
TEPAI_NO_PI = 1
TEPAI_TROTTER = 2
TEPAI_PER_GATE = 4
TEPAI_WORK_QUEUE = 8
TEPAI_ENUMERIC = -5
TEPAI_SAMPLE_NONFINITE = 1
TEPAI_SAMPLE_NONCONVERGED = 2


class tepai_term(C.Structure):
    _fields_ = [("nq", C.c_uint32), ("qubit", C.c_uint32 * 2), ("pauli", C.c_uint8 * 2),
                ("pad", C.c_uint8 * 6), ("coeff", C.c_double)]


class tepai_pauli_string(C.Structure):
    _fields_ = [("n_ops", C.c_uint32), ("observable", C.c_uint32),
                ("qubits", C.POINTER(C.c_uint32)), ("paulis", C.POINTER(C.c_uint8)),
                ("coeff", C.c_double)]


class tepai_mps(C.Structure):
    _fields_ = [("bond", C.POINTER(C.c_uint32)), ("tensors", C.POINTER(C.c_double)),
                ("qubit_at", C.POINTER(C.c_uint32)), ("centre", C.c_uint32),
                ("reserved", C.c_uint32)]


class tepai_problem(C.Structure):
    _fields_ = [("n_qubits", C.c_uint32), ("n_terms", C.c_uint32),
                ("terms", C.POINTER(tepai_term)), ("total_time", C.c_double),
                ("trotter_steps", C.c_uint32), ("delta", C.c_double),
                ("n_samples", C.c_uint64), ("sample_offset", C.c_uint64),
                ("seed", C.c_uint64), ("chi_max", C.c_uint32),
                ("chi_per_sample", C.POINTER(C.c_uint32)), ("svd_cutoff", C.c_double),
                ("initial_bits", C.POINTER(C.c_uint8)), ("n_obs", C.c_uint32),
                ("n_strings", C.c_uint32), ("strings", C.POINTER(tepai_pauli_string)),
                ("precision", C.c_uint32), ("flags", C.c_uint32),
                ("initial_mps", C.POINTER(tepai_mps))]


class tepai_sample_stats(C.Structure):
    _fields_ = [("n_gates", C.c_uint64), ("updates", C.c_uint64), ("swap_updates", C.c_uint64),
                ("shifts", C.c_uint64), ("jacobi_sweeps", C.c_uint64),
                ("nonconverged", C.c_uint64), ("ties", C.c_uint64),
                ("sum_chi3", C.c_double), ("nominal_flops", C.c_double),
                ("discarded", C.c_double), ("max_discarded", C.c_double),
                ("min_gap", C.c_double), ("sign", C.c_int32), ("layer", C.c_uint32),
                ("max_bond", C.c_uint32), ("flags", C.c_uint32)]


STATS_FIELDS = [f for f, _ in tepai_sample_stats._fields_]
STATS_DTYPE = np.dtype([(f, np.float64 if t in (C.c_double,) else np.int64)
                        for f, t in tepai_sample_stats._fields_])

# Exported symbols and their prototypes (restype, argtypes).
_P = C.c_void_p
PROTOTYPES = {
    "tepai_create": (C.c_int, [C.POINTER(_P), C.c_int]),
    "tepai_destroy": (None, [_P]),
    "tepai_last_error": (C.c_char_p, [_P]),
    "tepai_validate": (C.c_int, [_P, C.POINTER(tepai_problem)]),
    "tepai_pai_table": (C.c_int, [_P, C.POINTER(tepai_problem), C.c_uint32,
                                  C.POINTER(C.c_uint32), _P, _P, _P, _P,
                                  C.POINTER(C.c_double), C.POINTER(C.c_uint32)]),
    "tepai_sample_circuits": (C.c_int, [_P, C.POINTER(tepai_problem), C.c_uint64, C.c_uint64,
                                        C.c_uint32, C.c_uint64, _P, _P, _P]),
    "tepai_workspace_size": (C.c_int, [_P, C.POINTER(tepai_problem), C.c_uint32,
                                       C.POINTER(C.c_size_t)]),
    "tepai_batch_create": (C.c_int, [_P, C.POINTER(tepai_problem), C.c_uint64, C.c_uint32,
                                     _P, C.c_size_t, _P, C.POINTER(_P)]),
    "tepai_batch_evolve": (C.c_int, [_P, C.c_uint32]),
    "tepai_batch_observe": (C.c_int, [_P, _P, _P]),
    "tepai_batch_stats": (C.c_int, [_P, C.POINTER(tepai_sample_stats)]),
    "tepai_batch_read_mps": (C.c_int, [_P, C.c_uint32, C.c_uint64, _P, _P,
                                       C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), _P]),
    "tepai_batch_destroy": (None, [_P]),
    "tepai_reduce": (C.c_int, [_P, C.c_uint64, C.c_uint32, _P, _P, _P, _P, _P]),
    "tepai_run": (C.c_int, [_P, C.POINTER(tepai_problem), C.c_uint32, _P, _P, _P, _P,
                            C.POINTER(tepai_sample_stats)]),
    "tepai_batch_capture_step": (C.c_int, [_P, C.c_uint32, _P, _P, _P, _P, C.POINTER(_P)]),
    "tepai_batch_autotune": (C.c_int, [_P, C.c_uint32, _P, C.c_uint32, _P, C.c_size_t, _P, _P,
                                       C.POINTER(C.c_uint32)]),
    "tepai_step_graph_launch": (C.c_int, [_P]),
    "tepai_step_graph_destroy": (None, [_P]),
    "tepai_run_noalloc": (C.c_int, [_P, C.POINTER(tepai_problem), _P, _P, _P, _P, _P,
                                    C.POINTER(tepai_sample_stats)]),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libtepai.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TepaiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st: int, h) -> None:
    if st != TEPAI_OK:
        msg = load().tepai_last_error(h) if h else b""
        raise TepaiError(st, (msg or b"").decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ problem
class ProblemStruct:
    """A tepai_problem plus the host arrays it points to (kept alive here)."""

    def __init__(self, problem, chi_per_sample: Optional[Sequence[int]] = None,
                 precision: int = TEPAI_FP64, work_queue: bool = False):
        p = problem
        if len(p.initial_bits) != p.n_qubits:
            raise ValueError("initial_bits must hold one character per qubit")
        n_terms = len(p.terms)
        self._terms = (tepai_term * n_terms)()
        for k, t in enumerate(p.terms):
            tt = self._terms[k]
            tt.nq = len(t.qubits)
            for i, (q, ch) in enumerate(zip(t.qubits, t.paulis)):
                tt.qubit[i] = q
                tt.pauli[i] = PAULI_CODE[ch]
            tt.coeff = float(t.coeff)
        strings = [(o, ps) for o, obs in enumerate(p.observables) for ps in obs]
        self._strings = (tepai_pauli_string * max(len(strings), 1))()
        self._keep = []
        for i, (o, ps) in enumerate(strings):
            qa = np.ascontiguousarray(ps.qubits, dtype=np.uint32)
            pa = np.ascontiguousarray([PAULI_CODE[c] for c in ps.paulis], dtype=np.uint8)
            self._keep += [qa, pa]
            s = self._strings[i]
            s.n_ops = len(ps.qubits)
            s.observable = o
            s.qubits = qa.ctypes.data_as(C.POINTER(C.c_uint32))
            s.paulis = pa.ctypes.data_as(C.POINTER(C.c_uint8))
            s.coeff = float(ps.coeff)
        self._bits = np.ascontiguousarray([int(b) for b in p.initial_bits], dtype=np.uint8)
        cps = chi_per_sample if chi_per_sample is not None else p.chi_per_sample
        self._cps = None if cps is None else np.ascontiguousarray(cps, dtype=np.uint32)
        if self._cps is not None and self._cps.size != p.n_samples:
            raise ValueError("chi_per_sample must hold one cap per sample")
        s = tepai_problem()
        s.n_qubits = p.n_qubits
        s.n_terms = n_terms
        s.terms = C.cast(self._terms, C.POINTER(tepai_term))
        s.total_time = float(p.total_time)
        s.trotter_steps = int(p.trotter_steps)
        s.delta = float(p.delta)
        s.n_samples = int(p.n_samples)
        s.sample_offset = int(p.sample_offset)
        s.seed = int(p.seed)
        s.chi_max = int(p.chi_max)
        s.chi_per_sample = (self._cps.ctypes.data_as(C.POINTER(C.c_uint32))
                            if self._cps is not None else None)
        s.svd_cutoff = float(p.svd_cutoff)
        s.initial_bits = self._bits.ctypes.data_as(C.POINTER(C.c_uint8))
        s.n_obs = len(p.observables)
        s.n_strings = len(strings)
        s.strings = C.cast(self._strings, C.POINTER(tepai_pauli_string))
        s.precision = int(precision)
        s.flags = ((TEPAI_NO_PI if getattr(p, "no_pi", False) else 0)
                   | (TEPAI_TROTTER if getattr(p, "trotter", False) else 0)
                   | (TEPAI_PER_GATE if getattr(p, "per_gate", False) else 0)
                   | (TEPAI_WORK_QUEUE if work_queue else 0))
        init = getattr(p, "initial_mps", None)
        s.initial_mps = None
        if init is not None:
            if len(init.tensors) != p.n_qubits or len(init.qubit_at) != p.n_qubits:
                raise ValueError("initial_mps must hold one tensor and one qubit per site")
            bonds = np.ascontiguousarray(init.bonds(), dtype=np.uint32)
            packed = np.concatenate([np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)
                                     for a in init.tensors]).view(np.float64)
            qa = np.ascontiguousarray(init.qubit_at, dtype=np.uint32)
            self._init = (bonds, packed, qa)
            self._mps = tepai_mps(bonds.ctypes.data_as(C.POINTER(C.c_uint32)),
                                  packed.ctypes.data_as(C.POINTER(C.c_double)),
                                  qa.ctypes.data_as(C.POINTER(C.c_uint32)), int(init.centre), 0)
            s.initial_mps = C.pointer(self._mps)
        self.struct = s
        self.n_obs = s.n_obs

    def ref(self):
        return C.byref(self.struct)


# ------------------------------------------------------------------- handle
class Handle:
    def __init__(self, device: int = 0):
        lib = load()
        h = C.c_void_p()
        st = lib.tepai_create(C.byref(h), int(device))
        if st != TEPAI_OK:
            raise TepaiError(st, f"cannot open gfx950 device {device}")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            load().tepai_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _hh(h):
    return h.h if h is not None else None


def tepai_validate(h: Optional[Handle], ps: ProblemStruct) -> None:
    """Host-only; ``h`` may be None (then only the status code is reported)."""
    _check(load().tepai_validate(_hh(h), ps.ref()), _hh(h))


def tepai_pai_table(h: Optional[Handle], ps: ProblemStruct):
    """Host-only; ``h`` may be None."""
    lib = load()
    hh = _hh(h)
    n = C.c_uint32()
    lg = C.c_double()
    ns = C.c_uint32()
    st = lib.tepai_pai_table(hh, ps.ref(), 0, C.byref(n), None, None, None, None,
                             C.byref(lg), C.byref(ns))
    if st not in (TEPAI_OK, -3):
        _check(st, hh)
    L = n.value
    term = np.zeros(L, np.uint32)
    theta = np.zeros(L, np.float64)
    gamma = np.zeros((L, 3), np.float64)
    thr = np.zeros((L, 2), np.uint64)
    _check(lib.tepai_pai_table(hh, ps.ref(), L, C.byref(n), _ptr(term), _ptr(theta),
                               _ptr(gamma), _ptr(thr), C.byref(lg), C.byref(ns)), hh)
    return dict(l_eff=L, term=term, theta=theta, gamma=gamma, thresholds=thr,
                log_g1_step=lg.value, n_split_terms=ns.value)


def tepai_sample_circuits(h: Handle, ps: ProblemStruct, first: int, count: int, layers: int = 0):
    """Returns (offsets[count+1], words[...], signs[count])."""
    lib = load()
    offsets = np.zeros(count + 1, np.uint64)
    signs = np.zeros(count, np.int8)
    st = lib.tepai_sample_circuits(h.h, ps.ref(), first, count, layers, 0, _ptr(offsets),
                                   None, _ptr(signs))
    if st not in (TEPAI_OK, -3):
        _check(st, h.h)
    total = int(offsets[-1])
    words = np.zeros(max(total, 1), np.uint32)
    _check(lib.tepai_sample_circuits(h.h, ps.ref(), first, count, layers, total,
                                     _ptr(offsets), _ptr(words), _ptr(signs)), h.h)
    return offsets, words[:total], signs


def tepai_workspace_size(h: Optional[Handle], ps: ProblemStruct, count: int) -> int:
    """Host-only; ``h`` may be None."""
    b = C.c_size_t()
    _check(load().tepai_workspace_size(_hh(h), ps.ref(), count, C.byref(b)), _hh(h))
    return b.value


class MPSState:
    """A host copy of one sample's MPS, in the form a problem's initial_mps takes."""

    def __init__(self, tensors, centre, qubit_at):
        self.tensors, self.centre, self.qubit_at = tensors, centre, qubit_at

    def bonds(self):
        return (1,) + tuple(int(a.shape[2]) for a in self.tensors)


class Batch:
    """A batch of samples living in a torch-allocated device workspace."""

    def __init__(self, h: Handle, ps: ProblemStruct, first: int, count: int,
                 workspace=None, stream=None):
        import torch
        self.h, self.ps, self.count = h, ps, count
        need = tepai_workspace_size(h, ps, count)
        dev = torch.device("cuda", h.device)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        if workspace.numel() < need:
            raise TepaiError(-3, "workspace too small")
        self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        b = C.c_void_p()
        _check(load().tepai_batch_create(h.h, ps.ref(), first, count,
                                         C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(b)), h.h)
        self.b = b

    def evolve(self, n_layers: int) -> None:
        _check(load().tepai_batch_evolve(self.b, n_layers), self.h.h)

    def observe(self, d_values, d_weights) -> None:
        _check(load().tepai_batch_observe(self.b, C.c_void_p(d_values.data_ptr()),
                                          C.c_void_p(d_weights.data_ptr())), self.h.h)

    def stats(self) -> np.ndarray:
        arr = (tepai_sample_stats * self.count)()
        _check(load().tepai_batch_stats(self.b, arr), self.h.h)
        out = np.zeros(self.count, STATS_DTYPE)
        for i in range(self.count):
            for f in STATS_FIELDS:
                out[f][i] = getattr(arr[i], f)
        return out

    def read_mps(self, slot: int) -> "MPSState":
        """The MPS of one slot at its current step (host copy, complex128)."""
        n = int(self.ps.struct.n_qubits)
        bond = np.zeros(n + 1, dtype=np.uint32)
        qubit_at = np.zeros(n, dtype=np.uint32)
        centre, total = C.c_uint32(), C.c_uint64()
        lib = load()
        _check(lib.tepai_batch_read_mps(self.b, slot, 0, bond.ctypes.data, qubit_at.ctypes.data,
                                        C.byref(centre), C.byref(total), None), self.h.h)
        buf = np.zeros(2 * total.value, dtype=np.float64)
        _check(lib.tepai_batch_read_mps(self.b, slot, total.value, bond.ctypes.data,
                                        qubit_at.ctypes.data, C.byref(centre), C.byref(total),
                                        buf.ctypes.data), self.h.h)
        vals = buf.view(np.complex128)
        tensors, at = [], 0
        for k in range(n):
            a, c = int(bond[k]), int(bond[k + 1])
            tensors.append(vals[at:at + 2 * a * c].reshape(a, 2, c).copy())
            at += 2 * a * c
        return MPSState(tuple(tensors), int(centre.value), tuple(int(q) for q in qubit_at))

    def autotune(self, n_layers, candidates=(8, 16, 24, 32), scratch=None) -> dict:
        """Time the QR panel widths over the next n_layers steps (state
        restored after each) and keep the fastest; returns the timings."""
        import torch
        if scratch is None:
            scratch = torch.empty(self.workspace.numel(), dtype=torch.uint8,
                                  device=self.workspace.device)
        cand = np.asarray(candidates, dtype=np.uint32)
        ms = np.zeros(len(cand))
        fl = np.zeros(len(cand))
        chosen = C.c_uint32()
        _check(load().tepai_batch_autotune(self.b, n_layers, cand.ctypes.data, len(cand),
                                           C.c_void_p(scratch.data_ptr()), scratch.numel(),
                                           ms.ctypes.data, fl.ctypes.data, C.byref(chosen)),
               self.h.h)
        return {"chosen": int(chosen.value), "candidates": [int(c) for c in cand],
                "ms": ms.tolist(), "nominal_flops": fl.tolist()}

    def capture_step(self, n_layers, d_values, d_weights, d_mean, d_se) -> "StepGraph":
        """Record evolve(n_layers) + observe + reduce once as a HIP graph."""
        g = _P()
        _check(load().tepai_batch_capture_step(
            self.b, n_layers, C.c_void_p(d_values.data_ptr()), C.c_void_p(d_weights.data_ptr()),
            C.c_void_p(d_mean.data_ptr()), C.c_void_p(d_se.data_ptr()), C.byref(g)), self.h.h)
        return StepGraph(self, g, (d_values, d_weights, d_mean, d_se))

    def close(self):
        if self.b:
            load().tepai_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StepGraph:
    """A captured read-out step; keeps its batch and buffers alive."""

    def __init__(self, batch, g, buffers):
        self.batch, self.g, self.buffers = batch, g, buffers

    def launch(self) -> None:
        _check(load().tepai_step_graph_launch(self.g), self.batch.h.h)

    def close(self):
        if self.g:
            load().tepai_step_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tepai_batch_create(h, ps, first, count, workspace=None, stream=None) -> Batch:
    return Batch(h, ps, first, count, workspace, stream)


def tepai_batch_evolve(b: Batch, n_layers: int) -> None:
    b.evolve(n_layers)


def tepai_batch_observe(b: Batch, d_values, d_weights) -> None:
    b.observe(d_values, d_weights)


def tepai_batch_stats(b: Batch) -> np.ndarray:
    return b.stats()


def tepai_batch_read_mps(b: Batch, slot: int) -> MPSState:
    return b.read_mps(slot)


def tepai_batch_destroy(b: Batch) -> None:
    b.close()


def tepai_reduce(h: Handle, count: int, n_obs: int, d_values, d_weights, d_mean, d_se,
                 stream=None) -> None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load().tepai_reduce(h.h, count, n_obs, C.c_void_p(d_values.data_ptr()),
                               C.c_void_p(d_weights.data_ptr()), C.c_void_p(d_mean.data_ptr()),
                               C.c_void_p(d_se.data_ptr()), C.c_void_p(s.cuda_stream)), h.h)


def tepai_run(h: Handle, ps: ProblemStruct, batch: int = 0, want_values: bool = True,
              want_stats: bool = True):
    """Synchronous estimator; returns dict(mean, std_err, weights, values, stats).

    On TEPAI_ENUMERIC the library has still written every output: the raised
    TepaiError carries them as ``.result``."""
    p = ps.struct
    ns, no = int(p.n_samples), int(p.n_obs)
    mean = np.zeros(no)
    se = np.zeros(no)
    w = np.zeros(ns)
    vals = np.zeros((ns, no)) if want_values else None
    st_arr = (tepai_sample_stats * ns)() if want_stats else None
    st = load().tepai_run(h.h, ps.ref(), batch, _ptr(mean), _ptr(se), _ptr(w),
                          _ptr(vals) if vals is not None else None, st_arr)
    if st not in (TEPAI_OK, TEPAI_ENUMERIC):
        _check(st, h.h)
    stats = None
    if st_arr is not None:
        stats = np.zeros(ns, STATS_DTYPE)
        for i in range(ns):
            for f in STATS_FIELDS:
                stats[f][i] = getattr(st_arr[i], f)
    out = dict(mean=mean, std_err=se, weights=w, values=vals, stats=stats)
    if st == TEPAI_ENUMERIC:
        err = TepaiError(st, (load().tepai_last_error(h.h) or b"").decode())
        err.result = out
        raise err
    return out


NOALLOC_BYTES = 256 << 20


def tepai_run_noalloc(h: Handle, ps: ProblemStruct, d_mean, d_se, d_weights, d_values,
                      stream=None, want_stats: bool = True):
    """The estimator in the library's fixed device array (no device
    allocation); outputs go to the given device tensors.  Returns the
    per-sample stats (or None).  TEPAI_ENUMERIC raises TepaiError with
    ``.result`` = the stats, the device outputs being written."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    ns = int(ps.struct.n_samples)
    st_arr = (tepai_sample_stats * ns)() if want_stats else None
    st = load().tepai_run_noalloc(h.h, ps.ref(), C.c_void_p(s.cuda_stream),
                                  C.c_void_p(d_mean.data_ptr()), C.c_void_p(d_se.data_ptr()),
                                  C.c_void_p(d_weights.data_ptr()),
                                  C.c_void_p(d_values.data_ptr()), st_arr)
    if st not in (TEPAI_OK, TEPAI_ENUMERIC):
        _check(st, h.h)
    stats = None
    if st_arr is not None:
        stats = np.zeros(ns, STATS_DTYPE)
        for i in range(ns):
            for f in STATS_FIELDS:
                stats[f][i] = getattr(st_arr[i], f)
    if st == TEPAI_ENUMERIC:
        err = TepaiError(st, (load().tepai_last_error(h.h) or b"").decode())
        err.result = stats
        raise err
    return stats
