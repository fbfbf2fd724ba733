"""Throughput of batched MPS TE-PAI on one MI355X.

Workload: the n = 64 disordered XXZ ring (J_xy = 1, J_z = 0.5,
h_i ~ U[-2, 2]), T = 3, N = 800 Trotter steps, Delta = pi/256, bond cap
chi = 128, Neel start, observables <Z_i> for all i and <Z_0 Z_32>, complex128.

A step is one pass of the whole hot path over one batch of B samples held
in HBM: every sample draws its gate settings for the next J Trotter steps
(fused sampler), applies them to its MPS (single-site gates, truncated
two-site updates with Jacobi SVD, centre shifts, SWAP routing of the wrap
bond), then the batch reads out all observables at the reached time and the
weighted FP64 reduction forms the estimator for that time.

Two paths run the same samples: the batched mixed-precision path (complex64
site tensors, FP32 matrix-core contractions, FP64 QR / Jacobi / truncation /
estimator), whose rate is the reported value, and the plain FP64 path, whose
rate, the ratios and the largest per-sample difference between the two are
reported beside it.

A full sample is N = 800 Trotter steps; one step processes B * J / N sample
equivalents (J = 4 Trotter steps per step by default), so value =
B * K * J / N / t over K timed steps.  The timed window always starts at
Trotter step --start-step (96): the warm-up is max(--warmup, 96 / J) steps,
so the requested warm-up is a minimum and the window does not move with it.
By step 96 every sample of both paths has reached the bond cap chi = 128
(the FP64 path by step ~32, the mixed path, whose singular-value floor is
1e-7, by step ~90).  Later steps cost somewhat more again as the Schmidt
spectra flatten (about +20% per step from step 96 to step 320), so the value
is the rate of the saturated regime at this window, not a bound for the
whole circuit.

The plain FP64 path is timed on the first --fp64-steps (4) steps of the same
window only; the ratios mixed_over_plain (samples/s), ..._per_sum_chi3 and
..._per_nominal_flop compare the two paths over those same Trotter steps,
and the per-sample difference between the paths is taken there too.  The
CPU baseline times the oracle's own two-site update and centre shift at
bond 128 on the host's cores and applies them to the window's per-sample
work (``cpu_baseline_saturated``).
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (and FP64 MFMA), dense
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "evolve_kernel_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_13144_amd", "csrc", "kernels.hip"),
                  os.path.join(ROOT, "paper_2604_13144_amd", "build.py")]


def kernel_source_sha256() -> str:
    """Hash of the kernel source and of the build script that holds its flags."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM-side bytes per launch of the mixed evolve kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (calibrated by a 1 GiB copy), or
    None when the kernel source or its build flags have changed since the
    counters were taken."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        sha = kernel_source_sha256()
    except OSError:
        return None
    return rec["traffic_bytes_per_launch"] if rec.get("source_sha256") == sha else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed steps before the timed ones; the throughput workload "
                         "always warms up to at least Trotter step --start-step")
    ap.add_argument("--batch", type=int, default=None,
                    help="samples resident at once (default 256, one per CU; the hybrid "
                         "workload 768, so that CUs done with a small-cap sample take another)")
    ap.add_argument("--layers-per-step", type=int, default=4)
    ap.add_argument("--start-step", type=int, default=96,
                    help="throughput workload: first Trotter step of the timed window (both "
                         "paths have every bond at the cap by then)")
    ap.add_argument("--fp64-steps", type=int, default=4,
                    help="throughput workload: timed steps of the plain FP64 path (the first "
                         "ones of the mixed path's window)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", default="",
                    help="throughput workload: comma list of QR panel widths to time at the "
                         "start of the window (tepai_batch_autotune); the fastest is kept")
    ap.add_argument("--paths", default="mixed,fp64",
                    help="comma list of paths to time (the first one gives value)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (counter calibration) and exit")
    ap.add_argument("--workload", choices=("throughput", "truncation", "hybrid", "batching"),
                    default="throughput",
                    help="truncation: the chi = 2 vs 16 robustness experiment; hybrid: "
                         "Trotter-then-TE-PAI on the n = 100 ring (use --layers-per-step 32 "
                         "--warmup 4); batching: the n = 64 ring with caps 32/64/128 by "
                         "sample, 2048 samples in one batch (mixed path); default: the "
                         "throughput step")
    ap.add_argument("--t0", type=float, default=0.5,
                    help="hybrid workload: length of the Trotter segment")
    ap.add_argument("--pre-cap", type=int, default=32,
                    help="hybrid workload: bond cap of the Trotter segment; samples whose "
                         "cap is smaller truncate their copy of its state")
    ap.add_argument("--hybrid-precision", choices=("mixed", "fp64"), default="mixed",
                    help="hybrid workload: precision of the TE-PAI samples")
    ap.add_argument("--no-pi", action="store_true",
                    help="hybrid workload: the biased variant without pi rotations")
    ap.add_argument("--cycle-caps", action="store_true",
                    help="hybrid workload: caps 16, 32, 64 in turn instead of by thirds")
    ap.add_argument("--read-every", type=int, default=100,
                    help="truncation workload: Trotter steps between read-outs")
    ap.add_argument("--per-gate", action="store_true",
                    help="truncation workload: one truncated update per sampled gate "
                         "(TEPAI_PER_GATE) instead of one per same-pair run")
    ap.add_argument("--work-queue", action="store_true",
                    help="batching and hybrid workloads: evolve on one workgroup per CU "
                         "taking samples from a counter (TEPAI_WORK_QUEUE) instead of one "
                         "workgroup per sample")
    ap.add_argument("--delta-log2", type=int, default=12,
                    help="truncation workload: PAI angle Delta = pi / 2^k")
    return ap.parse_args()


def copy_probe(mib: int):
    """One plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counter
    readings calibrate those counters against bytes actually moved."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}))


def workload(batch):
    import tepai_inputs as ti
    return ti.config(4).with_(n_samples=max(batch, 1))


# ----------------------------------------------------------- CPU baseline
def _oracle_worker(args):
    sample, seconds, kind = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np  # noqa: F401
    from oracle import pai
    from oracle.mps import MPS
    from oracle.sampler import sample_circuit
    from oracle.schedule import build_schedule
    p = workload(1) if kind == "throughput" else hybrid_segment(16, False)
    t = pai.build_table(p)
    circ = sample_circuit(p, t, sample)
    chi = p.chi_max if p.chi_per_sample is None else p.chi_per_sample[sample]
    ops, _ = build_schedule(p, t, circ, chi)
    # layer boundaries in the op list: count ops until the time budget ends
    m = MPS(p.initial_bits, p.svd_cutoff)
    t0 = time.perf_counter()
    done_ops = 0
    for op in ops:
        m.run([op])
        done_ops += 1
        if time.perf_counter() - t0 > seconds:
            break
    el = time.perf_counter() - t0
    frac_updates = (m.stats.updates + m.stats.shifts) / max(1, sum(1 for o in ops if o[0] != "local"))
    return frac_updates, el, m.stats.updates, max(m.bonds())


def host_cores():
    """Worker processes for the oracle: the cores this process may run on,
    at most 16 (the host CPU share that comes with one GPU)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return min(avail, 16), avail, os.cpu_count()


def cpu_baseline(seconds: float, kind: str = "throughput"):
    cores, avail, nproc = host_cores()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(s, seconds, kind) for s in range(cores)])
    frac = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return {"value": frac / wall, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "host_cpus": {"affinity": avail, "nproc": nproc},
            "sample": (f"{cores} samples of the same workload, one per process (OMP 1 thread), "
                       f"each run from t=0 for {seconds:.0f} s; fraction of each sample's "
                       f"two-site updates and shifts done, summed, over wall time "
                       f"(max bond reached {max(r[3] for r in res)}; early steps are cheaper, "
                       f"so this favours the CPU)")}


def _saturated_worker(args):
    """Time the oracle's two-site update and centre shift at bond 128 (the
    saturated regime of the timed window) for about `seconds` seconds."""
    seconds, chi, seed = args
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy as np
    from oracle.mps import MPS
    from oracle.schedule import setting_operator
    rng = np.random.default_rng(seed)

    def rand_site():
        return rng.standard_normal((chi, 2, chi)) + 1j * rng.standard_normal((chi, 2, chi))

    m = MPS("000", 1e-12)
    m.A = [rand_site(), rand_site(), rand_site()]
    m.centre = 1
    gates = [setting_operator(ps, 0.01, math.pi / 256, 1) for ps in ("XX", "YY", "ZZ")]
    t_upd, n_upd = 0.0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.8 * seconds:
        g = gates[n_upd % 3]
        ts = time.perf_counter()
        if m.centre == 1 and n_upd % 2 == 0:
            m.update(0, g, chi, right=True)        # centre ends on site 1
        else:
            m.update(1, g, chi, right=False)       # centre ends on site 1
        t_upd += time.perf_counter() - ts
        n_upd += 1
    t_sh, n_sh = 0.0, 0
    while time.perf_counter() - t0 < seconds:
        ts = time.perf_counter()
        if m.centre == 1:
            m.shift(1, +1)
        else:
            m.shift(2, -1)
        t_sh += time.perf_counter() - ts
        n_sh += 1
    return t_upd / n_upd, t_sh / max(n_sh, 1), n_upd, n_sh


def cpu_baseline_saturated(seconds, updates_per_sample, shifts_per_sample, window_fraction,
                           chi=128):
    """The oracle on the timed window's work: every host process times the
    oracle's own two-site update (contraction, LAPACK SVD of the 2 chi x 2 chi
    matrix, truncation to chi) and centre shift at bond chi; the window's
    per-sample update and shift counts (identical on every path: the
    schedule does not depend on precision) turn those times into the time
    the oracle needs per sample for the window, and samples/s follows."""
    cores, avail, nproc = host_cores()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_saturated_worker, [(seconds, chi, 100 + i) for i in range(cores)])
    t_u = sum(r[0] for r in res) / len(res)
    t_s = sum(r[1] for r in res) / len(res)
    per_sample_window = updates_per_sample * t_u + shifts_per_sample * t_s
    value = cores * window_fraction / per_sample_window
    return {"value": value, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "host_cpus": {"affinity": avail, "nproc": nproc},
            "seconds_per_update": t_u, "seconds_per_shift": t_s,
            "sample": (f"oracle two-site update (einsum contraction, numpy/LAPACK SVD of "
                       f"{2 * chi}x{2 * chi} complex128, truncation to {chi}) and centre shift "
                       f"timed at bond {chi} for {seconds:.0f} s in each of {cores} processes "
                       f"(OMP 1 thread; {sum(r[2] for r in res)} updates, "
                       f"{sum(r[3] for r in res)} shifts), applied to the timed window's "
                       f"per-sample work ({updates_per_sample:.0f} updates, "
                       f"{shifts_per_sample:.0f} shifts, all at the cap), one sample per process")}


# ----------------------------------------------------------------- GPU run
def run_path(L, h, p, precision, J, K, W, B, match=None, autotune=None, work_queue=False):
    """W warm-up and K timed steps of one precision path on a fresh batch.

    ``match`` (<= K): also report the rate over the first ``match`` timed
    steps, the window the other path is timed on.  ``autotune`` (a tuple of
    QR panel widths): after the warm-up, time each over the next J steps
    (state restored after each) and keep the fastest for the timed steps."""
    import numpy as np
    import torch
    dev = torch.device("cuda", 0)
    ps = L.ProblemStruct(p, precision=precision, work_queue=work_queue)
    stream = torch.cuda.current_stream(dev)
    b = L.Batch(h, ps, 0, B, stream=stream)
    n_obs = ps.n_obs
    vals = torch.empty(B * n_obs, dtype=torch.float64, device=dev)
    wts = torch.empty(B, dtype=torch.float64, device=dev)
    mean = torch.empty(n_obs, dtype=torch.float64, device=dev)
    se = torch.empty(n_obs, dtype=torch.float64, device=dev)
    name = "mixed" if precision == L.TEPAI_FP32_MIXED else "fp64"

    def step(events=None):
        # the events sit on the stream the library launches on
        if events is not None:
            events[0].record(stream)
        b.evolve(J)
        if events is not None:
            events[1].record(stream)
        b.observe(vals, wts)
        L.tepai_reduce(h, B, n_obs, vals, wts, mean, se, stream)

    for i in range(W):
        t0 = time.time()
        step()
        torch.cuda.synchronize()
        print(f"[bench] {name} warmup step {i + 1}/{W}: {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    tuning = None
    if autotune:
        tuning = b.autotune(J, candidates=autotune)
        print(f"[bench] {name} autotune: {tuning}", file=sys.stderr, flush=True)
    fields = ("n_gates", "updates", "shifts", "nominal_flops", "jacobi_sweeps", "sum_chi3")
    s0 = b.stats()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    walls = []
    s_match = None
    t0 = time.perf_counter()
    for i in range(K):
        ts = time.perf_counter()
        step(evs[i])
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - ts)
        if match is not None and i + 1 == match:
            s_match = b.stats()
            v_match, m_match = vals.cpu().numpy().reshape(B, n_obs), mean.cpu().numpy()
        print(f"[bench] {name} timed step {i + 1}/{K}: {walls[-1]:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = b.stats()
    ms = [e0.elapsed_time(e1) for e0, e1 in evs]

    def delta(a, c):
        return {f: float(np.sum(c[f].astype(np.float64) - a[f].astype(np.float64))) for f in fields}

    d = delta(s0, s1)
    evolve_ms = sum(ms)
    out = {
        "value": B * K * J / p.trotter_steps / wall,
        "wall": wall,
        "ms_per_step": wall / K * 1e3,
        "gates_per_s": d["n_gates"] / wall,
        "updates_per_s": d["updates"] / wall,
        "sum_chi3_per_s": d["sum_chi3"] / wall,
        "mean_max_bond": float(np.mean(s1["max_bond"])),
        "sweeps": d["jacobi_sweeps"] / max(1.0, d["updates"] + d["shifts"]),
        "achieved": d["nominal_flops"] / (evolve_ms / 1e3) / 1e12,
        "kernel_ms_per_launch": evolve_ms / K,
        "flops_per_launch": d["nominal_flops"] / K,
        "updates_per_sample": d["updates"] / B,
        "shifts_per_sample": d["shifts"] / B,
        "sum_chi3_per_sample": d["sum_chi3"] / B,
        "values": vals.cpu().numpy().reshape(B, n_obs),
        "mean": mean.cpu().numpy(),
        "autotune": tuning,
    }
    if s_match is not None:
        dm = delta(s0, s_match)
        wm = sum(walls[:match])
        out["match"] = {"steps": match, "value": B * match * J / p.trotter_steps / wm,
                        "sum_chi3_per_s": dm["sum_chi3"] / wm,
                        "tflops": dm["nominal_flops"] / (sum(ms[:match]) / 1e3) / 1e12,
                        "values": v_match, "mean": m_match}
    return out


def truncation_experiment(L, h, read_every, delta_log2=12, per_gate=False):
    """The truncation-robustness experiment on the GPU (FP64 path).

    For each method (the deterministic product formula, one circuit; TE-PAI,
    N_s = 100 circuits) and bond cap chi in {2, 16}, every sample runs the
    n = 20, J = 1 ring to T = 1 (N = 2000) and the estimator of X_i, Y_i, Z_i
    on every qubit is read out every `read_every` steps.  The truncation error
    of a method at time t is the mean over the 60 observables of
    |<O>_{chi=2}(t) - <O>_{chi=16}(t)|; TE-PAI runs the same circuits at both
    caps (the sampler does not depend on chi), so the difference holds no
    sampling noise between the two caps.
    """
    import numpy as np
    import torch
    import tepai_inputs as ti
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    out = {}
    for method in ("trotter", "tepai"):
        for chi in (2, 16):
            p = ti.truncation_workload(chi, trotter=method == "trotter",
                                       delta=math.pi / 2 ** delta_log2, per_gate=per_gate)
            if read_every < 1 or p.trotter_steps % read_every:
                raise SystemExit("--read-every must divide N = %d" % p.trotter_steps)
            ps = L.ProblemStruct(p)
            B, n_obs = p.n_samples, ps.n_obs
            b = L.Batch(h, ps, 0, B, stream=stream)
            vals = torch.empty(B * n_obs, dtype=torch.float64, device=dev)
            wts = torch.empty(B, dtype=torch.float64, device=dev)
            mean = torch.empty(n_obs, dtype=torch.float64, device=dev)
            se = torch.empty(n_obs, dtype=torch.float64, device=dev)
            series, errs, steps, xs = [], [], [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j in range(read_every, p.trotter_steps + 1, read_every):
                b.evolve(read_every)
                b.observe(vals, wts)
                L.tepai_reduce(h, B, n_obs, vals, wts, mean, se, stream)
                series.append(mean.cpu().numpy())
                x = vals.view(B, n_obs) * wts.view(B, 1)          # weighted sample values
                xs.append(x.cpu().numpy())
                errs.append(se.cpu().numpy())
                steps.append(j)
                print(f"[bench] truncation {method} chi={chi}: step {j}/{p.trotter_steps}",
                      file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = b.stats()
            out[(method, chi)] = {"mean": np.array(series), "std_err": np.array(errs),
                                  "x": np.array(xs),
                                  "steps": steps, "wall_s": wall, "T": p.total_time,
                                  "N": p.trotter_steps,
                                  "gates_per_sample": float(np.mean(st["n_gates"])),
                                  "updates_per_sample": float(np.mean(st["updates"])),
                                  "max_bond": int(np.max(st["max_bond"])),
                                  "discarded_per_sample": float(np.mean(st["discarded"]))}
            print(f"[bench] truncation {method} chi={chi}: {wall:.1f} s", file=sys.stderr, flush=True)
            b.close()
    r = out[("trotter", 2)]
    times = [j * r["T"] / r["N"] for j in r["steps"]]

    def trunc_err(method):
        return np.mean(np.abs(out[(method, 2)]["mean"] - out[(method, 16)]["mean"]), axis=1)

    et, ep = trunc_err("trotter"), trunc_err("tepai")
    ref = out[("trotter", 16)]["mean"]
    tepai2_vs_ref = np.mean(np.abs(out[("tepai", 2)]["mean"] - ref), axis=1)
    gap16 = np.mean(np.abs(out[("tepai", 16)]["mean"] - ref), axis=1)
    se16 = np.mean(out[("tepai", 16)]["std_err"], axis=1)
    # cancellation across the ensemble: error of the mean over the mean of the
    # per-sample errors of the weighted values w_s <O>_s (1 = no cancellation)
    dx = out[("tepai", 2)]["x"] - out[("tepai", 16)]["x"]          # [t, s, o]
    per_sample = np.mean(np.abs(dx), axis=(1, 2))
    of_mean = np.mean(np.abs(np.mean(dx, axis=1)), axis=1)
    return {
        "workload": "truncation: n=20 ring J=1 omega~U[-1,1], T=1, N=2000, Delta=pi/2^%d, "
                    "N_s=100, start |+..+-+..+>, X/Y/Z of every qubit, chi in {2,16}, %s"
                    % (delta_log2, "one truncated update per gate" if per_gate
                       else "one truncated update per same-pair run"),
        "dtype": "f64",
        "data": "synthetic",
        "times": times,
        "trotter_truncation_error": et.tolist(),
        "tepai_truncation_error": ep.tolist(),
        "tepai_below_trotter_fraction": float(np.mean(ep < et)),
        "mean_error_ratio_tepai_over_trotter": float(np.mean(ep) / np.mean(et)),
        "tepai_chi2_vs_trotter_chi16": tepai2_vs_ref.tolist(),
        "tepai_chi16_vs_trotter_chi16": gap16.tolist(),
        "tepai_chi16_mean_std_err": se16.tolist(),
        "tepai_per_sample_truncation_error": per_sample.tolist(),
        "tepai_cancellation_ratio": (of_mean / np.maximum(per_sample, 1e-300)).tolist(),
        "runs": {f"{m}_chi{c}": {k: v for k, v in d.items() if k not in ("mean", "std_err", "steps", "x")}
                 for (m, c), d in out.items()},
    }


def hybrid_segment(n_samples, no_pi, initial_mps=None, cycled=False):
    """The TE-PAI segment of the combined long-time configuration: the n = 100
    Heisenberg ring (h ~ U[-1,1]), T = 2, N = 1024, Delta = pi/512, bond caps
    64, 32 and 16 for the first, second and last third of the samples, <Z_i>
    and the half-ring sum of Z_i Z_{i+1}.  The library starts the samples by
    decreasing cap whatever their order, so the longest work starts first
    and the small-cap samples fill the CUs that free up."""
    import tepai_inputs as ti
    if cycled:      # 16, 32, 64 in turn (for comparison)
        caps = tuple((16, 32, 64)[s % 3] for s in range(n_samples))
    else:
        caps = tuple((64, 32, 16)[min(2, 3 * s // n_samples)] for s in range(n_samples))
    return ti.config(5).with_(n_samples=n_samples, chi_per_sample=caps, no_pi=no_pi,
                              initial_mps=initial_mps)


def hybrid_experiment(L, h, a):
    """Trotter-then-TE-PAI on the GPU (sec. "Implementation"): a deterministic
    product-formula segment of one sample to t0 (TEPAI_TROTTER, bond cap 16,
    N(t0) steps of the first-order reference rule), its MPS read back, then
    a batch of TE-PAI samples (or the biased no-pi variant) continuing from
    that shared state with per-sample caps 16/32/64.  W windows of J steps
    warm the batch up, K windows are timed; every window ends with a
    read-out and the weighted reduction (time series of the estimate)."""
    import numpy as np
    import torch
    import tepai_inputs as ti
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    t0_time = a.t0
    n0 = ti.trotter_steps_for(t0_time)
    pre = ti.config(5).with_(trotter=True, total_time=t0_time, trotter_steps=n0,
                             n_samples=1, chi_max=a.pre_cap)
    bt = L.Batch(h, L.ProblemStruct(pre), 0, 1, stream=stream)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    step = max(1, n0 // 10)
    for j in range(0, n0, step):
        bt.evolve(min(step, n0 - j))
        torch.cuda.synchronize()
        print(f"[bench] hybrid Trotter segment: step {min(j + step, n0)}/{n0}", file=sys.stderr, flush=True)
    prep_s = time.perf_counter() - tp
    shared = bt.read_mps(0)
    prep_stats = bt.stats()
    bt.close()
    B, J, K, W = a.batch or 4096, a.layers_per_step, a.steps, a.warmup
    p = hybrid_segment(B, a.no_pi, shared, a.cycle_caps)
    if (W + K) * J > p.trotter_steps:
        raise SystemExit("warmup + steps exceed the circuit")
    precision = L.TEPAI_FP32_MIXED if a.hybrid_precision == "mixed" else L.TEPAI_FP64
    ps = L.ProblemStruct(p, precision=precision, work_queue=a.work_queue)
    b = L.Batch(h, ps, 0, B, stream=stream)
    n_obs = ps.n_obs
    vals = torch.empty(B * n_obs, dtype=torch.float64, device=dev)
    wts = torch.empty(B, dtype=torch.float64, device=dev)
    mean = torch.empty(n_obs, dtype=torch.float64, device=dev)
    se = torch.empty(n_obs, dtype=torch.float64, device=dev)
    series = []
    s0 = None
    evolve_ms, t_timed = 0.0, 0.0
    for i in range(W + K):
        timed = i >= W
        if timed and s0 is None:
            torch.cuda.synchronize()
            s0 = b.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        tw = time.perf_counter()
        e0.record(stream)
        b.evolve(J)
        e1.record(stream)
        b.observe(vals, wts)
        L.tepai_reduce(h, B, n_obs, vals, wts, mean, se, stream)
        torch.cuda.synchronize()
        if timed:
            t_timed += time.perf_counter() - tw
            evolve_ms += e0.elapsed_time(e1)
        m, e = mean.cpu().numpy(), se.cpu().numpy()
        t_now = t0_time + (i + 1) * J * p.total_time / p.trotter_steps
        series.append([round(t_now, 6), float(m[0]), float(e[0]), float(m[-1]), float(e[-1])])
        print(f"[bench] hybrid TE-PAI window {i + 1}/{W + K}{' (timed)' if timed else ''}: "
              f"{time.perf_counter() - tw:.1f} s", file=sys.stderr, flush=True)
    s1 = b.stats()
    b.close()
    d = {f: float(np.sum(s1[f].astype(np.float64) - s0[f].astype(np.float64)))
         for f in ("n_gates", "updates", "nominal_flops")}
    achieved = d["nominal_flops"] / (evolve_ms / 1e3) / 1e12
    line = {
        "metric": "TE-PAI MPS samples/s from a shared Trotter state (hybrid), n=100 ring, chi 64/32/16",
        "value": B * K * J / p.trotter_steps / t_timed,
        "unit": "samples/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": t_timed / K * 1e3,
        "higher_is_better": True,
        "dtype": ("mixed: c64 storage, f32 MFMA contractions, f64 QR/Jacobi/truncation/estimator"
                  if precision == L.TEPAI_FP32_MIXED else "f64"),
        "data": "synthetic",
        "variant": "no_pi (biased, Statement 3)" if a.no_pi else "unbiased TE-PAI",
        "config": {"workload": "hybrid: n=100 Heisenberg ring h~U[-1,1]; Trotter segment to "
                               f"t0={t0_time:g} (N0={n0}, chi={a.pre_cap}) on the GPU, then TE-PAI "
                               "T=2, N=1024, Delta=pi/512, caps " + ("16/32/64 in turn" if a.cycle_caps else "64/32/16 by thirds") + " (a cap below the shared state's bonds truncates its copy), Neel start of the segment",
                   "batch_samples": B, "trotter_steps_per_step": J,
                   "timed_trotter_steps": [W * J, (W + K) * J],
                   "schedule": ("work queue, one workgroup per CU" if a.work_queue
                                else "one workgroup per sample")},
        "trotter_segment": {"seconds": prep_s, "steps": n0, "updates": int(prep_stats["updates"][0]),
                            "max_bond": int(prep_stats["max_bond"][0]),
                            "shared_state_bonds_max": max(shared.bonds())},
        "gates_per_s": d["n_gates"] / t_timed,
        "updates_per_s": d["updates"] / t_timed,
        "series_t_Z0_se_halfZZ_se": series,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "%s<2, %s>" % ("evolve_queue_kernel" if a.work_queue else "evolve_kernel",
                                               "true" if precision == L.TEPAI_FP32_MIXED else "false"),
                     "kernel_ms_per_launch": evolve_ms / K,
                     "flops_per_launch": d["nominal_flops"] / K},
    }
    if not a.no_cpu_baseline:
        cb = cpu_baseline(a.cpu_seconds, "hybrid")
        cb["sample"] = cb["sample"].replace("the same workload", "the TE-PAI segment").replace(
            "from t=0", "from the Neel product state (the oracle does not take the GPU's shared state)")
        line["cpu_baseline"] = cb
    return line


def batching_experiment(L, h, a):
    """The batching configuration at scale: the n = 64 XXZ ring of the
    throughput workload with bond caps 32, 64 and 128 by sample index mod 3,
    B samples (default 2048, eight per CU) resident in one batch on the
    mixed path.  One workgroup runs one sample; the library launches the
    slots by decreasing cap, and a CU that finishes a small-cap sample takes
    the next slot, so the hardware scheduler packs the uneven work
    (--work-queue: one workgroup per CU takes the slots from a counter in
    the same order instead).  The
    timed window starts at Trotter step --start-step (96) as in the
    throughput step; value = B K J / N / t as there."""
    import tepai_inputs as ti
    B = a.batch or 2048
    J, K = a.layers_per_step, a.steps
    W = max(a.warmup, -(-a.start_step // J))
    base = ti.config(3)
    p = base.with_(n_samples=B, chi_per_sample=base.chi_per_sample[:B])
    if (W + K) * J > p.trotter_steps:
        raise SystemExit("warmup + steps exceed the circuit")
    r = run_path(L, h, p, L.TEPAI_FP32_MIXED, J, K, W, B, work_queue=a.work_queue)
    kernel = ("evolve_queue_kernel<4, true> (mixed, work queue)" if a.work_queue
              else "evolve_kernel<4, true> (mixed)")
    return {
        "metric": "TE-PAI MPS samples/s, n=64 XXZ ring, caps 32/64/128 by sample (batching)",
        "value": r["value"],
        "unit": "samples/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "dtype": "mixed: c64 storage, f32 MFMA contractions, f64 QR/Jacobi/truncation/estimator",
        "data": "synthetic",
        "config": {"workload": "batching: n=64 XXZ ring J_xy=1 J_z=0.5 h~U[-2,2], T=3, N=800, "
                               "Delta=pi/256, caps (32, 64, 128)[s mod 3], Neel, <Z_i> all i + "
                               "<Z_0 Z_32>",
                   "batch_samples": B, "trotter_steps_per_step": J,
                   "timed_trotter_steps": [W * J, (W + K) * J],
                   "schedule": ("work queue, one workgroup per CU" if a.work_queue
                                else "one workgroup per sample")},
        "gates_per_s": r["gates_per_s"],
        "updates_per_s": r["updates_per_s"],
        "sum_chi3_per_s": r["sum_chi3_per_s"],
        "jacobi_sweeps_per_factorisation": r["sweeps"],
        "sum_chi3_per_sample_in_window": r["sum_chi3_per_sample"],
        "roofline": {"bound": "alu", "achieved": r["achieved"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": r["achieved"] / FP64_PEAK_TFLOPS,
                     "traffic": None, "kernel": kernel,
                     "kernel_ms_per_launch": r["kernel_ms_per_launch"],
                     "flops_per_launch": r["flops_per_launch"]},
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.workload == "hybrid":
        import torch
        torch.cuda.init()
        from paper_2604_13144_amd import _lib as L
        print(json.dumps(hybrid_experiment(L, L.Handle(0), a)))
        return
    if a.workload == "batching":
        import torch
        torch.cuda.init()
        from paper_2604_13144_amd import _lib as L
        print(json.dumps(batching_experiment(L, L.Handle(0), a)))
        return
    if a.workload == "truncation":
        import torch
        torch.cuda.init()
        from paper_2604_13144_amd import _lib as L
        print(json.dumps(truncation_experiment(L, L.Handle(0), a.read_every, a.delta_log2,
                                               a.per_gate)))
        return
    import numpy as np
    import torch
    torch.cuda.init()          # torch's HIP context first, then the library's handle
    from paper_2604_13144_amd import _lib as L

    B = a.batch or 256
    p = workload(B)
    J, K = a.layers_per_step, a.steps
    # the timed window starts at a fixed saturated Trotter step whatever the
    # requested warm-up: --warmup is a minimum
    W = max(a.warmup, -(-a.start_step // J))
    if (W + K) * J > p.trotter_steps:
        raise SystemExit("warmup + steps exceed the circuit")
    Kp = min(K, a.fp64_steps)
    h = L.Handle(0)
    paths = a.paths.split(",")
    tune = tuple(int(x) for x in a.autotune.split(",") if x) or None
    mixed = (run_path(L, h, p, L.TEPAI_FP32_MIXED, J, K, W, B, match=Kp, autotune=tune)
             if "mixed" in paths else None)
    plain = run_path(L, h, p, L.TEPAI_FP64, J, Kp, W, B, autotune=tune) if "fp64" in paths else None
    if mixed is None or plain is None:
        # one path only (profiling runs): report it alone
        r = mixed or plain
        print(json.dumps({"path": "mixed" if mixed else "fp64", "value": r["value"], "unit": "samples/s",
                          "autotune": r["autotune"],
                          "kernel_ms_per_launch": r["kernel_ms_per_launch"],
                          "flops_per_launch": r["flops_per_launch"],
                          "achieved_tflops": r["achieved"],
                          "timed_trotter_steps": [W * J, (W + (K if mixed else Kp)) * J]}))
        return
    # accuracy at the same Trotter step: the mixed read-out after its first Kp
    # timed steps against the FP64 read-out at the end of its window
    mm = mixed["match"]
    err = float(np.max(np.abs(mm["values"] - plain["values"])))
    est_err = float(np.max(np.abs(mm["mean"] - plain["mean"])))
    traffic = measured_traffic()
    line = {
        "metric": "TE-PAI MPS samples/s at n=64, chi=128 (batched mixed vs plain FP64) at fixed err",
        "value": mixed["value"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "warmup_requested": a.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed: c64 storage, f32 MFMA contractions, f64 QR/Jacobi/truncation/estimator",
        "data": "synthetic",
        "config": {"workload": "xxz_ring_n64_chi128: n=64 XXZ ring J_xy=1 J_z=0.5 h~U[-2,2], "
                               "T=3, N=800, Delta=pi/256, chi=128, Neel, <Z_i> all i + <Z_0 Z_32>",
                   "batch_samples": B, "trotter_steps_per_step": J,
                   "timed_trotter_steps": [W * J, (W + K) * J],
                   "path": "batched mixed precision (one workgroup per sample, fused sampler)"},
        "gates_per_s": mixed["gates_per_s"],
        "updates_per_s": mixed["updates_per_s"],
        "sum_chi3_per_s": mixed["sum_chi3_per_s"],
        "mean_max_bond": mixed["mean_max_bond"],
        "jacobi_sweeps_per_factorisation": mixed["sweeps"],
        "autotune": ({"mixed": mixed["autotune"], "fp64": plain["autotune"]}
                     if mixed["autotune"] else None),
        "plain_fp64": {"value": plain["value"], "unit": "samples/s", "dtype": "c128 (f64)",
                       "steps": Kp, "timed_trotter_steps": [W * J, (W + Kp) * J],
                       "ms_per_step": plain["ms_per_step"], "gates_per_s": plain["gates_per_s"],
                       "sum_chi3_per_s": plain["sum_chi3_per_s"],
                       "jacobi_sweeps_per_factorisation": plain["sweeps"],
                       "kernel_ms_per_launch": plain["kernel_ms_per_launch"],
                       "achieved_tflops": plain["achieved"],
                       "frac": plain["achieved"] / FP64_PEAK_TFLOPS},
        # both paths over the same Trotter steps (the first Kp timed steps)
        "mixed_over_plain": mm["value"] / plain["value"],
        "mixed_over_plain_per_sum_chi3": mm["sum_chi3_per_s"] / plain["sum_chi3_per_s"],
        "mixed_over_plain_per_nominal_flop": mm["tflops"] / plain["achieved"],
        "mixed_over_plain_window": [W * J, (W + Kp) * J],
        "max_sample_err_mixed_vs_fp64": err,
        "max_estimator_err_mixed_vs_fp64": est_err,
        "err_at_trotter_step": (W + Kp) * J,
        "roofline": {"bound": "alu", "achieved": mixed["achieved"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": mixed["achieved"] / FP64_PEAK_TFLOPS,
                     "traffic": traffic,
                     "traffic_source": ("rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel source "
                                        "(profiles/evolve_kernel_traffic.json), not measured in this run"
                                        if traffic is not None else None),
                     "kernel": "evolve_kernel (mixed)",
                     "kernel_ms_per_launch": mixed["kernel_ms_per_launch"],
                     "flops_per_launch": mixed["flops_per_launch"],
                     "flops_model": "Golub-Reinsch nominal per update: 8*(2cl)*cm*(2cr) "
                                    "+ 4*(4m^2n+8mn^2+9n^3), m,n = 2cl,2cr"},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_saturated(
            a.cpu_seconds, mixed["updates_per_sample"], mixed["shifts_per_sample"],
            K * J / p.trotter_steps)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
