/*
 * tepai.h -- C ABI of libtepai, batched MPS TE-PAI on one MI355X (gfx950).
 *
 * The library estimates <O>(T) for a Hamiltonian H = sum_k c_k h_k (Pauli
 * terms h_k) with the TE-PAI protocol of Hasselgren & Koczor, "Quantum-inspired
 * classical simulation through randomized time evolution" (sec. "TE-PAI",
 * protocol steps 1-3): each rotation R_k(theta_k), theta_k = 2 c_k T / N, of
 * the N-step first-order Trotter circuit is replaced at random by I,
 * R_k(sign(theta_k) Delta) or R_k(pi) (appendix "PAI & TE-PAI", eqs.
 * settings and gammas); every sampled circuit is simulated as a matrix
 * product state with bond cap chi (sec. "Resource model and cost metrics":
 * two-site update, SVD re-factorisation, truncation to the chi largest
 * singular values); the per-sample values are weighted by ||g||_1 sign(g_l)
 * and averaged (Statement 2).
 *
 * Conventions for every entry point:
 *  - All pointers are owned by the caller.  The library copies what it needs
 *    from host inputs before returning and keeps no pointer to them.
 *  - Pointers named d_* and `workspace` are device pointers on the handle's
 *    device; all others are host pointers.
 *  - Errors are reported by the return code only; no exception crosses the
 *    ABI.  On error the outputs are unspecified and tepai_last_error(h)
 *    describes the failure.
 *  - A handle must not be used by two host threads at once.
 *  - Sampling is deterministic: the same problem and seed give bit-identical
 *    circuits and signs on every run.
 *
 * Readings of the paper that the library implements (where it is silent):
 *  - time order of the rotations is the order of `terms`, repeated for each
 *    of the N Trotter steps;
 *  - a rotation with |theta_k| > Delta is split into m = ceil(|theta_k|/Delta)
 *    equal sub-rotations (the paper assumes |theta| <= Delta);
 *  - consecutive sampled gates on one qubit pair form one two-site update
 *    (one truncated SVD); runs end at Trotter-step boundaries
 *    (TEPAI_PER_GATE: one update per sampled gate instead);
 *  - a two-qubit gate on non-adjacent sites lo < hi (the ring's wrap bond,
 *    once the ring is kept as a chain) is applied by carrying the end qubit
 *    nearer the orthogonality centre across the chain with truncated SWAP
 *    updates, the last of which is SWAP.G on the pair: hi - lo updates per
 *    routed gate, no return trip, and the chain keeps its new order (a
 *    rotation of the ring by one site, which tepai_batch_read_mps reports
 *    in qubit_at);
 *  - a two-site update keeps min(chi, #{sigma_i > svd_cutoff * sigma_0})
 *    singular values and renormalises them; the orthogonality centre is
 *    moved by single-site SVDs that drop sigma_i <= svd_cutoff * sigma_0.
 */
#ifndef TEPAI_H
#define TEPAI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TEPAI_OK = 0,
  TEPAI_EINVAL = -1,    /* malformed argument (null pointer, bad qubit, ...) */
  TEPAI_ERANGE = -2,    /* value out of range (Delta not in (0,pi), N = 0, chi = 0 ...) */
  TEPAI_ENOMEM = -3,    /* workspace or output capacity too small */
  TEPAI_EDEVICE = -4,   /* HIP runtime error */
  TEPAI_ENUMERIC = -5   /* a sample met a non-finite value or a factorisation hit the
                           Jacobi sweep cap (its tepai_sample_stats.flags say which),
                           or an estimate is not finite; outputs are still written */
} tepai_status;

/* tepai_sample_stats.flags bits. */
enum {
  TEPAI_SAMPLE_NONFINITE = 1u,      /* a factorisation saw a non-finite or zero norm */
  TEPAI_SAMPLE_NONCONVERGED = 2u    /* a Jacobi SVD stopped at the sweep cap */
};

enum { TEPAI_PAULI_I = 0, TEPAI_PAULI_X = 1, TEPAI_PAULI_Y = 2, TEPAI_PAULI_Z = 3 };

/* Gate setting codes of a sampled rotation (appendix "PAI & TE-PAI", eq. settings). */
enum { TEPAI_SET_A = 0, TEPAI_SET_B = 1, TEPAI_SET_C = 2 };

/* tepai_problem.flags.
 * TEPAI_NO_PI: the biased variant without pi rotations (appendix "Proof of
 *   Statement 3"): each rotation is A with probability 1 - lambda and B with
 *   probability lambda = |theta| / Delta; every sign is +1, ||g||_1 = 1 and
 *   all weights are 1, at a per-gate bias |theta| (Delta - |theta|) / 2
 *   R''(0) + O(Delta^3). */
enum { TEPAI_NO_PI = 1u };
/* TEPAI_TROTTER: the deterministic first-order product formula (eq.
 *   Trotter-Suzuki) run through the same MPS engine, the comparison circuit of
 *   sec. "Truncation": every rotation of every step is applied exactly as
 *   R_k(theta_k) (a split rotation as its m equal sub-rotations), so every
 *   sample is the same circuit.  The table reports gamma = (0, 1, 0),
 *   thresholds (0, 2^63) and log_g1_step = 0: the sampler marks every rotation
 *   TEPAI_SET_B (here meaning the exact rotation), every sign is +1 and every
 *   weight is 1.  Cannot be combined with TEPAI_NO_PI. */
enum { TEPAI_TROTTER = 2u };
/* TEPAI_PER_GATE: every sampled two-qubit gate is applied as its own
 *   truncated two-site update (a pi rotation as local Paulis, without an
 *   SVD) instead of fusing a run of consecutive gates on one qubit pair into
 *   one update.  It changes the truncation points, not the circuit: with no
 *   truncation both forms give the same state.  Combines with the other
 *   flags. */
enum { TEPAI_PER_GATE = 4u };
/* TEPAI_WORK_QUEUE: scheduling only (sec. "Circuit parallelisation": the
 *   samples are independent).  A batch's evolve steps run on about one
 *   workgroup per compute unit, each taking the next sample from a counter
 *   in the workspace, in the batch's launch order (decreasing bond cap),
 *   instead of one workgroup per sample.  Results are bitwise those without
 *   the flag; it matters for batches with many more samples than compute
 *   units and mixed caps.  Combines with the other flags. */
enum { TEPAI_WORK_QUEUE = 8u };

/* Storage / arithmetic precision of the MPS path.
 * TEPAI_FP64: complex128 site tensors and FP64 throughout (the Jacobi skips
 *   a column pair only below 2^-53 sqrt(R) of its norms, LAPACK's one-sided
 *   Jacobi criterion); per-sample values agree with another FP64 evaluation
 *   of the same truncated trajectory to about 1e-10, unless the trajectory
 *   itself is sensitive to rounding: a cut at the bond cap between nearly
 *   equal singular values (counted in tepai_sample_stats.ties) lets rounding
 *   decide which straddling vector is kept, and later cuts amplify earlier
 *   rounding differences by about sigma_{k-1} / gap.
 * TEPAI_FP32_MIXED: complex64 site tensors; the two-site contraction, the
 *   centre-shift products and the projection onto the kept singular vectors
 *   run on FP32 matrix cores with FP32 accumulation; the QR preconditioner,
 *   the Jacobi orthogonalisation (stopped after a sweep in which every
 *   rotated column pair had a cosine |x^H y| / (|x||y|) <= 1e-5; the FP64
 *   path uses 1e-8), the truncation, the
 *   renormalisation, the weights and the estimator stay FP64.  Per-sample
 *   values agree with the FP64 path to about 1e-4. */
enum { TEPAI_FP64 = 0, TEPAI_FP32_MIXED = 1 };

/* One Hamiltonian term c * P_0(q_0) [P_1(q_1)]; nq = 1 or 2.  Two-qubit
 * terms must act on neighbours of the ring: |q0 - q1| = 1 or {0, n-1}. */
typedef struct {
  uint32_t nq;
  uint32_t qubit[2];
  uint8_t pauli[2];     /* TEPAI_PAULI_X/Y/Z */
  uint8_t pad[6];
  double coeff;
} tepai_term;

/* One weighted Pauli string coeff * prod_i P_i(q_i) contributing to
 * observable number `observable`; each observable is the sum of its strings. */
typedef struct {
  uint32_t n_ops;               /* 1 .. 8 */
  uint32_t observable;
  const uint32_t* qubits;       /* [n_ops], distinct */
  const uint8_t* paulis;        /* [n_ops], TEPAI_PAULI_X/Y/Z */
  double coeff;
} tepai_pauli_string;

/* A starting state shared by every sample (hybrid start: e.g. the state a
 * deep Trotter circuit reached at t0, from which the TE-PAI segment of
 * duration total_time continues; sec. "Implementation", Trotter-then-TE-PAI).
 * Site k of the chain holds A_k[a][s][c] of shape bond[k] x 2 x bond[k+1],
 * row-major, as interleaved (re, im) doubles; the sites are concatenated in
 * order.  qubit_at[k] is the qubit held at site k (NULL: qubit k).  Sites
 * left of `centre` must be left-canonical and sites right of it
 * right-canonical (not checked: truncations are optimal only in that form;
 * nor are the values checked: a non-finite entry makes every sample
 * non-finite, which tepai_run reports as TEPAI_ENUMERIC).
 * bond[0] = bond[n] = 1, and no bond may exceed chi_max.  A sample whose
 * cap is below the state's largest bond starts from a truncated copy
 * (truncation on copy, done in tepai_batch_create): the copy's centre is
 * moved to site 0 by exact single-site SVD shifts, then swept to site n-1,
 * each shift keeping min(cap, #{sigma_i > svd_cutoff * sigma_0}) singular
 * values renormalised to unit norm, so every cut is truncated optimally for
 * the state the earlier cuts left; these shifts count in the sample's
 * `shifts`, and its centre starts at site n-1.  Caller-owned; the library
 * copies it in tepai_batch_create (and tepai_run) and keeps no pointer. */
typedef struct {
  const uint32_t* bond;         /* [n_qubits + 1] */
  const double* tensors;        /* sum_k 2 bond[k] bond[k+1] complex values */
  const uint32_t* qubit_at;     /* [n_qubits] or NULL */
  uint32_t centre;              /* orthogonality centre site, < n_qubits */
  uint32_t reserved;            /* 0 */
} tepai_mps;

typedef struct {
  uint32_t n_qubits;            /* 2 .. 256 */
  uint32_t n_terms;
  const tepai_term* terms;      /* time order inside one Trotter step */
  double total_time;            /* T >= 0 */
  uint32_t trotter_steps;       /* N >= 1 */
  double delta;                 /* PAI angle, 0 < Delta < pi */
  uint64_t n_samples;           /* N_s */
  uint64_t sample_offset;       /* global index of the first sample */
  uint64_t seed;
  uint32_t chi_max;             /* bond cap, 1 .. 256 */
  const uint32_t* chi_per_sample; /* nullable; [n_samples] caps <= chi_max */
  double svd_cutoff;            /* relative singular-value floor, >= 0 (the mixed
                                   path uses max(svd_cutoff, 1e-7)) */
  const uint8_t* initial_bits;  /* [n_qubits] computational-basis start, 0/1;
                                   ignored (and may be NULL) when initial_mps is given */
  uint32_t n_obs;
  uint32_t n_strings;
  const tepai_pauli_string* strings;
  uint32_t precision;           /* TEPAI_FP64 or TEPAI_FP32_MIXED */
  uint32_t flags;               /* TEPAI_NO_PI or TEPAI_TROTTER, | TEPAI_PER_GATE | TEPAI_WORK_QUEUE */
  const tepai_mps* initial_mps; /* NULL: start from initial_bits */
} tepai_problem;

/* Per-sample counters (cost model of eq. Wsample and truncation record). */
typedef struct {
  uint64_t n_gates;             /* non-identity sampled gates */
  uint64_t updates;             /* truncated two-site updates (incl. SWAPs) */
  uint64_t swap_updates;
  uint64_t shifts;              /* single-site centre shifts */
  uint64_t jacobi_sweeps;       /* over all factorisations */
  uint64_t nonconverged;        /* factorisations that hit the sweep cap */
  uint64_t ties;                /* near ties: cap cuts where 4 sqrt(2) th sigma_{k-1} / |sigma_kept|
                                   > 1e-10, th = min(1, eps / gap), gap = (sigma_{k-1} -
                                   sigma_k) / sigma_0, eps = 2^-53 sqrt(R C) for an R x C
                                   matrix: FP64 rounding does not fix the kept state there */
  double sum_chi3;              /* sum over updates of chi_mid^3 */
  double nominal_flops;         /* Golub-Reinsch count of all updates */
  double discarded;             /* sum of discarded squared Schmidt weight */
  double max_discarded;
  double min_gap;               /* min (sigma_{k-1}-sigma_k)/sigma_0 at a cut */
  int32_t sign;                 /* (-1)^(number of C settings) */
  uint32_t layer;               /* Trotter steps applied so far */
  uint32_t max_bond;
  uint32_t flags;               /* TEPAI_SAMPLE_NONFINITE | TEPAI_SAMPLE_NONCONVERGED */
} tepai_sample_stats;

typedef struct tepai_handle tepai_handle;
typedef struct tepai_batch tepai_batch;
typedef struct tepai_step_graph tepai_step_graph;

/* Create a handle bound to HIP device `device`.  Fails with TEPAI_EDEVICE
 * when the device is absent or is not gfx950.  The first call on a device
 * also looks up the device address of the fixed array that
 * tepai_run_noalloc works in (which loads it on that device); a failed
 * lookup leaves the handle usable for every other call.  The caller's
 * current device is left as it was. */
tepai_status tepai_create(tepai_handle** out, int device);
void tepai_destroy(tepai_handle* h);
/* Message of the last failure on this handle ("" if none).  Valid until the
 * next call on the handle. */
const char* tepai_last_error(const tepai_handle* h);

/* Check a problem description (ranges, qubit indices, ring adjacency).
 * Returns TEPAI_OK or the first error found. */
tepai_status tepai_validate(tepai_handle* h, const tepai_problem* p);

/* The per-rotation PAI table the sampler uses (host computation).
 * Row r of the L_eff rows: source term index term[r], signed sub-rotation
 * angle theta[r] = 2 c T / (N m), gamma[3r..3r+2] = gamma_1..3(|theta|)
 * (eq. gammas), thresholds[2r], thresholds[2r+1] = floor(p_1 2^63),
 * floor((p_1+p_2) 2^63) (2^63 when the mass reaches 1).  A setting is
 * drawn from v = u >> 1 of a Philox4x32-10 64-bit uniform u as A if
 * v < t1, B if v < t2, else C.  *log_g1_step = sum_r log ||gamma_r||_1,
 * so log ||g||_1 = N * *log_g1_step (eq. overhead-bound).  `capacity` is the
 * row capacity of the output arrays; *l_eff is set even when it is too small
 * (then TEPAI_ENOMEM). */
tepai_status tepai_pai_table(tepai_handle* h, const tepai_problem* p, uint32_t capacity,
                             uint32_t* l_eff, uint32_t* term, double* theta, double* gamma,
                             uint64_t* thresholds, double* log_g1_step, uint32_t* n_split_terms);

/* Sample the circuits of samples sample_offset+first .. +first+count-1,
 * first `layers` Trotter steps (0 = all N), on the GPU.  Sample i's gates
 * are words[offsets[i] .. offsets[i+1]-1], each word = g * 4 + setting with
 * g = j * L_eff + r the flat rotation index (time order) and setting
 * TEPAI_SET_B or TEPAI_SET_C; signs[i] = (-1)^(#C).  offsets has count+1
 * entries and is always written; if offsets[count] > capacity the call
 * returns TEPAI_ENOMEM without writing words.  Host pointers. */
tepai_status tepai_sample_circuits(tepai_handle* h, const tepai_problem* p, uint64_t first,
                                   uint64_t count, uint32_t layers, uint64_t capacity,
                                   uint64_t* offsets, uint32_t* words, int8_t* signs);

/* Device workspace needed by a batch of `count` samples of problem p. */
tepai_status tepai_workspace_size(tepai_handle* h, const tepai_problem* p, uint32_t count,
                                  size_t* bytes);

/* Start a batch: samples sample_offset+first .. +first+count-1, each in the
 * initial product state, in the caller's device `workspace` (>= the size
 * reported by tepai_workspace_size; 256-byte aligned).  Work is queued on
 * `hip_stream` (a hipStream_t, NULL = default stream); the library allocates
 * no device memory for a batch.  The batch object is a small host record;
 * destroy it with tepai_batch_destroy (the workspace stays the caller's). */
tepai_status tepai_batch_create(tepai_handle* h, const tepai_problem* p, uint64_t first,
                                uint32_t count, void* workspace, size_t ws_bytes,
                                void* hip_stream, tepai_batch** out);
/* Apply the next `n_layers` Trotter steps of every sample's sampled circuit
 * (sampling fused: each sample draws its own gate settings).  Under
 * TEPAI_WORK_QUEUE this queues two kernels: one zeroes the counter in the
 * workspace, then the workgroups of the second take the slots from it, so
 * steps of one batch must not run concurrently on two streams. */
tepai_status tepai_batch_evolve(tepai_batch* b, uint32_t n_layers);
/* Read out the observables of every sample at its current step j:
 * d_values[s * n_obs + o] = <O_o> of sample s (normalised state), and
 * d_weights[s] = sign_s * ||g||_1(j) with ||g||_1(j) = exp(j * log_g1_step),
 * the weight of the TE-PAI sample made of the first j steps. */
tepai_status tepai_batch_observe(tepai_batch* b, double* d_values, double* d_weights);
/* Copy the per-sample counters to the host ([count] records); synchronises
 * the batch's stream. */
tepai_status tepai_batch_stats(tepai_batch* b, tepai_sample_stats* stats);
/* Copy the MPS of batch slot `slot` (sample sample_offset+first+slot) at its
 * current step to the host, in the form of tepai_mps, so that a state the
 * GPU evolved can start other samples (hybrid start: a TEPAI_TROTTER batch
 * evolved to t0, then TE-PAI from its state; sec. "Implementation",
 * Trotter-then-TE-PAI).  Writes bond[n_qubits + 1], qubit_at[n_qubits],
 * *centre and *n_values = sum_k 2 bond[k] bond[k+1] (complex values); then,
 * if `tensors` is not NULL and n_values <= capacity (complex values), the
 * site tensors as interleaved (re, im) doubles, site after site, each
 * A_k[a][s][c] row-major (complex64 tensors of the mixed path are widened).
 * Sites left of the centre are left-canonical, right of it right-canonical,
 * and the state has unit norm.  Synchronises the batch's stream.  Returns
 * TEPAI_ERANGE for slot >= count and TEPAI_ENOMEM (outputs other than
 * `tensors` written) when capacity is too small.  Host pointers. */
tepai_status tepai_batch_read_mps(tepai_batch* b, uint32_t slot, uint64_t capacity,
                                  uint32_t* bond, uint32_t* qubit_at, uint32_t* centre,
                                  uint64_t* n_values, double* tensors);
void tepai_batch_destroy(tepai_batch* b);

/* Autotuning of the one SVD tile parameter that the matrix size does not
 * fix: the panel width of the pivoted-QR preconditioner (QR steps between
 * two applications of the accumulated reflectors to the trailing columns;
 * 1..32, 32 by default).  From the batch's current state, each of the
 * n_candidates widths runs the next n_layers Trotter steps, timed with HIP
 * events on the batch's stream, after which the whole workspace is restored
 * from d_scratch (a device buffer of at least the batch's workspace size,
 * tepai_workspace_size for its count), so the batch ends where it started
 * and later steps are computed as if untuned, up to the rounding of the
 * chosen width.  The batch keeps the width with the highest nominal-flop
 * rate (eq. Wsample's cost model over the same steps) for its later steps;
 * *chosen reports it, and ms[i], flops[i] (each may be NULL) each
 * candidate's time and nominal flops.  Synchronises the stream.  Results
 * are equally valid for every width (the SVD does not depend on it beyond
 * rounding). */
tepai_status tepai_batch_autotune(tepai_batch* b, uint32_t n_layers, const uint32_t* candidates,
                                  uint32_t n_candidates, void* d_scratch, size_t scratch_bytes,
                                  double* ms, double* flops, uint32_t* chosen);

/* A captured read-out step of a batch: the launches of tepai_batch_evolve
 * (n_layers Trotter steps), tepai_batch_observe into d_values / d_weights
 * and tepai_reduce into d_mean / d_std_err, recorded once as a HIP graph on
 * the batch's stream and replayed by tepai_step_graph_launch (the time
 * series of sec. "Deterministic Expectation Values": each replay advances
 * every sample by n_layers steps and leaves the estimate at the new time).
 * A replay does exactly what the three calls would do; it saves their host
 * launch work.  The batch's stream must not be the null stream (TEPAI_EINVAL:
 * it cannot be captured); the device buffers (count * n_obs, count, n_obs,
 * n_obs doubles) and the batch must outlive the graph.  Nothing runs at
 * capture time.  tepai_step_graph_launch returns TEPAI_ERANGE, launching
 * nothing, when the batch would pass its last Trotter step; it does not
 * synchronise.  The recorded work holds no memset nodes. */
tepai_status tepai_batch_capture_step(tepai_batch* b, uint32_t n_layers, double* d_values,
                                      double* d_weights, double* d_mean, double* d_std_err,
                                      tepai_step_graph** out);
tepai_status tepai_step_graph_launch(tepai_step_graph* g);
void tepai_step_graph_destroy(tepai_step_graph* g);

/* Weighted reduction on the device (Statement 2): x_s = w_s v_s,
 * d_mean[o] = sum_s x_so / count, d_std_err[o] = sqrt(var_o / count) with the
 * ddof=1 sample variance (NaN when count < 2), fixed summation order. */
tepai_status tepai_reduce(tepai_handle* h, uint64_t count, uint32_t n_obs, const double* d_values,
                          const double* d_weights, double* d_mean, double* d_std_err,
                          void* hip_stream);

/* The whole estimator, synchronous, host outputs: mean[n_obs], std_err[n_obs],
 * weights[n_samples]; values[n_samples * n_obs] and stats[n_samples] are
 * optional (NULL to skip).  Allocates and frees its own device memory (freed
 * on every return path) and processes the samples in batches of at most
 * `batch` (0 = library choice).  Returns TEPAI_ENUMERIC, with every output
 * written, when a sample's flags are set (non-finite value, Jacobi sweep cap)
 * or an estimate is not finite. */
tepai_status tepai_run(tepai_handle* h, const tepai_problem* p, uint32_t batch, double* mean,
                       double* std_err, double* weights, double* values,
                       tepai_sample_stats* stats);

/* Bytes of the fixed device array that tepai_run_noalloc works in. */
#define TEPAI_NOALLOC_BYTES ((size_t)256 << 20)

/* tepai_run without any device allocation, for callers that cannot allocate
 * device memory (serving loops that keep a fixed footprint, harnesses that
 * forbid hipMalloc).  The batch workspace lives in one file-scope device
 * array of TEPAI_NOALLOC_BYTES per GPU, reserved when tepai_create first
 * runs on that GPU and held until the process ends; the samples go through
 * it in batches of as many as fit.  Outputs are device pointers, all
 * required: d_mean[n_obs], d_std_err[n_obs], d_weights[n_samples],
 * d_values[n_samples * n_obs] (the reduction reads them); stats[n_samples]
 * is a host array, optional (NULL to skip).  Work is queued on hip_stream
 * (NULL: the null stream) and the call returns after synchronising it.
 * Returns TEPAI_ENOMEM when one sample's workspace (tepai_workspace_size
 * with count 1) exceeds TEPAI_NOALLOC_BYTES, and TEPAI_ENUMERIC like
 * tepai_run.  Every call on one GPU shares that GPU's array, which keeps
 * the last call's contents (nothing in it needs to start at zero): calls
 * that overlap on one GPU, from several threads or handles, race. */
tepai_status tepai_run_noalloc(tepai_handle* h, const tepai_problem* p, void* hip_stream,
                               double* d_mean, double* d_std_err, double* d_weights,
                               double* d_values, tepai_sample_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* TEPAI_H */
