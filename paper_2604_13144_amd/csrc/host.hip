// Host side of libtepai: validation, the PAI table, workspace layout, the
// batch interface and the synchronous estimator.  Every C entry point of
// tepai.h is defined here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tepai_internal.h"

struct tepai_handle {
  int device = 0;
  void* scratch = nullptr;   // device address of this GPU's copy of `scratch`
  std::string scratch_err;   // why that address is missing, if it is
  std::string err;
};

// Workspace of tepai_run_noalloc: one copy per GPU, loaded with the code
// object.  In host code the name stands for a host-side handle, not for the
// device memory: only the address that hipGetSymbolAddress returns for the
// current device may be handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[TEPAI_NOALLOC_BYTES];

namespace tepai {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kThresholdOne = 1ull << 63;

tepai_status fail(tepai_handle* h, tepai_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

#define TEPAI_HIP(h, expr)                                                           \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((h), TEPAI_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// Device allocations of the synchronous calls, freed on every return path.
struct DeviceBuffers {
  std::vector<void*> ptrs;
  DeviceBuffers() = default;
  DeviceBuffers(const DeviceBuffers&) = delete;
  DeviceBuffers& operator=(const DeviceBuffers&) = delete;
  ~DeviceBuffers() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t bytes) {
    *out = nullptr;
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e == hipSuccess) {
      ptrs.push_back(q);
      *out = static_cast<T*>(q);
    } else {
      // reported through the status code; clear it so that it does not
      // surface again in the caller's next launch check
      (void)hipGetLastError();
    }
    return e;
  }
};

// ------------------------------------------------------------ PAI table
// gamma_1..3 at angle |theta| for PAI angle Delta (appendix "PAI & TE-PAI",
// eq. gammas).
void pai_gammas(double t, double d, double g[3]) {
  g[0] = std::cos(t / 2.0) * std::sin(d / 2.0 - t / 2.0) / std::sin(d / 2.0);
  g[1] = std::sin(t) / std::sin(d);
  g[2] = -std::sin(t / 2.0) * std::sin(d / 2.0 - t / 2.0) / std::cos(d / 2.0);
}

uint64_t threshold(double p) {
  if (p >= 1.0) return kThresholdOne;
  if (p <= 0.0) return 0;
  return (uint64_t)(p * 9223372036854775808.0);   // p * 2^63, exact scaling
}

struct HostRow {
  uint32_t term;
  double theta;
  double g[3];
  double norm1;
  uint64_t t1, t2;
};

struct Table {
  std::vector<HostRow> rows;
  double log_step = 0.0;
  uint32_t n_split = 0;
};

// theta_k = 2 c_k T / N (appendix "PAI & TE-PAI"); a rotation with
// |theta_k| > Delta becomes ceil(|theta_k| / Delta) equal sub-rotations.
Table build_table(const tepai_problem& p) {
  Table t;
  for (uint32_t k = 0; k < p.n_terms; ++k) {
    const double theta = 2.0 * p.terms[k].coeff * p.total_time / (double)p.trotter_steps;
    uint32_t m = 1;
    if (std::fabs(theta) > p.delta) {
      m = (uint32_t)std::ceil(std::fabs(theta) / p.delta);
      t.n_split += 1;
    }
    HostRow r;
    r.term = k;
    r.theta = theta / (double)m;
    if (p.flags & TEPAI_TROTTER) {
      // deterministic product formula: the exact rotation every time
      r.g[0] = 0.0;
      r.g[1] = 1.0;
      r.g[2] = 0.0;
      r.norm1 = 1.0;
      r.t1 = 0;
      r.t2 = kThresholdOne;
    } else if (p.flags & TEPAI_NO_PI) {
      // gamma~ = (1 - lambda, lambda, 0): probabilities themselves, ||.||_1 = 1
      const double lam = std::fabs(r.theta) / p.delta;
      r.g[0] = 1.0 - lam;
      r.g[1] = lam;
      r.g[2] = 0.0;
      r.norm1 = 1.0;
      r.t1 = threshold(r.g[0]);
      r.t2 = kThresholdOne;
    } else {
      pai_gammas(std::fabs(r.theta), p.delta, r.g);
      r.norm1 = std::fabs(r.g[0]) + std::fabs(r.g[1]) + std::fabs(r.g[2]);
      const double p1 = std::fabs(r.g[0]) / r.norm1, p2 = std::fabs(r.g[1]) / r.norm1;
      r.t1 = threshold(p1);
      r.t2 = threshold(p1 + p2);
    }
    for (uint32_t i = 0; i < m; ++i) t.rows.push_back(r);
  }
  for (const HostRow& r : t.rows) t.log_step += std::log(r.norm1);
  return t;
}

std::vector<DevRow> device_rows(const tepai_problem& p, const Table& t) {
  std::vector<DevRow> out(t.rows.size());
  for (size_t i = 0; i < t.rows.size(); ++i) {
    const HostRow& r = t.rows[i];
    const tepai_term& term = p.terms[r.term];
    // setting B is R(sign(theta) Delta); under TEPAI_TROTTER it is R(theta)
    const double phi = (p.flags & TEPAI_TROTTER) ? r.theta
                       : r.theta != 0.0 ? std::copysign(p.delta, r.theta) : p.delta;
    DevRow d{};
    d.t1 = r.t1;
    d.t2 = r.t2;
    d.cb = std::cos(phi / 2.0);
    d.sb = std::sin(phi / 2.0);
    d.nq = term.nq;
    d.q0 = term.qubit[0];
    d.q1 = term.nq == 2 ? term.qubit[1] : 0;
    d.p0 = term.pauli[0];
    d.p1 = term.nq == 2 ? term.pauli[1] : 0;
    out[i] = d;
  }
  return out;
}

// ----------------------------------------------------------- validation
tepai_status validate(tepai_handle* h, const tepai_problem* p) {
  if (!p) return fail(h, TEPAI_EINVAL, "problem is NULL");
  const uint32_t n = p->n_qubits;
  if (n < 2 || n > (uint32_t)kMaxQubits) return fail(h, TEPAI_ERANGE, "n_qubits must be in [2, 256]");
  if (!p->terms || p->n_terms == 0) return fail(h, TEPAI_EINVAL, "no Hamiltonian terms");
  for (uint32_t k = 0; k < p->n_terms; ++k) {
    const tepai_term& t = p->terms[k];
    if (t.nq != 1 && t.nq != 2) return fail(h, TEPAI_EINVAL, "term " + std::to_string(k) + ": nq must be 1 or 2");
    for (uint32_t i = 0; i < t.nq; ++i) {
      if (t.qubit[i] >= n) return fail(h, TEPAI_EINVAL, "term " + std::to_string(k) + ": qubit out of range");
      if (t.pauli[i] < 1 || t.pauli[i] > 3) return fail(h, TEPAI_EINVAL, "term " + std::to_string(k) + ": Pauli code must be X, Y or Z");
    }
    if (t.nq == 2) {
      const uint32_t a = t.qubit[0], b = t.qubit[1];
      const uint32_t d = a > b ? a - b : b - a;
      if (!(d == 1 || (d == n - 1 && n > 2)))
        return fail(h, TEPAI_EINVAL, "term " + std::to_string(k) + ": two-qubit terms must act on ring neighbours");
    }
    if (!std::isfinite(t.coeff)) return fail(h, TEPAI_ERANGE, "non-finite coefficient");
  }
  if (!std::isfinite(p->total_time) || p->total_time < 0.0) return fail(h, TEPAI_ERANGE, "total_time must be finite and >= 0");
  if (p->trotter_steps == 0) return fail(h, TEPAI_ERANGE, "trotter_steps must be >= 1");
  if (!(p->delta > 0.0 && p->delta < kPi)) return fail(h, TEPAI_ERANGE, "delta must lie in (0, pi)");
  if (p->n_samples == 0) return fail(h, TEPAI_ERANGE, "n_samples must be >= 1");
  if (p->sample_offset + p->n_samples > (1ull << 32) || p->sample_offset + p->n_samples < p->sample_offset)
    return fail(h, TEPAI_ERANGE, "sample indices must stay below 2^32");
  if (p->chi_max < 1 || p->chi_max > (uint32_t)kMaxChi) return fail(h, TEPAI_ERANGE, "chi_max must be in [1, 256]");
  if (p->chi_per_sample)
    for (uint64_t s = 0; s < p->n_samples; ++s)
      if (p->chi_per_sample[s] < 1 || p->chi_per_sample[s] > p->chi_max)
        return fail(h, TEPAI_ERANGE, "chi_per_sample entries must be in [1, chi_max]");
  if (!std::isfinite(p->svd_cutoff) || p->svd_cutoff < 0.0) return fail(h, TEPAI_ERANGE, "svd_cutoff must be finite and >= 0");
  if (!p->initial_mps) {
    // the computational-basis start is used only without a shared MPS
    if (!p->initial_bits) return fail(h, TEPAI_EINVAL, "initial_bits is NULL and no initial_mps is given");
    for (uint32_t i = 0; i < n; ++i)
      if (p->initial_bits[i] > 1) return fail(h, TEPAI_EINVAL, "initial_bits entries must be 0 or 1");
  }
  if (p->n_obs > 256) return fail(h, TEPAI_ERANGE, "at most 256 observables");
  if (p->n_strings && !p->strings) return fail(h, TEPAI_EINVAL, "strings is NULL");
  for (uint32_t s = 0; s < p->n_strings; ++s) {
    const tepai_pauli_string& ps = p->strings[s];
    if (ps.n_ops < 1 || ps.n_ops > (uint32_t)kMaxStringOps) return fail(h, TEPAI_ERANGE, "Pauli strings hold 1..8 factors");
    if (ps.observable >= p->n_obs) return fail(h, TEPAI_EINVAL, "string observable index out of range");
    if (!ps.qubits || !ps.paulis) return fail(h, TEPAI_EINVAL, "string qubits/paulis NULL");
    for (uint32_t i = 0; i < ps.n_ops; ++i) {
      if (ps.qubits[i] >= n) return fail(h, TEPAI_EINVAL, "string qubit out of range");
      if (ps.paulis[i] < 1 || ps.paulis[i] > 3) return fail(h, TEPAI_EINVAL, "string Pauli code must be X, Y or Z");
      for (uint32_t j = 0; j < i; ++j)
        if (ps.qubits[j] == ps.qubits[i]) return fail(h, TEPAI_EINVAL, "string qubits must be distinct");
    }
    if (!std::isfinite(ps.coeff)) return fail(h, TEPAI_ERANGE, "non-finite string coefficient");
  }
  if (const tepai_mps* m = p->initial_mps) {
    if (!m->bond || !m->tensors) return fail(h, TEPAI_EINVAL, "initial_mps bond/tensors NULL");
    if (m->bond[0] != 1 || m->bond[n] != 1) return fail(h, TEPAI_EINVAL, "initial_mps end bonds must be 1");
    for (uint32_t k = 0; k <= n; ++k)
      if (m->bond[k] < 1 || m->bond[k] > p->chi_max)
        return fail(h, TEPAI_ERANGE, "initial_mps bond " + std::to_string(k) + " outside [1, chi_max]");
    if (m->centre >= n) return fail(h, TEPAI_ERANGE, "initial_mps centre out of range");
    if (m->qubit_at) {
      std::vector<int> seen(n, 0);
      for (uint32_t k = 0; k < n; ++k) {
        if (m->qubit_at[k] >= n || seen[m->qubit_at[k]]++)
          return fail(h, TEPAI_EINVAL, "initial_mps qubit_at must be a permutation");
      }
    }
    if (m->reserved != 0) return fail(h, TEPAI_EINVAL, "initial_mps reserved must be 0");
  }
  if (p->precision != TEPAI_FP64 && p->precision != TEPAI_FP32_MIXED)
    return fail(h, TEPAI_EINVAL, "unsupported precision");
  if ((p->flags & ~(uint32_t)(TEPAI_NO_PI | TEPAI_TROTTER | TEPAI_PER_GATE | TEPAI_WORK_QUEUE)) != 0)
    return fail(h, TEPAI_EINVAL, "unsupported flags");
  if ((p->flags & TEPAI_NO_PI) && (p->flags & TEPAI_TROTTER))
    return fail(h, TEPAI_EINVAL, "TEPAI_NO_PI and TEPAI_TROTTER exclude each other");
  return TEPAI_OK;
}

// ------------------------------------------------------- workspace layout
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t rows, strings, bits, caps, queue, states, tensors, work, init, total;
  uint64_t site_stride, work_stride;
  uint64_t init_elems;     // packed complex values of the initial MPS (0: none)
};

// bytes of the staged initial MPS: offsets, bonds, qubits, then the tensors
static size_t init_bytes(uint32_t n, uint64_t elems) {
  return align256(sizeof(uint64_t) * (n + 1)) + align256(sizeof(uint32_t) * (n + 1)) +
         align256(sizeof(uint16_t) * n) + sizeof(double2) * elems;
}

Layout layout(const tepai_problem& p, uint32_t l_eff, uint32_t count) {
  Layout L{};
  const uint64_t chi = p.chi_max;
  L.site_stride = 2 * chi * chi;
  // three scratch matrices of (2 chi)^2, each at least one element per
  // thread (the QR's trailing pass parks out-of-column stores in the third)
  L.work_stride = 3 * std::max<uint64_t>((2 * chi) * (2 * chi), kThreads);
  size_t off = 0;
  L.rows = off;
  off = align256(off + sizeof(DevRow) * l_eff);
  L.strings = off;
  off = align256(off + sizeof(DevString) * std::max<uint32_t>(p.n_strings, 1));
  L.bits = off;
  off = align256(off + p.n_qubits);
  L.caps = off;     // per-slot caps, then the launch order of the slots
  off = align256(off + sizeof(uint32_t) * 2 * count);
  L.queue = off;    // work-queue counter (TEPAI_WORK_QUEUE)
  off = align256(off + sizeof(uint32_t));
  L.states = off;
  off = align256(off + sizeof(SampleState) * count);
  L.tensors = off;
  const size_t elem = p.precision == TEPAI_FP32_MIXED ? sizeof(float2) : sizeof(double2);
  off = align256(off + elem * L.site_stride * p.n_qubits * count);
  L.work = off;
  off = align256(off + sizeof(double2) * L.work_stride * count);
  L.init = off;
  L.init_elems = 0;
  if (p.initial_mps) {
    for (uint32_t k = 0; k < p.n_qubits; ++k)
      L.init_elems += 2ull * p.initial_mps->bond[k] * p.initial_mps->bond[k + 1];
    off = align256(off + init_bytes(p.n_qubits, L.init_elems));
  }
  L.total = off;
  return L;
}

}  // namespace
}  // namespace tepai

using namespace tepai;

struct tepai_batch {
  tepai_handle* h;
  hipStream_t stream;
  EngineArgs args;
  void* ws;           // the caller's workspace and the bytes the batch uses of it
  size_t ws_bytes;
  uint32_t trotter_steps;
  uint32_t layers_done;
  uint32_t n_obs;
  uint32_t* queue;      // work-queue counter in the workspace; null: one workgroup per slot
  uint32_t queue_grid;  // workgroups of a work-queue launch (all resident at once)
  // host staging kept alive until destroy (async uploads)
  std::vector<DevRow> rows;
  std::vector<DevString> strings;
  std::vector<uint8_t> bits;
  std::vector<uint32_t> caps;
  std::vector<uint64_t> init_off;
  std::vector<uint32_t> init_bond;
  std::vector<uint16_t> init_qubit;
  std::vector<double2> init_tensors;
};

namespace {

// The evolve launch of a batch, in its scheduling form.
hipError_t evolve_launch(const tepai_batch* b, uint32_t n_layers) {
  return b->queue ? launch_evolve_queue(b->args, n_layers, b->queue, b->queue_grid, b->stream)
                  : launch_evolve(b->args, n_layers, b->stream);
}

// The batch loop of the synchronous estimator: samples in batches of at most
// B in the device workspace `ws`, each evolved through all N Trotter steps
// (launches of at most 16 steps keep single kernels short), read out into
// d_v / d_w, its per-sample counters copied to stats_out; then the weighted
// reduction into d_m / d_se.  Work is queued on `stream` and synchronised
// per batch.
tepai_status run_batches(tepai_handle* h, const tepai_problem* p, uint32_t B, void* ws,
                         size_t ws_bytes, hipStream_t stream, double* d_v, double* d_w,
                         double* d_m, double* d_se, tepai_sample_stats* stats_out) {
  const uint64_t ns = p->n_samples;
  tepai_status st = TEPAI_OK;
  for (uint64_t first = 0; first < ns && st == TEPAI_OK; first += B) {
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(B, ns - first);
    tepai_batch* b = nullptr;
    st = tepai_batch_create(h, p, first, cnt, ws, ws_bytes, stream, &b);
    if (st != TEPAI_OK) break;
    for (uint32_t done = 0; done < p->trotter_steps && st == TEPAI_OK;) {
      const uint32_t step = std::min<uint32_t>(16, p->trotter_steps - done);
      st = tepai_batch_evolve(b, step);
      done += step;
    }
    if (st == TEPAI_OK) st = tepai_batch_observe(b, d_v + first * p->n_obs, d_w + first);
    if (st == TEPAI_OK) st = tepai_batch_stats(b, stats_out + first);   // synchronises
    tepai_batch_destroy(b);
  }
  if (st == TEPAI_OK) st = tepai_reduce(h, ns, p->n_obs, d_v, d_w, d_m, d_se, stream);
  if (st == TEPAI_OK) {
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) st = fail(h, TEPAI_EDEVICE, std::string("estimator: ") + hipGetErrorString(e));
  }
  return st;
}

// TEPAI_ENUMERIC when a sample met a non-finite value or a factorisation hit
// the sweep cap (its flags say which), or an estimate (host copy, may be NULL)
// is not finite; the outputs are written either way.
tepai_status numeric_status(tepai_handle* h, const tepai_problem* p,
                            const tepai_sample_stats* stats, const double* mean) {
  uint64_t nonfinite = 0, nonconv = 0;
  for (uint64_t s = 0; s < p->n_samples; ++s) {
    nonfinite += (stats[s].flags & TEPAI_SAMPLE_NONFINITE) ? 1 : 0;
    nonconv += (stats[s].flags & TEPAI_SAMPLE_NONCONVERGED) ? 1 : 0;
  }
  bool bad_mean = false;
  if (mean)
    for (uint32_t o = 0; o < p->n_obs; ++o) bad_mean = bad_mean || !std::isfinite(mean[o]);
  if (nonfinite || nonconv || bad_mean)
    return fail(h, TEPAI_ENUMERIC,
                std::to_string(nonfinite) + " sample(s) with a non-finite value, " +
                    std::to_string(nonconv) + " with a factorisation at the sweep cap" +
                    (bad_mean ? ", non-finite estimate" : ""));
  return TEPAI_OK;
}

// Device address of `scratch` on each GPU, looked up once per device (with
// that device current) by the first tepai_create on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

tepai_status tepai_create(tepai_handle** out, int device) {
  if (!out) return TEPAI_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TEPAI_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TEPAI_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TEPAI_EDEVICE;
  if (device >= kMaxDevices) return TEPAI_EDEVICE;
  // the lookup needs the device current; the caller's current device is
  // restored.  A failed lookup leaves the handle usable for everything but
  // tepai_run_noalloc, which then reports it.
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return TEPAI_EDEVICE;
  void* addr = nullptr;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = scratch_address(device, &addr);
  if (hipSetDevice(prev) != hipSuccess) return TEPAI_EDEVICE;
  auto* h = new tepai_handle;
  h->device = device;
  h->scratch = addr;
  if (e != hipSuccess)
    h->scratch_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
  *out = h;
  return TEPAI_OK;
}

void tepai_destroy(tepai_handle* h) { delete h; }

const char* tepai_last_error(const tepai_handle* h) { return h ? h->err.c_str() : "no handle"; }

tepai_status tepai_validate(tepai_handle* h, const tepai_problem* p) {
  if (h) h->err.clear();
  return validate(h, p);
}

tepai_status tepai_pai_table(tepai_handle* h, const tepai_problem* p, uint32_t capacity,
                             uint32_t* l_eff, uint32_t* term, double* theta, double* gamma,
                             uint64_t* thresholds, double* log_g1_step, uint32_t* n_split_terms) {
  tepai_status st = validate(h, p);
  if (st != TEPAI_OK) return st;
  if (!l_eff) return fail(h, TEPAI_EINVAL, "l_eff is NULL");
  const Table t = build_table(*p);
  *l_eff = (uint32_t)t.rows.size();
  if (log_g1_step) *log_g1_step = t.log_step;
  if (n_split_terms) *n_split_terms = t.n_split;
  if (t.rows.size() > capacity) return fail(h, TEPAI_ENOMEM, "table capacity too small");
  for (size_t i = 0; i < t.rows.size(); ++i) {
    if (term) term[i] = t.rows[i].term;
    if (theta) theta[i] = t.rows[i].theta;
    if (gamma) std::memcpy(gamma + 3 * i, t.rows[i].g, 3 * sizeof(double));
    if (thresholds) {
      thresholds[2 * i] = t.rows[i].t1;
      thresholds[2 * i + 1] = t.rows[i].t2;
    }
  }
  return TEPAI_OK;
}

tepai_status tepai_sample_circuits(tepai_handle* h, const tepai_problem* p, uint64_t first,
                                   uint64_t count, uint32_t layers, uint64_t capacity,
                                   uint64_t* offsets, uint32_t* words, int8_t* signs) {
  if (!h) return TEPAI_EINVAL;
  tepai_status st = validate(h, p);
  if (st != TEPAI_OK) return st;
  if (!offsets || !signs) return fail(h, TEPAI_EINVAL, "offsets/signs NULL");
  if (count == 0) {
    offsets[0] = 0;
    return TEPAI_OK;
  }
  if (first + count > p->n_samples) return fail(h, TEPAI_ERANGE, "samples beyond n_samples");
  if (count > (1u << 30)) return fail(h, TEPAI_ERANGE, "count too large");
  const Table t = build_table(*p);
  const uint32_t L = (uint32_t)t.rows.size();
  const uint32_t J = layers ? layers : p->trotter_steps;
  if (J > p->trotter_steps) return fail(h, TEPAI_ERANGE, "layers beyond trotter_steps");
  const uint64_t n_draws = (uint64_t)J * L;
  if (n_draws >= (1ull << 30)) return fail(h, TEPAI_ERANGE, "N * L_eff must be < 2^30 for gate words");
  const std::vector<DevRow> rows = device_rows(*p, t);
  if (!words && capacity > 0) return fail(h, TEPAI_EINVAL, "words is NULL with a non-zero capacity");
  TEPAI_HIP(h, hipSetDevice(h->device));
  DeviceBuffers bufs;
  DevRow* d_rows = nullptr;
  uint64_t* d_counts = nullptr;
  int8_t* d_signs = nullptr;
  TEPAI_HIP(h, bufs.alloc(&d_rows, sizeof(DevRow) * L));
  TEPAI_HIP(h, bufs.alloc(&d_counts, sizeof(uint64_t) * (count + 1)));
  TEPAI_HIP(h, bufs.alloc(&d_signs, count));
  TEPAI_HIP(h, hipMemcpy(d_rows, rows.data(), sizeof(DevRow) * L, hipMemcpyHostToDevice));
  const uint64_t s0 = p->sample_offset + first;
  TEPAI_HIP(h, launch_sample_count(d_rows, L, p->seed, s0, count, n_draws, d_counts, d_signs, 0));
  std::vector<uint64_t> counts(count);
  TEPAI_HIP(h, hipMemcpy(counts.data(), d_counts, sizeof(uint64_t) * count, hipMemcpyDeviceToHost));
  TEPAI_HIP(h, hipMemcpy(signs, d_signs, count, hipMemcpyDeviceToHost));
  offsets[0] = 0;
  for (uint64_t i = 0; i < count; ++i) offsets[i + 1] = offsets[i] + counts[i];
  if (offsets[count] > capacity) return fail(h, TEPAI_ENOMEM, "gate capacity too small");
  if (offsets[count] > 0) {
    uint32_t* d_words = nullptr;
    TEPAI_HIP(h, hipMemcpy(d_counts, offsets, sizeof(uint64_t) * count, hipMemcpyHostToDevice));
    TEPAI_HIP(h, bufs.alloc(&d_words, sizeof(uint32_t) * offsets[count]));
    TEPAI_HIP(h, launch_sample_write(d_rows, L, p->seed, s0, count, n_draws, d_counts, d_words, 0));
    TEPAI_HIP(h, hipMemcpy(words, d_words, sizeof(uint32_t) * offsets[count], hipMemcpyDeviceToHost));
  }
  return TEPAI_OK;
}

tepai_status tepai_workspace_size(tepai_handle* h, const tepai_problem* p, uint32_t count,
                                  size_t* bytes) {
  tepai_status st = validate(h, p);
  if (st != TEPAI_OK) return st;
  if (!bytes) return fail(h, TEPAI_EINVAL, "bytes is NULL");
  const Table t = build_table(*p);
  *bytes = layout(*p, (uint32_t)t.rows.size(), count).total;
  return TEPAI_OK;
}

tepai_status tepai_batch_create(tepai_handle* h, const tepai_problem* p, uint64_t first,
                                uint32_t count, void* workspace, size_t ws_bytes,
                                void* hip_stream, tepai_batch** out) {
  if (!h || !out) return TEPAI_EINVAL;
  *out = nullptr;
  tepai_status st = validate(h, p);
  if (st != TEPAI_OK) return st;
  if (count == 0) return fail(h, TEPAI_ERANGE, "count must be >= 1");
  if (first + count > p->n_samples) return fail(h, TEPAI_ERANGE, "batch beyond n_samples");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(h, TEPAI_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const Table t = build_table(*p);
  const uint32_t L = (uint32_t)t.rows.size();
  if (L > (uint32_t)kMaxRows) return fail(h, TEPAI_ERANGE, "more than 4096 table rows per Trotter step");
  const Layout lay = layout(*p, L, count);
  if (ws_bytes < lay.total) return fail(h, TEPAI_ENOMEM, "workspace smaller than tepai_workspace_size");
  TEPAI_HIP(h, hipSetDevice(h->device));
  auto* b = new tepai_batch;
  b->h = h;
  b->stream = (hipStream_t)hip_stream;
  b->ws = workspace;
  b->ws_bytes = lay.total;
  b->trotter_steps = p->trotter_steps;
  b->layers_done = 0;
  b->n_obs = p->n_obs;
  b->queue = nullptr;
  b->queue_grid = 0;
  b->rows = device_rows(*p, t);
  b->strings.resize(std::max<uint32_t>(p->n_strings, 1));
  for (uint32_t s = 0; s < p->n_strings; ++s) {
    DevString d{};
    d.n_ops = p->strings[s].n_ops;
    d.observable = p->strings[s].observable;
    d.coeff = p->strings[s].coeff;
    for (uint32_t i = 0; i < d.n_ops; ++i) {
      d.q[i] = p->strings[s].qubits[i];
      d.p[i] = p->strings[s].paulis[i];
    }
    b->strings[s] = d;
  }
  if (p->initial_bits && !p->initial_mps)
    b->bits.assign(p->initial_bits, p->initial_bits + p->n_qubits);
  else
    b->bits.assign(p->n_qubits, 0);
  b->caps.resize(2 * (size_t)count);
  for (uint32_t i = 0; i < count; ++i)
    b->caps[i] = p->chi_per_sample ? p->chi_per_sample[first + i] : p->chi_max;
  // workgroups start roughly in index order and a CU runs one sample at a
  // time, so the slots are launched by decreasing bond cap (stable): the
  // longest samples start first and the cheap ones fill the CUs that free up
  {
    uint32_t* ord = b->caps.data() + count;
    for (uint32_t i = 0; i < count; ++i) ord[i] = i;
    const uint32_t* cap = b->caps.data();
    std::stable_sort(ord, ord + count, [cap](uint32_t x, uint32_t y) { return cap[x] > cap[y]; });
  }
  char* ws = (char*)workspace;
  EngineArgs& a = b->args;
  a.rows = (const DevRow*)(ws + lay.rows);
  a.strings = (const DevString*)(ws + lay.strings);
  a.init_bits = (const uint8_t*)(ws + lay.bits);
  a.chi_caps = (const uint32_t*)(ws + lay.caps);
  a.launch_order = a.chi_caps + count;
  a.states = (SampleState*)(ws + lay.states);
  a.tensors = (double2*)(ws + lay.tensors);
  a.work = (double2*)(ws + lay.work);
  a.site_stride = lay.site_stride;
  a.work_stride = lay.work_stride;
  a.first_sample = p->sample_offset + first;
  a.seed = p->seed;
  a.mixed = p->precision == TEPAI_FP32_MIXED ? 1u : 0u;
  // complex64 contractions leave rounding noise near 1e-8 sigma_0 in the
  // spectrum; the mixed path does not count it as Schmidt rank
  a.cutoff = a.mixed ? std::max(p->svd_cutoff, kCutoffMixed) : p->svd_cutoff;
  a.stop_cos = a.mixed ? kStopCosMixed : kStopCosFp64;
  a.skip_tol = a.mixed ? kSkipMixed : kSkipFp64;
  a.per_gate = (p->flags & TEPAI_PER_GATE) ? 1u : 0u;
  a.qr_panel = 32;
  a.log_g1_step = t.log_step;
  a.l_eff = L;
  a.n = p->n_qubits;
  a.chi_max = p->chi_max;
  a.count = count;
  a.n_strings = p->n_strings;
  a.n_obs = p->n_obs;
  a.init_tensors = nullptr;
  a.init_off = nullptr;
  a.init_bond = nullptr;
  a.init_qubit = nullptr;
  a.init_centre = 0;
  a.init_max_bond = 0;
  const uint32_t n = p->n_qubits;
  if (const tepai_mps* m = p->initial_mps) {
    // stage the shared MPS in the batch (the caller's buffers are not kept)
    b->init_off.resize(n + 1);
    b->init_bond.assign(m->bond, m->bond + n + 1);
    b->init_qubit.resize(n);
    uint64_t off = 0;
    for (uint32_t k = 0; k < n; ++k) {
      b->init_off[k] = off;
      off += 2ull * m->bond[k] * m->bond[k + 1];
      b->init_qubit[k] = (uint16_t)(m->qubit_at ? m->qubit_at[k] : k);
    }
    b->init_off[n] = off;
    b->init_tensors.resize(off);
    std::memcpy(b->init_tensors.data(), m->tensors, sizeof(double2) * off);
    char* base = ws + lay.init;
    a.init_off = (const uint64_t*)base;
    base += align256(sizeof(uint64_t) * (n + 1));
    a.init_bond = (const uint32_t*)base;
    base += align256(sizeof(uint32_t) * (n + 1));
    a.init_qubit = (const uint16_t*)base;
    base += align256(sizeof(uint16_t) * n);
    a.init_tensors = (const double2*)base;
    a.init_centre = m->centre;
    a.init_max_bond = *std::max_element(m->bond, m->bond + n + 1);
  }
  hipError_t e = hipSuccess;
  if (p->flags & TEPAI_WORK_QUEUE) {
    // as many workgroups as the device holds at once
    b->queue = (uint32_t*)(ws + lay.queue);
    e = evolve_queue_grid(a, h->device, &b->queue_grid);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + lay.rows, b->rows.data(), sizeof(DevRow) * L, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + lay.strings, b->strings.data(), sizeof(DevString) * b->strings.size(), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + lay.bits, b->bits.data(), p->n_qubits, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + lay.caps, b->caps.data(), sizeof(uint32_t) * 2 * count, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && a.init_tensors) {
    e = hipMemcpyAsync((void*)a.init_off, b->init_off.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)a.init_bond, b->init_bond.data(), sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)a.init_qubit, b->init_qubit.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)a.init_tensors, b->init_tensors.data(), sizeof(double2) * b->init_tensors.size(), hipMemcpyHostToDevice, b->stream);
  }
  if (e == hipSuccess) e = launch_init(a, b->stream);
  // truncation on copy, for slots whose cap is below the shared start's bonds
  bool truncate = false;
  for (uint32_t i = 0; i < count; ++i) truncate = truncate || b->caps[i] < a.init_max_bond;
  if (e == hipSuccess && truncate) e = launch_start(a, b->stream);
  if (e != hipSuccess) {
    delete b;
    return fail(h, TEPAI_EDEVICE, std::string("batch set-up: ") + hipGetErrorString(e));
  }
  *out = b;
  return TEPAI_OK;
}

tepai_status tepai_batch_evolve(tepai_batch* b, uint32_t n_layers) {
  if (!b) return TEPAI_EINVAL;
  if (n_layers == 0) return TEPAI_OK;
  if ((uint64_t)b->layers_done + n_layers > b->trotter_steps)
    return fail(b->h, TEPAI_ERANGE, "evolve beyond the last Trotter step");
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  TEPAI_HIP(b->h, evolve_launch(b, n_layers));
  b->layers_done += n_layers;
  return TEPAI_OK;
}

tepai_status tepai_batch_observe(tepai_batch* b, double* d_values, double* d_weights) {
  if (!b) return TEPAI_EINVAL;
  if (!d_values || !d_weights) return fail(b->h, TEPAI_EINVAL, "output pointers NULL");
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  TEPAI_HIP(b->h, launch_observe(b->args, d_values, d_weights, b->stream));
  return TEPAI_OK;
}

tepai_status tepai_batch_stats(tepai_batch* b, tepai_sample_stats* out) {
  if (!b || !out) return TEPAI_EINVAL;
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  std::vector<SampleState> st(b->args.count);
  TEPAI_HIP(b->h, hipMemcpyAsync(st.data(), b->args.states, sizeof(SampleState) * st.size(), hipMemcpyDeviceToHost, b->stream));
  TEPAI_HIP(b->h, hipStreamSynchronize(b->stream));
  for (size_t i = 0; i < st.size(); ++i) {
    const SampleState& s = st[i];
    tepai_sample_stats& o = out[i];
    o.n_gates = s.n_gates;
    o.updates = s.updates;
    o.swap_updates = s.swap_updates;
    o.shifts = s.shifts;
    o.jacobi_sweeps = s.sweeps;
    o.nonconverged = s.nonconverged;
    o.ties = s.ties;
    o.sum_chi3 = s.sum_chi3;
    o.nominal_flops = s.nominal_flops;
    o.discarded = s.discarded;
    o.max_discarded = s.max_discarded;
    o.min_gap = s.min_gap;
    o.sign = s.sign;
    o.layer = s.layer;
    o.max_bond = s.max_bond;
    o.flags = s.flags;
  }
  return TEPAI_OK;
}

tepai_status tepai_batch_read_mps(tepai_batch* b, uint32_t slot, uint64_t capacity,
                                  uint32_t* bond, uint32_t* qubit_at, uint32_t* centre,
                                  uint64_t* n_values, double* tensors) {
  if (!b || !bond || !qubit_at || !centre || !n_values) return TEPAI_EINVAL;
  if (slot >= b->args.count) return fail(b->h, TEPAI_ERANGE, "slot out of range");
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  SampleState st;
  TEPAI_HIP(b->h, hipMemcpyAsync(&st, b->args.states + slot, sizeof(SampleState), hipMemcpyDeviceToHost, b->stream));
  TEPAI_HIP(b->h, hipStreamSynchronize(b->stream));
  const uint32_t n = b->args.n;
  uint64_t total = 0;
  for (uint32_t k = 0; k <= n; ++k) bond[k] = st.bond[k];
  for (uint32_t k = 0; k < n; ++k) {
    qubit_at[k] = st.qubit_at[k];
    total += 2ull * st.bond[k] * st.bond[k + 1];
  }
  *centre = (uint32_t)st.centre;
  *n_values = total;
  if (!tensors) return TEPAI_OK;
  if (total > capacity) return fail(b->h, TEPAI_ENOMEM, "tensor capacity too small");
  // each site's tensor is the first 2 bond[k] bond[k+1] values of its slot
  const bool mixed = b->args.mixed != 0;
  const size_t elem = mixed ? sizeof(float2) : sizeof(double2);
  const char* base = reinterpret_cast<const char*>(b->args.tensors);
  std::vector<float2> narrow(mixed ? total : 0);
  uint64_t at = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const uint64_t m = 2ull * st.bond[k] * st.bond[k + 1];
    const char* src = base + ((uint64_t)slot * n + k) * b->args.site_stride * elem;
    void* dst = mixed ? (void*)(narrow.data() + at) : (void*)(tensors + 2 * at);
    TEPAI_HIP(b->h, hipMemcpyAsync(dst, src, m * elem, hipMemcpyDeviceToHost, b->stream));
    at += m;
  }
  TEPAI_HIP(b->h, hipStreamSynchronize(b->stream));
  for (uint64_t i = 0; i < narrow.size(); ++i) {
    tensors[2 * i] = narrow[i].x;
    tensors[2 * i + 1] = narrow[i].y;
  }
  return TEPAI_OK;
}

void tepai_batch_destroy(tepai_batch* b) { delete b; }

tepai_status tepai_batch_autotune(tepai_batch* b, uint32_t n_layers, const uint32_t* candidates,
                                  uint32_t n_candidates, void* d_scratch, size_t scratch_bytes,
                                  double* ms, double* flops, uint32_t* chosen) {
  if (!b || !candidates || !chosen || n_candidates == 0) return TEPAI_EINVAL;
  if (n_layers == 0) return fail(b->h, TEPAI_ERANGE, "n_layers must be >= 1");
  for (uint32_t i = 0; i < n_candidates; ++i)
    if (candidates[i] < 1 || candidates[i] > 32)
      return fail(b->h, TEPAI_ERANGE, "QR panel widths are 1..32");
  if ((uint64_t)b->layers_done + n_layers > b->trotter_steps)
    return fail(b->h, TEPAI_ERANGE, "tuning steps beyond the last Trotter step");
  if (!d_scratch || scratch_bytes < b->ws_bytes)
    return fail(b->h, TEPAI_ENOMEM, "scratch smaller than the batch's workspace");
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  const uint32_t count = b->args.count;
  std::vector<SampleState> st(count);
  auto work = [&](double* out) -> hipError_t {   // summed nominal flops of the batch
    hipError_t e = hipMemcpyAsync(st.data(), b->args.states, sizeof(SampleState) * count,
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    double f = 0.0;
    for (const SampleState& s : st) f += s.nominal_flops;
    *out = f;
    return e;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_scratch, b->ws, b->ws_bytes, hipMemcpyDeviceToDevice, b->stream);
  double f0 = 0.0;
  if (e == hipSuccess) e = work(&f0);
  const uint32_t before = b->args.qr_panel;
  uint32_t best = before;
  double best_rate = -1.0;
  for (uint32_t i = 0; i < n_candidates && e == hipSuccess; ++i) {
    b->args.qr_panel = candidates[i];
    e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) e = evolve_launch(b, n_layers);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    double f1 = 0.0;
    if (e == hipSuccess) e = work(&f1);
    // back to the state before the candidate ran
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->ws, d_scratch, b->ws_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) break;
    if (ms) ms[i] = t;
    if (flops) flops[i] = f1 - f0;
    const double rate = t > 0.0f ? (f1 - f0) / t : 0.0;
    if (rate > best_rate) {
      best_rate = rate;
      best = candidates[i];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    b->args.qr_panel = before;
    return fail(b->h, TEPAI_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  }
  b->args.qr_panel = best;
  *chosen = best;
  return TEPAI_OK;
}

}  // extern "C"

struct tepai_step_graph {
  tepai_batch* b = nullptr;
  uint32_t n_layers = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~tepai_step_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

extern "C" {

tepai_status tepai_batch_capture_step(tepai_batch* b, uint32_t n_layers, double* d_values,
                                      double* d_weights, double* d_mean, double* d_std_err,
                                      tepai_step_graph** out) {
  if (!b || !out) return TEPAI_EINVAL;
  *out = nullptr;
  if (n_layers == 0) return fail(b->h, TEPAI_ERANGE, "n_layers must be >= 1");
  if (!d_values || !d_weights || !d_mean || !d_std_err)
    return fail(b->h, TEPAI_EINVAL, "output pointers NULL");
  if (!b->stream) return fail(b->h, TEPAI_EINVAL, "the null stream cannot be captured");
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  auto* g = new tepai_step_graph;
  g->b = b;
  g->n_layers = n_layers;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t work = evolve_launch(b, n_layers);
    if (work == hipSuccess) work = launch_observe(b->args, d_values, d_weights, b->stream);
    if (work == hipSuccess)
      work = launch_reduce(b->args.count, b->n_obs, d_values, d_weights, d_mean, d_std_err,
                           b->stream);
    const hipError_t end = hipStreamEndCapture(b->stream, &g->graph);   // always ends it
    e = work != hipSuccess ? work : end;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    delete g;
    (void)hipGetLastError();
    return fail(b->h, TEPAI_EDEVICE, std::string("step capture: ") + hipGetErrorString(e));
  }
  *out = g;
  return TEPAI_OK;
}

tepai_status tepai_step_graph_launch(tepai_step_graph* g) {
  if (!g) return TEPAI_EINVAL;
  tepai_batch* b = g->b;
  if ((uint64_t)b->layers_done + g->n_layers > b->trotter_steps)
    return fail(b->h, TEPAI_ERANGE, "evolve beyond the last Trotter step");
  TEPAI_HIP(b->h, hipSetDevice(b->h->device));
  TEPAI_HIP(b->h, hipGraphLaunch(g->exec, b->stream));
  b->layers_done += g->n_layers;
  return TEPAI_OK;
}

void tepai_step_graph_destroy(tepai_step_graph* g) { delete g; }

tepai_status tepai_reduce(tepai_handle* h, uint64_t count, uint32_t n_obs, const double* d_values,
                          const double* d_weights, double* d_mean, double* d_std_err,
                          void* hip_stream) {
  if (!h) return TEPAI_EINVAL;
  if (count == 0 || n_obs == 0) return fail(h, TEPAI_ERANGE, "count and n_obs must be >= 1");
  if (!d_values || !d_weights || !d_mean || !d_std_err) return fail(h, TEPAI_EINVAL, "NULL pointer");
  TEPAI_HIP(h, hipSetDevice(h->device));
  TEPAI_HIP(h, launch_reduce(count, n_obs, d_values, d_weights, d_mean, d_std_err, (hipStream_t)hip_stream));
  return TEPAI_OK;
}

tepai_status tepai_run(tepai_handle* h, const tepai_problem* p, uint32_t batch, double* mean,
                       double* std_err, double* weights, double* values,
                       tepai_sample_stats* stats) {
  if (!h) return TEPAI_EINVAL;
  tepai_status st = validate(h, p);
  if (st != TEPAI_OK) return st;
  if (!mean || !std_err || !weights) return fail(h, TEPAI_EINVAL, "output pointers NULL");
  if (p->n_obs == 0) return fail(h, TEPAI_ERANGE, "n_obs must be >= 1");
  TEPAI_HIP(h, hipSetDevice(h->device));
  const uint64_t ns = p->n_samples;
  size_t per1 = 0, per2 = 0;
  if ((st = tepai_workspace_size(h, p, 1, &per1)) != TEPAI_OK) return st;
  if ((st = tepai_workspace_size(h, p, 2, &per2)) != TEPAI_OK) return st;
  const size_t per = per2 - per1;
  size_t free_b = 0, total_b = 0;
  TEPAI_HIP(h, hipMemGetInfo(&free_b, &total_b));
  uint64_t B = batch ? batch : 1024;
  B = std::min<uint64_t>(B, ns);
  while (B > 1 && per1 + per * (B - 1) > free_b / 2) B /= 2;
  size_t ws_bytes = 0;
  if ((st = tepai_workspace_size(h, p, (uint32_t)B, &ws_bytes)) != TEPAI_OK) return st;
  DeviceBuffers bufs;
  void* ws = nullptr;
  double *d_v = nullptr, *d_w = nullptr, *d_m = nullptr, *d_se = nullptr;
  TEPAI_HIP(h, bufs.alloc(&ws, ws_bytes));
  TEPAI_HIP(h, bufs.alloc(&d_v, sizeof(double) * ns * p->n_obs));
  TEPAI_HIP(h, bufs.alloc(&d_w, sizeof(double) * ns));
  TEPAI_HIP(h, bufs.alloc(&d_m, sizeof(double) * p->n_obs));
  TEPAI_HIP(h, bufs.alloc(&d_se, sizeof(double) * p->n_obs));
  std::vector<tepai_sample_stats> sbuf(stats ? 0 : ns);
  tepai_sample_stats* sout = stats ? stats : sbuf.data();
  st = run_batches(h, p, (uint32_t)B, ws, ws_bytes, nullptr, d_v, d_w, d_m, d_se, sout);
  if (st != TEPAI_OK) return st;
  hipError_t e = hipMemcpy(mean, d_m, sizeof(double) * p->n_obs, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(std_err, d_se, sizeof(double) * p->n_obs, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(weights, d_w, sizeof(double) * ns, hipMemcpyDeviceToHost);
  if (e == hipSuccess && values) e = hipMemcpy(values, d_v, sizeof(double) * ns * p->n_obs, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(h, TEPAI_EDEVICE, std::string("copy-out: ") + hipGetErrorString(e));
  return numeric_status(h, p, sout, mean);
}

tepai_status tepai_run_noalloc(tepai_handle* h, const tepai_problem* p, void* hip_stream,
                               double* d_mean, double* d_std_err, double* d_weights,
                               double* d_values, tepai_sample_stats* stats) {
  if (!h) return TEPAI_EINVAL;
  tepai_status st = validate(h, p);
  if (st != TEPAI_OK) return st;
  if (!d_mean || !d_std_err || !d_weights || !d_values)
    return fail(h, TEPAI_EINVAL, "device output pointers NULL");
  if (p->n_obs == 0) return fail(h, TEPAI_ERANGE, "n_obs must be >= 1");
  if (!h->scratch)
    return fail(h, TEPAI_EDEVICE, "no device address for the fixed workspace (" + h->scratch_err + ")");
  TEPAI_HIP(h, hipSetDevice(h->device));
  const uint64_t ns = p->n_samples;
  const size_t cap = TEPAI_NOALLOC_BYTES;
  size_t per1 = 0, per2 = 0;
  if ((st = tepai_workspace_size(h, p, 1, &per1)) != TEPAI_OK) return st;
  if ((st = tepai_workspace_size(h, p, 2, &per2)) != TEPAI_OK) return st;
  if (per1 > cap)
    return fail(h, TEPAI_ENOMEM, "one sample needs " + std::to_string(per1) +
                                     " bytes of workspace, more than the fixed " +
                                     std::to_string(cap));
  // as many samples per batch as the array holds
  const size_t per = per2 - per1;
  uint64_t B = per ? 1 + (cap - per1) / per : ns;
  B = std::min<uint64_t>(std::min<uint64_t>(B, ns), 0xffffffffull);
  size_t need = 0;
  for (;;) {
    if ((st = tepai_workspace_size(h, p, (uint32_t)B, &need)) != TEPAI_OK) return st;
    if (need <= cap || B == 1) break;
    B -= 1;
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  std::vector<tepai_sample_stats> sbuf(stats ? 0 : ns);   // host memory
  tepai_sample_stats* sout = stats ? stats : sbuf.data();
  st = run_batches(h, p, (uint32_t)B, h->scratch, cap, stream, d_values, d_weights, d_mean,
                   d_std_err, sout);
  if (st != TEPAI_OK) return st;
  std::vector<double> mean(p->n_obs);
  TEPAI_HIP(h, hipMemcpyAsync(mean.data(), d_mean, sizeof(double) * p->n_obs,
                              hipMemcpyDeviceToHost, stream));
  TEPAI_HIP(h, hipStreamSynchronize(stream));
  return numeric_status(h, p, sout, mean.data());
}

}  // extern "C"
