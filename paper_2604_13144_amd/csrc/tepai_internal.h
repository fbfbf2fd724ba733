// Internal layout shared by the host and device halves of libtepai.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "tepai.h"

namespace tepai {

constexpr int kMaxQubits = 256;
constexpr int kMaxChi = 256;
constexpr int kMaxRows = 4096;        // PAI table rows per Trotter step
constexpr int kMaxStringOps = 8;
constexpr int kThreads = 512;         // engine block: eight wave64 wavefronts
constexpr int kMaxSweeps = 60;           // Jacobi sweep cap per factorisation
constexpr double kStopCosFp64 = 1e-8;    // FP64 path: residual ~1e-16
constexpr double kStopCosMixed = 1e-5;   // mixed path: residual ~1e-10
constexpr double kCutoffMixed = 1e-7;    // mixed path: relative singular-value floor
constexpr double kSkipFp64 = 0x1p-53;    // FP64 path: Jacobi pair threshold u sqrt(R)
constexpr double kSkipMixed = 1e-15;     // mixed path: inputs carry ~1e-7 errors anyway

// One row of the PAI table: a (sub-)rotation of one Trotter step.
struct DevRow {
  uint64_t t1, t2;      // 63-bit thresholds: v < t1 -> A, v < t2 -> B, else C
  double cb, sb;        // setting B = cb I - i sb P: sb = sin(sign(theta) Delta / 2), or
                        // sin(theta / 2) for the deterministic product formula
  uint32_t nq;          // 1 or 2
  uint32_t q0, q1;      // qubits (q1 unused when nq == 1)
  uint32_t p0, p1;      // Pauli codes 1..3
  uint32_t pad;
};

struct DevString {
  uint32_t n_ops, observable;
  uint32_t q[kMaxStringOps];
  uint32_t p[kMaxStringOps];
  double coeff;
};

// Per-sample state that persists between launches (one per batch slot).
struct SampleState {
  int32_t centre;
  int32_t sign;
  uint32_t layer;
  uint32_t flags;
  uint32_t chi_cap;
  uint32_t max_bond;
  uint64_t n_gates, updates, swap_updates, shifts, sweeps, nonconverged, ties;
  double sum_chi3, nominal_flops, discarded, max_discarded, min_gap;
  uint16_t bond[kMaxQubits + 1];   // bond[k] = dimension between sites k-1 and k
  uint16_t qubit_at[kMaxQubits];   // chain order: qubit held by each site
};

// Everything a kernel launch needs; passed by value.
struct EngineArgs {
  const DevRow* rows;
  const DevString* strings;
  const uint8_t* init_bits;
  const uint32_t* chi_caps;   // [count] per-slot bond caps
  const uint32_t* launch_order;  // [count] slot run by workgroup b (decreasing cap)
  SampleState* states;
  double2* tensors;       // [count][n][site_stride]
  double2* work;          // [count][work_stride]
  uint64_t site_stride;   // complex elements per site slot: 2 chi_max^2
  uint64_t work_stride;   // complex elements of scratch per sample: 3 max((2 chi_max)^2, kThreads)
  uint64_t first_sample;  // global index of slot 0
  uint64_t seed;
  double cutoff;
  double stop_cos;        // Jacobi stop: a sweep whose rotated pairs all had cosine <= this
  double skip_tol;        // Jacobi skips a pair with |x^H y| <= skip_tol sqrt(R) |x||y|
  double log_g1_step;
  uint32_t l_eff;
  uint32_t n;
  uint32_t chi_max;
  uint32_t count;
  uint32_t n_strings;
  uint32_t n_obs;
  uint32_t mixed;         // 1: TEPAI_FP32_MIXED (complex64 site tensors)
  uint32_t per_gate;      // 1: TEPAI_PER_GATE (no fusion of same-pair runs)
  // shared starting MPS (null init_tensors: computational-basis start)
  const double2* init_tensors;   // packed site tensors, site k at init_off[k]
  const uint64_t* init_off;      // [n + 1]
  const uint32_t* init_bond;     // [n + 1]
  const uint16_t* init_qubit;    // [n]
  uint32_t init_centre;
  uint32_t init_max_bond;        // largest bond of the shared start (0: none)
  uint32_t qr_panel;             // QR steps per panel of lazy trailing updates (1..32)
};

// Engine instantiation (rows per lane) for matrices of up to 2 chi_max rows.
inline int rows_per_lane(uint32_t chi_max) {
  const uint32_t r = 2 * chi_max;
  return r <= 64 ? 1 : r <= 128 ? 2 : r <= 256 ? 4 : 8;
}

// Kernel launchers (kernels.hip; the work-queue form in queue.hip).
hipError_t launch_init(const EngineArgs& a, hipStream_t s);
hipError_t launch_start(const EngineArgs& a, hipStream_t s);
hipError_t launch_evolve(const EngineArgs& a, uint32_t n_layers, hipStream_t s);
// Work-queue form: `grid` workgroups (clamped to [1, count]) take the slots
// in launch order from the counter at `queue`, which it resets first.
hipError_t launch_evolve_queue(const EngineArgs& a, uint32_t n_layers, uint32_t* queue,
                               uint32_t grid, hipStream_t s);
// Workgroups of the work-queue kernel for these arguments that the device
// holds at once: resident workgroups per CU times the CU count.
hipError_t evolve_queue_grid(const EngineArgs& a, int device, uint32_t* grid);
hipError_t launch_observe(const EngineArgs& a, double* d_values, double* d_weights, hipStream_t s);
hipError_t launch_reduce(uint64_t count, uint32_t n_obs, const double* v, const double* w,
                         double* mean, double* se, hipStream_t s);
hipError_t launch_sample_count(const DevRow* rows, uint32_t l_eff, uint64_t seed,
                               uint64_t first_sample, uint64_t count, uint64_t n_draws,
                               uint64_t* d_counts, int8_t* d_signs, hipStream_t s);
hipError_t launch_sample_write(const DevRow* rows, uint32_t l_eff, uint64_t seed,
                               uint64_t first_sample, uint64_t count, uint64_t n_draws,
                               const uint64_t* d_offsets, uint32_t* d_words, hipStream_t s);

}  // namespace tepai
