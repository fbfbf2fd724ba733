// Device side of libtepai: TE-PAI sampling, the per-sample MPS engine,
// observables and the weighted reduction, written for gfx950 (wave64).
//
// One workgroup owns one sample for the whole launch.  It draws the sample's
// gate settings itself (Philox4x32-10, counter = (g_lo, g_hi, sample, 1),
// key = seed), so no gate stream is ever materialised, and applies them to
// the sample's MPS, which lives in HBM in the caller's workspace:
//   site k of slot b: tensors + (b * n + k) * site_stride, layout A[a][s][c]
//   (row-major, actual bond dimensions), complex128 as z2.
// Every factorisation is a one-sided (Hestenes) Jacobi SVD done by the eight
// waves of the workgroup.  Each 16-lane row of a wave owns one column pair at
// a time (E = 4 RPL matrix rows per lane), so the three inner products of a
// pair are reduced with four DPP steps inside the row and a wave rotates four
// pairs at once.  A sweep visits the columns, sorted by decreasing norm
// (de Rijk's ordering), in blocks of JB: one block stays in registers (one
// column per row) while every later block is staged through LDS and each of
// its columns meets each register column once; the pairs inside a block are
// then done in LDS.  Every column pair is rotated exactly once per sweep, as
// in the cyclic method, while HBM sees each block only a few times per sweep.
//
// The engine is instantiated for RPL = 1, 2, 4, 8 (matrices of up to 64 RPL
// rows, i.e. chi_max <= 32 RPL), which sizes registers and LDS blocks.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <cmath>
#include <cstdint>

#include "tepai_internal.h"

namespace tepai {
namespace {

constexpr int NT = kThreads;
constexpr int NW = kThreads / 64;
constexpr int NROWS = NT / 16;    // 16-lane rows per block

template <int RPL>
struct JCfg {
  static constexpr int E = 4 * RPL;                    // matrix rows per lane of a 16-lane row
  static constexpr int JB = RPL <= 4 ? NROWS : NROWS / 2;   // columns per Jacobi block
  static constexpr int LR = 16 * E + 1;                // LDS column stride (padded)
};

// LDS staging block size (complex elements) that serves the Jacobi of every
// row class up to RPL (a launch runs smaller matrices with smaller E).
template <int RPL>
constexpr int jl_size() {
  constexpr int own = JCfg<RPL>::JB * JCfg<RPL>::LR;
  if constexpr (RPL > 1) {
    constexpr int half = jl_size<RPL / 2>();
    return own > half ? own : half;
  } else {
    return own;
  }
}

// ---------------------------------------------------------------- complex
// complex128 as a native two-lane vector (loads/stores of 16 bytes), with
// pointer types that pin LDS (ds_*) and global (global_*) address spaces.
typedef double z2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) z2 lz2;
typedef __attribute__((address_space(1))) z2 gz2;
typedef __attribute__((address_space(3))) double ld;
// complex64 storage of the mixed-precision path's site tensors
typedef float f2 __attribute__((ext_vector_type(2)));
template <typename T>
using glob = __attribute__((address_space(1))) T;

__device__ __forceinline__ z2 cmk(double r, double i) {
  z2 v;
  v.x = r;
  v.y = i;
  return v;
}
__device__ __forceinline__ z2 cadd(z2 a, z2 b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ z2 cmul(z2 a, z2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ z2 cconj(z2 a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ z2 cscale(z2 a, double s) { return cmk(a.x * s, a.y * s); }

// Site-tensor element type: complex128, or complex64 on the mixed path.
template <bool MIX>
using TSite = typename std::conditional<MIX, f2, z2>::type;
__device__ __forceinline__ z2 toz(z2 v) { return v; }
__device__ __forceinline__ z2 toz(f2 v) { return cmk((double)v.x, (double)v.y); }
template <typename T>
__device__ __forceinline__ T fromz(z2 v);
template <>
__device__ __forceinline__ z2 fromz<z2>(z2 v) { return v; }
template <>
__device__ __forceinline__ f2 fromz<f2>(z2 v) {
  f2 r;
  r.x = (float)v.x;
  r.y = (float)v.y;
  return r;
}
// acc += a * b
__device__ __forceinline__ void cfma(z2& acc, z2 a, z2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__device__ __forceinline__ void cfmac(z2& acc, z2 a, z2 b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// key advanced by the Weyl constants between rounds.
__device__ __forceinline__ uint64_t philox_u64(uint64_t seed, uint32_t sample, uint64_t g,
                                               uint32_t stream) {
  uint32_t c0 = (uint32_t)g, c1 = (uint32_t)(g >> 32), c2 = sample, c3 = stream;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return ((uint64_t)c1 << 32) | c0;
}

__device__ __forceinline__ uint8_t draw_setting(const DevRow& row, uint64_t seed, uint32_t sample,
                                                uint64_t g) {
  const uint64_t v = philox_u64(seed, sample, g, 1u) >> 1;
  return v < row.t1 ? 0 : (v < row.t2 ? 1 : 2);
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// max into a non-negative LDS double (compare-and-swap on the bit pattern,
// which orders like the value for non-negative doubles)
__device__ __forceinline__ void atomicMax_double(double* a, double v) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(a);
  unsigned long long cur = *p;
  const unsigned long long nv = (unsigned long long)__double_as_longlong(v);
  while (nv > cur) {
    const unsigned long long prev = atomicCAS(p, cur, nv);
    if (prev == cur) break;
    cur = prev;
  }
}


// Ordering key of a squared column norm: a NaN sorts below every number, so
// the rank computations below always produce a permutation (a non-finite
// matrix must still leave every index in range).
__device__ __forceinline__ double norm_key(double v) { return v == v ? v : -1.0; }

// 1/sqrt(x) and 1/x from the hardware estimates refined by two Newton steps
// (each step squares the relative error) for the rotation parameters.
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

// Move a double between lanes with a DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}

// Sum over the 16 lanes of each DPP row.  Every step adds the values of two
// lanes that exchange with each other (xor 1, xor 2, mirror, half-mirror), so
// both partners add the same two operands and all 16 lanes end with the
// bitwise-identical sum (Q0 + Q3) + (Q1 + Q2) of the four quad sums; lanes
// that later derive a rotation from these sums therefore all apply the same
// rotation, even where the sign of |y|^2 - |x|^2 is decided by rounding.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_f64<0x140>(v);   // row_mirror: lane <-> 15 - lane (quad q <-> 3 - q)
  v += dpp_f64<0x141>(v);   // row_half_mirror: quad 0 <-> 1, quad 2 <-> 3
  return v;
}

// Workgroup barrier for data that waves hand to each other through global
// memory (site tensors, the scratch matrices).  The compiler's
// workgroup-scope fence around __syncthreads waits only for LDS operations
// (outstanding vector memory operations are not awaited when a work-group
// runs on one CU), so a wave's global store, or a global load still in
// flight, could race with another wave's access after the barrier: measured
// as occasional stale columns (errors of the order of the last Jacobi sweep's
// rotations) in the factorisations.  Waiting for every vector memory
// operation of the wave first orders those hand-offs.
__device__ __forceinline__ void sync_block() {
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// Fixed-order block sum (deterministic); all threads get the result.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  sync_block();
  if (lane == 0) red[wv] = v;
  sync_block();
  double t = 0.0;
  for (int w = 0; w < NW; ++w) t += red[w];
  sync_block();
  return t;
}

// ---------------------------------------------------------------- Paulis
// Element (r, c) of Pauli p (1 = X, 2 = Y, 3 = Z).
__device__ __forceinline__ z2 pauli_el(uint32_t p, int r, int c) {
  if (p == 1) return cmk(r != c ? 1.0 : 0.0, 0.0);
  if (p == 2) return r == c ? cmk(0.0, 0.0) : cmk(0.0, r == 0 ? -1.0 : 1.0);
  if (p == 3) return cmk(r == c ? (r == 0 ? 1.0 : -1.0) : 0.0, 0.0);
  return cmk(r == c ? 1.0 : 0.0, 0.0);
}

// -------------------------------------------------------- shared memory
struct Shared {
  z2 G[16];              // operator of the two-site update in progress (site order)
  z2 pM[16];             // pending two-site operator, (qa, qb) order
  z2 pLa[4], pLb[4];     // its local factors while it holds only C settings
  z2 pPhase;
  double sig2[2 * kMaxChi];   // squared column norms after Jacobi
  double jn[NROWS];           // squared norms of the columns staged in LDS
  double red[NW * 4];
  uint16_t perm[2 * kMaxChi]; // columns by descending norm
  uint16_t order[2 * kMaxChi];// Jacobi sweep order
  uint16_t piv[2 * kMaxChi];  // column pivots of the QR preconditioner
  double qr_vn0[2 * kMaxChi]; // QR: column norms at the start of the panel
  z2 qr_t[32];                // QR: u_k^H u_i for the panel's reflectors i < k
  z2 qr_w[32];                // QR: W_i(pivot column) of the panel's reflectors
  int qr_p, qr_mark, qr_done;
  double qr_v, qr_k;
  uint16_t bond[kMaxQubits + 1];
  uint16_t qubit_at[kMaxQubits];
  uint16_t site_of[kMaxQubits];
  uint8_t choice[kMaxRows];
  int flag;
  double tmax;
  int p_active, p_has, p_qa, p_qb;
  int centre;
  // statistics (thread 0 writes)
  uint64_t updates, swap_updates, shifts, sweeps, nonconv, ties, n_gates;
  double sum_chi3, flops, discarded, max_disc, min_gap;
  int n_c;
  uint32_t max_bond;
  uint32_t sflags;       // TEPAI_SAMPLE_* bits
  int qr_panel;          // QR steps per panel (1..32; the autotuned parameter)
};

struct Slot {
  void* T;   // site tensors of this sample (z2, or f2 on the mixed path)
  z2* Y0;     // scratch: factorised matrix (kept)
  z2* W;      // scratch: Jacobi working copy
  z2* P;      // scratch: projections
  z2* Jl;     // LDS staging block of the Jacobi sweeps
  uint64_t ss;     // site stride
  double stop;       // Jacobi stops after a sweep whose pair cosines were all <= stop
  double skip;       // Jacobi skips a pair with |x^H y| <= skip sqrt(R) |x||y|
  double cutoff;
  uint32_t chi;
  uint32_t n;
  uint32_t per_gate;  // every two-qubit gate its own update (no run fusion)
};

template <typename TS>
__device__ __forceinline__ TS* site(const Slot& s, int k) { return (TS*)s.T + (uint64_t)k * s.ss; }

__device__ double svd_flops(double m, double n) {
  if (m < n) {
    const double t = m;
    m = n;
    n = t;
  }
  return 4.0 * (4.0 * m * m * n + 8.0 * m * n * n + 9.0 * n * n * n);
}

// ---------------------------------------------------------------- Jacobi
// Round-robin pairing of Cp (even) columns: Cp-1 rounds of Cp/2 disjoint pairs.
__device__ __forceinline__ void rr_pair(int round, int k, int Cp, int& p, int& q) {
  const int m = Cp - 1;
  if (k == 0) {
    p = m;
    q = round;
  } else {
    p = (round + k) % m;
    q = (round - k + m) % m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// Sum over G consecutive 16-lane rows of a wave (G = 1, 2, 4).  The 16-lane
// sum is symmetric (row16_sum); the row pairs then exchange with the gfx950
// permlane swaps (rows 2k <-> 2k+1, then halves), and both partners add the
// same two operands in the same order, so all G rows end bitwise-equal.
template <int W>
__device__ __forceinline__ double swap_add(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  if constexpr (W == 16) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  }
}

template <int G>
__device__ __forceinline__ double rows_sum(double v) {
  v = row16_sum(v);
  if constexpr (G >= 2) v = swap_add<16>(v);
  if constexpr (G >= 4) v = swap_add<32>(v);
  return v;
}

// Rotation parameters from alpha = |x|^2, beta = |y|^2, gamma = x^H y:
// zeta = (beta - alpha) / (2 |gamma|), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1/sqrt(1+t^2), s = c t, e^{i phi} = gamma/|gamma|.  The rotation
// x <- c x - s e^{-i phi} y, y <- s e^{i phi} x + c y zeroes x^H y and moves
// t |gamma| of squared norm from x to y: |x'|^2 = alpha - t|gamma|,
// |y'|^2 = beta + t|gamma| (the two-sided Jacobi update of the 2 x 2 Gram
// matrix).
struct Rot {
  double c, sr, si, t, tg;   // cosine, s e^{i phi} = sr + i si, tan, t |gamma|
};

__device__ __forceinline__ Rot rot_params(double al, double be, double gr, double gi, double g2) {
  Rot r;
  const double ig = rsq_nr(g2);
  const double zeta = (be - al) * 0.5 * ig;
  const double q = 1.0 + zeta * zeta;
  const double hq = q * rsq_nr(q);
  r.t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(zeta) + hq);
  r.c = rsq_nr(1.0 + r.t * r.t);
  const double s = r.c * r.t;
  r.sr = s * (gr * ig);
  r.si = s * (gi * ig);
  r.tg = r.t * (g2 * ig);
  return r;
}

// x <- c x - conj(s e^{i phi}) y, y <- (s e^{i phi}) x + c y: three real
// multiply-adds per output component.
__device__ __forceinline__ void rot_apply(const Rot& r, z2& a, z2& b) {
  const z2 x = a, y = b;
  a = cmk(fma(-r.si, y.y, fma(-r.sr, y.x, r.c * x.x)), fma(r.si, y.x, fma(-r.sr, y.y, r.c * x.y)));
  b = cmk(fma(-r.si, x.y, fma(r.sr, x.x, r.c * y.x)), fma(r.si, x.x, fma(r.sr, x.y, r.c * y.y)));
}

// A squared norm carried through rotations by the update above loses
// accuracy when most of it cancels; below this fraction of its previous
// value it is recomputed from the column.
constexpr double kNormRecompute = 0.25;

// One Jacobi rotation per 16-lane row: the row's lanes hold E elements each
// of the column x in registers (element e of lane l is matrix row l + 16 e)
// with its squared norm al; the partner column y is read from LDS once and
// held in registers between the inner product and the update, and its
// squared norm lives in LDS at yn.  All E elements are processed without
// per-element conditions (matrix rows beyond R are zero in registers and in
// LDS and stay zero), so the element loop is straight-line code that the
// compiler can interleave.  Rows that are inactive or
// already orthogonal to tolerance leave both columns untouched.  Returns
// the squared cosine |x^H y|^2 / (|x|^2 |y|^2) of the pair before the
// rotation (no division or square root on the rotation's path), or -1 when
// this row did not rotate.
template <int E>
__device__ __forceinline__ double rotate_rows(z2 (&x)[E], double& al, lz2* y, ld* yn, int l16,
                                              bool active, double tiny, double tol2) {
  double gr = 0.0, gi = 0.0;
  z2 yv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const z2 b = y[l16 + 16 * e];
    yv[e] = b;
    gr = fma(x[e].x, b.x, fma(x[e].y, b.y, gr));
    gi = fma(x[e].x, b.y, fma(-x[e].y, b.x, gi));
  }
  gr = row16_sum(gr);
  gi = row16_sum(gi);
  const double be = *yn;
  const double g2 = gr * gr + gi * gi;
  const bool rot = active && al > tiny && be > tiny && g2 > tol2 * al * be;
  double tabs = -1.0;
  if (rot) {
    const Rot r = rot_params(al, be, gr, gi, g2);
    tabs = g2 * rcp_nr(al * be);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      rot_apply(r, x[e], yv[e]);
      y[l16 + 16 * e] = yv[e];
    }
    double an = al - r.tg, bn = be + r.tg;
    if (an < kNormRecompute * al) {
      double a = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) a = fma(x[e].x, x[e].x, fma(x[e].y, x[e].y, a));
      an = row16_sum(a);
    }
    if (bn < kNormRecompute * be) {
      double a = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) a = fma(yv[e].x, yv[e].x, fma(yv[e].y, yv[e].y, a));
      bn = row16_sum(a);
    }
    al = an;
    if (l16 == 0) *yn = bn;
  }
  return tabs;
}

// One rotation of the LDS columns xp and yq, shared by G consecutive rows of
// a wave: the row with part h (e0 = h EG) handles elements [e0, e0 + EG) of
// both columns (EG = E / G), and the inner product and any norm
// recomputation are summed over the G rows.  The squared norms live in LDS
// at pn and qn; the part-0 row writes their updates.
template <int EG, int G>
__device__ __forceinline__ double rotate_split(lz2* xp, lz2* yq, ld* pn, ld* qn, int e0,
                                               int l16, bool first, bool active,
                                               double tiny, double tol2) {
  z2 xv[EG], yv[EG];
  double gr = 0.0, gi = 0.0;
#pragma unroll
  for (int e = 0; e < EG; ++e) {
    xv[e] = xp[l16 + 16 * (e0 + e)];
    yv[e] = yq[l16 + 16 * (e0 + e)];
    gr = fma(xv[e].x, yv[e].x, fma(xv[e].y, yv[e].y, gr));
    gi = fma(xv[e].x, yv[e].y, fma(-xv[e].y, yv[e].x, gi));
  }
  gr = rows_sum<G>(gr);
  gi = rows_sum<G>(gi);
  const double al = *pn, be = *qn;
  const double g2 = gr * gr + gi * gi;
  const bool rot = active && al > tiny && be > tiny && g2 > tol2 * al * be;
  double tabs = -1.0;
  if (rot) {
    const Rot r = rot_params(al, be, gr, gi, g2);
    tabs = g2 * rcp_nr(al * be);
#pragma unroll
    for (int e = 0; e < EG; ++e) {
      rot_apply(r, xv[e], yv[e]);
      xp[l16 + 16 * (e0 + e)] = xv[e];
      yq[l16 + 16 * (e0 + e)] = yv[e];
    }
    double an = al - r.tg, bn = be + r.tg;
    if (an < kNormRecompute * al) {
      double a = 0.0;
#pragma unroll
      for (int e = 0; e < EG; ++e) a = fma(xv[e].x, xv[e].x, fma(xv[e].y, xv[e].y, a));
      an = rows_sum<G>(a);
    }
    if (bn < kNormRecompute * be) {
      double a = 0.0;
#pragma unroll
      for (int e = 0; e < EG; ++e) a = fma(yv[e].x, yv[e].x, fma(yv[e].y, yv[e].y, a));
      bn = rows_sum<G>(a);
    }
    if (first && l16 == 0) {
      *pn = an;
      *qn = bn;
    }
  }
  return tabs;
}

// Column <-> row registers.  From/to global memory only rows < R exist; the
// register (and LDS) copies are zero-padded to 16 E rows.
template <int E>
__device__ __forceinline__ void row_load_g(z2 (&x)[E], const gz2* col, int R, int l16) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int r = l16 + 16 * e;
    const z2 v = col[r < R ? r : R - 1];     // in-bounds load, no branch
    x[e] = r < R ? v : cmk(0.0, 0.0);
  }
}

template <int E>
__device__ __forceinline__ void row_store_g(const z2 (&x)[E], gz2* col, int R, int l16) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int r = l16 + 16 * e;
    if (r < R) col[r] = x[e];
  }
}

template <int E>
__device__ __forceinline__ void row_load_l(z2 (&x)[E], const lz2* col, int l16) {
#pragma unroll
  for (int e = 0; e < E; ++e) x[e] = col[l16 + 16 * e];
}

template <int E>
__device__ __forceinline__ void row_store_l(const z2 (&x)[E], lz2* col, int l16) {
#pragma unroll
  for (int e = 0; e < E; ++e) col[l16 + 16 * e] = x[e];
}

template <int E>
__device__ __forceinline__ double row_norm2(const z2 (&x)[E]) {
  double a = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) a = fma(x[e].x, x[e].x, fma(x[e].y, x[e].y, a));
  return row16_sum(a);
}

// One-sided Jacobi on the columns of W (R x C, column-major, R <= 64 RPL):
// on return the columns are mutually orthogonal (W <- W V).  Jl_ is the LDS
// staging block (JB columns).  Returns the number of sweeps, or -1 when the
// sweep cap was reached.
template <int RPL>
__device__ __noinline__ int jacobi(z2* W_, int R, int C, Shared& sh, z2* Jl_, double stop,
                                   double skip) {
  using K = JCfg<RPL>;
  constexpr int E = K::E, JB = K::JB, LR = K::LR;
  gz2* W = (gz2*)W_;
  lz2* Jl = (lz2*)Jl_;
  ld* jn = (ld*)sh.jn;
  const int l16 = threadIdx.x & 15, row = threadIdx.x >> 4;
  if (C < 2) return 0;
  // column norms (also the first sweep's ordering) and ||W||_F^2
#pragma unroll 1
  for (int j = row; j < C; j += NROWS) {
    z2 x[E];
    row_load_g<E>(x, W + (uint64_t)j * R, R, l16);
    const double a = row_norm2<E>(x);
    if (l16 == 0) sh.sig2[j] = a;
  }
  sync_block();
  double fro2 = 0.0;
  for (int j = 0; j < C; ++j) fro2 += sh.sig2[j];
  const double tiny = 1e-32 * fro2;     // sigma_j^2 below this is numerically zero
  const double tol = skip * sqrt((double)R);
  const double tol2 = tol * tol;
  const int nb = (C + JB - 1) / JB;
#pragma unroll 1
  for (int sweep = 1; sweep <= kMaxSweeps; ++sweep) {
    // order columns by decreasing norm (ties by index): de Rijk's ordering
    for (int j = threadIdx.x; j < C; j += NT) {
      const double v = norm_key(sh.sig2[j]);
      int rank = 0;
#pragma unroll 4
      for (int i = 0; i < C; ++i) {
        const double u = norm_key(sh.sig2[i]);
        rank += (u > v) || (u == v && i < j);
      }
      sh.order[rank] = (uint16_t)j;
    }
    if (threadIdx.x == 0) {
      sh.flag = 0;
      sh.tmax = 0.0;
    }
    sync_block();
    double tmx = -1.0;     // largest squared cosine of the pairs this thread's row rotated
#pragma unroll 1
    for (int I = 0; I < nb; ++I) {
      const int pi = I * JB + row;                       // position of this row's column
      const bool ai = row < JB && pi < C;
      const int ci = ai ? sh.order[pi] : 0;
      z2 xi[E];
      if (ai) {
        row_load_g<E>(xi, W + (uint64_t)ci * R, R, l16);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) xi[e] = cmk(0.0, 0.0);
      }
      double al = row_norm2<E>(xi);      // carried through the rotations
#pragma unroll 1
      for (int J = I + 1; J < nb; ++J) {
        if (row < JB) {   // stage block J: one column per row
          const int pj = J * JB + row;
          z2 y[E];
          if (pj < C) {
            row_load_g<E>(y, W + (uint64_t)sh.order[pj] * R, R, l16);
          } else {
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = cmk(0.0, 0.0);
          }
          row_store_l<E>(y, Jl + row * LR, l16);
          const double b = row_norm2<E>(y);
          if (l16 == 0) jn[row] = b;
        }
        sync_block();
        // Cross pairs in 4 x 4 tiles: wave w (rows 4w..4w+3) owns I-tile w and
        // visits the J-tiles (w + R) mod NTILE; inside a tile its four rows
        // meet the four J columns in four wave-local rounds (LDS is in order
        // within a wave), so the workgroup synchronises once per tile
        // rotation instead of once per round.
        constexpr int NTILE = JB / 4;
        const int wv = row >> 2, r4 = row & 3;
#pragma unroll 1
        for (int Rr = 0; Rr < NTILE; ++Rr) {
          if (wv < NTILE) {
            const int tb = (wv + Rr) % NTILE;
#pragma unroll 1
            for (int r = 0; r < 4; ++r) {
              const int jj = 4 * tb + ((r4 + r) & 3);
              const bool act = ai && J * JB + jj < C;
              tmx = fmax(tmx, rotate_rows<E>(xi, al, Jl + jj * LR, jn + jj, l16, act, tiny, tol2));
              __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
          }
          sync_block();
        }
        if (row < JB && J * JB + row < C) {
          z2 y[E];
          row_load_l<E>(y, Jl + row * LR, l16);
          row_store_g<E>(y, W + (uint64_t)sh.order[J * JB + row] * R, R, l16);
        }
        sync_block();
      }
      // pairs inside block I, in LDS (round-robin over the block's columns,
      // rounded up to an even count); each of the pairs of a round is shared
      // by G rows of one wave, so every row of the workgroup works
      if (row < JB) {
        row_store_l<E>(xi, Jl + row * LR, l16);
        if (l16 == 0) jn[row] = al;
      }
      sync_block();
      {
        constexpr int G = NROWS / (JB / 2), EG = E / G;
        const int k = row / G, h = row - k * G;
        const int ncol = (C - I * JB) < JB ? (C - I * JB) : JB;
        const int Cp = ncol + (ncol & 1);
#pragma unroll 1
        for (int round = 0; round < Cp - 1; ++round) {
          int p = 0, q = 1;
          const bool pk = k < Cp / 2;
          if (pk) rr_pair(round, k, Cp, p, q);
          const bool act = pk && I * JB + q < C;
          tmx = fmax(tmx, rotate_split<EG, G>(Jl + p * LR, Jl + q * LR, jn + p, jn + q, h * EG,
                                               l16, h == 0, act, tiny, tol2));
          sync_block();
        }
      }
      // write block I back and record its final column norms for the next order
      if (ai) {
        z2 x[E];
        row_load_l<E>(x, Jl + row * LR, l16);
        row_store_g<E>(x, W + (uint64_t)ci * R, R, l16);
        const double a = row_norm2<E>(x);
        if (l16 == 0) sh.sig2[ci] = a;
      }
      sync_block();
    }
    // Stop when no pair rotated, or when every pair this sweep rotated had a
    // cosine |x^H y| / (|x||y|) <= stop: the sweep then leaves a
    // non-orthogonality of ~stop^2 (1e-16 at the FP64 path's 1e-8, where a
    // further sweep would find nothing above the tolerance).  The test is on
    // the cosine, not on the rotation's tangent, which is smaller by the
    // ratio of the two norms: a column far smaller than its partner can meet
    // a tangent bound while still far from orthogonal to it.
    tmx = wave_max(tmx);
    if ((threadIdx.x & 63) == 0 && tmx >= 0.0) {
      sh.flag = 1;
      atomicMax_double(&sh.tmax, tmx);
    }
    sync_block();
    const int rotated = sh.flag;
    const double tm = sh.tmax;
    sync_block();
    if (!rotated || tm <= stop * stop) return sweep;
  }
  return -1;
}

// ------------------------------------------------------- complex GEMM
// C = A B for complex128 operands given by element accessors fa(i, k),
// fb(k, j) and a store fc(i, j, value), on FP64 matrix cores.  Each wave owns
// 32 x 32 output tiles (2 x 2 blocks of 16 x 16) and walks K in chunks of 8,
// issuing the chunk's operand loads before its MFMAs.  A complex product
// takes four real v_mfma_f64_16x16x4: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
// Operand layout of v_mfma_f64_16x16x4 (lane l): A[l % 16][l / 16],
// B[l / 16][l % 16]; the accumulator holds D[l / 16 + 4 r][l % 16], r < 4.
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename FA, typename FB, typename FC>
__device__ __forceinline__ void zgemm(int M, int N, int K, const FA& fa, const FB& fb,
                                      const FC& fc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (M + 31) >> 5, tn = (N + 31) >> 5;
#pragma unroll 1
  for (int t = wv; t < tm * tn; t += NW) {
    const int i0 = (t / tn) * 32, j0 = (t - (t / tn) * tn) * 32;
    d4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        ci[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      }
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 8) {
      z2 av[2][2], bv[2][2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int k = k0 + 4 * s + lk;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int i = i0 + 16 * q + li, j = j0 + 16 * q + li;
          av[s][q] = (i < M && k < K) ? fa(i, k) : cmk(0.0, 0.0);
          bv[s][q] = (j < N && k < K) ? fb(k, j) : cmk(0.0, 0.0);
        }
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a].x, bv[s][b].x, cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a].x, bv[s][b].y, ci[a][b], 0, 0, 0);
          }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            // - Ai Bi with the instruction's own negation of source A (the
            // NEG[0] bit in the BLGP field of an FP64 MFMA), so no VALU
            // writes a negated copy into registers an MFMA in flight reads
            cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a].y, bv[s][b].y, cr[a][b], 0, 0, 1);
            ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][a].y, bv[s][b].x, ci[a][b], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * a + lk + 4 * r, j = j0 + 16 * b + li;
          if (i < M && j < N) fc(i, j, cmk(cr[a][b][r], ci[a][b][r]));
        }
  }
}

// The same product on FP32 matrix cores (mixed path): operands rounded to
// complex64, FP32 accumulation (v_mfma_f32_16x16x4f32, lane layout as above
// for A and B; the accumulator holds D[4 (l / 16) + r][l % 16], r < 4).
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename FA, typename FB, typename FC>
__device__ __forceinline__ void zgemm32(int M, int N, int K, const FA& fa, const FB& fb,
                                        const FC& fc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (M + 31) >> 5, tn = (N + 31) >> 5;
#pragma unroll 1
  for (int t = wv; t < tm * tn; t += NW) {
    const int i0 = (t / tn) * 32, j0 = (t - (t / tn) * tn) * 32;
    f4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        ci[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 8) {
      f2 av[2][2], bv[2][2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int k = k0 + 4 * s + lk;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int i = i0 + 16 * q + li, j = j0 + 16 * q + li;
          av[s][q] = fromz<f2>((i < M && k < K) ? fa(i, k) : cmk(0.0, 0.0));
          bv[s][q] = fromz<f2>((j < N && k < K) ? fb(k, j) : cmk(0.0, 0.0));
        }
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s][a].x, bv[s][b].x, cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s][a].x, bv[s][b].y, ci[a][b], 0, 0, 0);
          }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[s][a].y, bv[s][b].y, cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s][a].y, bv[s][b].x, ci[a][b], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * a + 4 * lk + r, j = j0 + 16 * b + li;
          if (i < M && j < N) fc(i, j, cmk((double)cr[a][b][r], (double)ci[a][b][r]));
        }
  }
}

// Contraction on the path's matrix cores: FP64, or FP32 on the mixed path.
template <bool MIX, typename FA, typename FB, typename FC>
__device__ __forceinline__ void zgemm_p(int M, int N, int K, const FA& fa, const FB& fb,
                                        const FC& fc) {
  if constexpr (MIX) {
    zgemm32(M, N, K, fa, fb, fc);
  } else {
    zgemm(M, N, K, fa, fb, fc);
  }
}

// ------------------------------------------------- QR preconditioning
// Householder QR with column pivoting of Z (nr x nc, column-major, global):
// Z P = Q Rz.  On return the upper trapezoid of Z holds Rz and sh.piv[j] is
// the original index of the column at position j; Q is not formed and the
// part below the diagonal is scratch.  Step j takes as pivot the remaining
// column with the largest norm below row j (lowest index on ties).  The
// reflector for x = Z[j:, j], x_0 = |x_0| e^{i phi}: beta = -e^{i phi} |x|,
// u = x - beta e_0, H = I - kappa u u^H with kappa = 1 / (|x| (|x| + |x_0|));
// H is unitary and Hermitian and maps x to beta e_0.
//
// The trailing columns are updated lazily, in panels of up to 32 steps (the
// blocked pivoted QR of LAPACK's xLAQPS): with u_i and W_i(c) = kappa_i u_i^H
// (column c after reflectors < i) kept for the panel's steps, the current
// column c is Z0_c - sum_i u_i W_i(c), where Z0 is the matrix at the start
// of the panel.  Step k forms W_k(c) = kappa_k (u_k^H Z0_c - sum_{i<k}
// (u_k^H u_i) W_i(c)) in one read-only pass, writes the new row k of R and
// downdates the squared norms by its entries; the matrix itself is updated
// once per panel (one GEMM).  A panel ends early when a downdated norm has
// lost more than six digits, and every panel starts from exact norms, so
// no pivot is chosen on a norm that cancellation has spoiled.  u_i live in
// LDS (Ul), W_i(c) in global scratch (Wb, nb x nc).
template <int RPL>
__device__ __noinline__ void qrcp(z2* Z_, int nr, int nc, Shared& sh, z2* Ul_, z2* Wb_) {
  constexpr int E = 4 * RPL;
  gz2* Z = (gz2*)Z_;
  lz2* Ul = (lz2*)Ul_;
  gz2* Wb = (gz2*)Wb_;
  ld* vn = (ld*)sh.sig2;
  ld* vn0 = (ld*)sh.qr_vn0;
  const int l16 = threadIdx.x & 15, row = threadIdx.x >> 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = nr < nc ? nr : nc;
  const int pw = sh.qr_panel < 32 ? sh.qr_panel : 32;
  const int nbmax = (jl_size<RPL>() / nr) < pw ? (jl_size<RPL>() / nr) : pw;

  // exact squared norms of rows r0.. of columns r0.. (all rows read, in-bounds)
  auto exact_norms = [&](int r0) {
#pragma unroll 1
    for (int i = r0 + row; i < nc; i += NROWS) {
      const gz2* col = Z + (uint64_t)i * nr;
      double a = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = r0 + l16 + 16 * e;
        const z2 v = col[r < nr ? r : nr - 1];
        const double w = r < nr ? 1.0 : 0.0;
        a = fma(w * v.x, v.x, fma(w * v.y, v.y, a));
      }
      a = row16_sum(a);
      if (l16 == 0) {
        vn[i] = a;
        vn0[i] = a;
      }
    }
  };
  exact_norms(0);
  for (int i = threadIdx.x; i < nc; i += NT) sh.piv[i] = (uint16_t)i;
  if (threadIdx.x == 0) sh.qr_done = 0;
  sync_block();

#pragma unroll 1
  for (int j0 = 0; j0 < m;) {
    const int kmax = (m - j0) < nbmax ? (m - j0) : nbmax;
    if (threadIdx.x == 0) sh.qr_mark = 0;
    sync_block();
    int kb = 0;
#pragma unroll 1
    for (int k = 0; k < kmax; ++k) {
      const int j = j0 + k;
      if (wv == 0) {
        double best = -1.0;
        int bi = nc;
        for (int i = j + lane; i < nc; i += 64) {
          const double v = vn[i];
          if (v > best) {
            best = v;
            bi = i;
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (lane == 0) {
          sh.qr_p = bi;
          sh.qr_v = best;
          if (!(best > 0.0) && k == 0) sh.qr_done = 1;   // exact norms: the rest is zero
        }
      }
      sync_block();
      const int p = sh.qr_p;
      if (!(sh.qr_v > 0.0)) break;     // (downdated norms: re-check after the update)
      if (p != j) {
        gz2* a = Z + (uint64_t)j * nr;
        gz2* b = Z + (uint64_t)p * nr;
        for (int r = threadIdx.x; r < nr; r += NT) {
          const z2 t = a[r];
          a[r] = b[r];
          b[r] = t;
        }
        for (int i = threadIdx.x; i < k; i += NT) {
          const z2 t = Wb[(uint64_t)i * nc + j];
          Wb[(uint64_t)i * nc + j] = Wb[(uint64_t)i * nc + p];
          Wb[(uint64_t)i * nc + p] = t;
        }
        if (threadIdx.x == 0) {
          double t = vn[j];
          vn[j] = vn[p];
          vn[p] = t;
          t = vn0[j];
          vn0[j] = vn0[p];
          vn0[p] = t;
          const uint16_t q = sh.piv[j];
          sh.piv[j] = sh.piv[p];
          sh.piv[p] = q;
        }
      }
      if (threadIdx.x < k) sh.qr_w[threadIdx.x] = Wb[(uint64_t)threadIdx.x * nc + j];
      sync_block();
      // the pivot column brought up to date, and its reflector (wave 0)
      if (wv == 0) {
        const gz2* col = Z + (uint64_t)j * nr;
        z2 v[RPL];
        double x2 = 0.0;
        z2 alpha = cmk(0.0, 0.0);
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const int r = lane + 64 * e;
          z2 t = (r >= j && r < nr) ? (z2)col[r] : cmk(0.0, 0.0);
          if (r >= j && r < nr) {
            for (int i = 0; i < k; ++i) {
              const z2 ui = Ul[i * nr + r], wi = sh.qr_w[i];
              t = cmk(t.x - (ui.x * wi.x - ui.y * wi.y), t.y - (ui.x * wi.y + ui.y * wi.x));
            }
          }
          v[e] = t;
          x2 = fma(t.x, t.x, fma(t.y, t.y, x2));
          if (r == j) alpha = t;
        }
        x2 = wave_sum(x2);
        alpha.x = wave_sum(alpha.x);      // one lane holds it, the others hold 0
        alpha.y = wave_sum(alpha.y);
        const double aa = sqrt(alpha.x * alpha.x + alpha.y * alpha.y);
        const double xn = sqrt(x2);
        const z2 ph = aa > 0.0 ? cmk(alpha.x / aa, alpha.y / aa) : cmk(1.0, 0.0);
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const int r = lane + 64 * e;
          if (r < nr) Ul[k * nr + r] = r < j ? cmk(0.0, 0.0) : (r == j ? cmk(ph.x * (aa + xn), ph.y * (aa + xn)) : v[e]);
        }
        if (lane == 0) {
          Z[(uint64_t)j * nr + j] = cmk(-ph.x * xn, -ph.y * xn);
          sh.qr_k = xn > 0.0 ? 1.0 / (xn * (xn + aa)) : 0.0;
        }
      }
      sync_block();
      // t_i = u_k^H u_i for the panel's earlier reflectors
      if (row < k) {
        double tr = 0.0, ti = 0.0;
        for (int r = j + l16; r < nr; r += 16) {
          const z2 a = Ul[k * nr + r], b = Ul[row * nr + r];
          tr = fma(a.x, b.x, fma(a.y, b.y, tr));
          ti = fma(a.x, b.y, fma(-a.y, b.x, ti));
        }
        tr = row16_sum(tr);
        ti = row16_sum(ti);
        if (l16 == 0) sh.qr_t[row] = cmk(tr, ti);
      }
      sync_block();
      // trailing columns: W_k(c), the new row j of R, downdated norms (read-only pass)
      {
        const double kap = sh.qr_k;
        const int ea = (nr - j + 15) >> 4;
        z2 uv[E];
#pragma unroll
        for (int g = 0; g < E / 4; ++g) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = 4 * g + q, r = j + l16 + 16 * e;
            const z2 u = (4 * g < ea) ? (z2)Ul[k * nr + (r < nr ? r : nr - 1)] : cmk(0.0, 0.0);
            uv[e] = r < nr ? u : cmk(0.0, 0.0);
          }
        }
        // two columns per row at a time (independent loads and reductions in flight)
        const z2 t0 = l16 < k ? sh.qr_t[l16] : cmk(0.0, 0.0);
        const z2 t1 = l16 + 16 < k ? sh.qr_t[l16 + 16] : cmk(0.0, 0.0);
        const z2 u0 = l16 < k ? (z2)Ul[l16 * nr + j] : cmk(0.0, 0.0);
        const z2 u1 = l16 + 16 < k ? (z2)Ul[(l16 + 16) * nr + j] : cmk(0.0, 0.0);
        const z2 uk = Ul[k * nr + j];
#pragma unroll 1
        for (int cb = j + 1 + row; cb < nc; cb += 2 * NROWS) {
          int cc[2];
          cc[0] = cb;
          cc[1] = cb + NROWS;
          double gr[2], gi[2], tr[2], ti[2], ur[2], ui[2];
          z2 z0[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bool live = cc[h] < nc;
            const int c = live ? cc[h] : cb;            // a dead half reads column cb again
            const gz2* col = Z + (uint64_t)c * nr;
            // the panel's W_i(c), i < k, spread over the row's lanes (two per lane)
            z2 w0 = cmk(0.0, 0.0), w1 = cmk(0.0, 0.0);
            if (l16 < k) w0 = Wb[(uint64_t)l16 * nc + c];
            if (l16 + 16 < k) w1 = Wb[(uint64_t)(l16 + 16) * nc + c];
            double a = 0.0, b = 0.0;
            z0[h] = cmk(0.0, 0.0);
#pragma unroll
            for (int g = 0; g < E / 4; ++g) {
              if (4 * g < ea) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int e = 4 * g + q, r = j + l16 + 16 * e;
                  const z2 v0 = col[r < nr ? r : nr - 1];
                  const z2 v = r < nr ? v0 : cmk(0.0, 0.0);
                  if (e == 0) z0[h] = v;
                  a = fma(uv[e].x, v.x, fma(uv[e].y, v.y, a));
                  b = fma(uv[e].x, v.y, fma(-uv[e].y, v.x, b));
                }
              }
            }
            gr[h] = a;
            gi[h] = b;
            // sum_{i<k} t_i W_i(c) and sum_{i<k} u_i[j] W_i(c)
            tr[h] = t0.x * w0.x - t0.y * w0.y + t1.x * w1.x - t1.y * w1.y;
            ti[h] = t0.x * w0.y + t0.y * w0.x + t1.x * w1.y + t1.y * w1.x;
            ur[h] = u0.x * w0.x - u0.y * w0.y + u1.x * w1.x - u1.y * w1.y;
            ui[h] = u0.x * w0.y + u0.y * w0.x + u1.x * w1.y + u1.y * w1.x;
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            gr[h] = row16_sum(gr[h]);
            gi[h] = row16_sum(gi[h]);
            tr[h] = row16_sum(tr[h]);
            ti[h] = row16_sum(ti[h]);
            ur[h] = row16_sum(ur[h]);
            ui[h] = row16_sum(ui[h]);
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int c = cc[h];
            if (l16 == 0 && c < nc) {
              // W_k(c) = kappa (u_k^H Z0_c - sum_{i<k} t_i W_i(c)); z0 = Z0[j, c]
              const z2 w = cscale(cmk(gr[h] - tr[h], gi[h] - ti[h]), kap);
              const z2 nrow = cmk(z0[h].x - ur[h] - (uk.x * w.x - uk.y * w.y),
                                  z0[h].y - ui[h] - (uk.x * w.y + uk.y * w.x));
              Wb[(uint64_t)k * nc + c] = w;
              Z[(uint64_t)c * nr + j] = nrow;          // row j of R
              const double nv = vn[c] - (nrow.x * nrow.x + nrow.y * nrow.y);
              vn[c] = nv;
              if (!(nv > 1e-6 * vn0[c])) sh.qr_mark = 1;
            }
          }
        }
      }
      sync_block();
      ++kb;
      if (sh.qr_mark) break;
    }
    // apply the panel's kb reflectors to rows and columns from r0 = j0 + kb on
    const int r0 = j0 + kb;
    if (kb > 0 && r0 < nc && r0 < nr) {
      zgemm(nr - r0, nc - r0, kb, [&](int r, int i) { return (z2)Ul[i * nr + r0 + r]; },
            [&](int i, int c) { return (z2)Wb[(uint64_t)i * nc + r0 + c]; },
            [&](int r, int c, z2 v) {
              gz2* at = Z + (uint64_t)(r0 + c) * nr + r0 + r;
              const z2 o = *at;
              *at = cmk(o.x - v.x, o.y - v.y);
            });
      sync_block();
    }
    if (r0 < nc) exact_norms(r0 < nr ? r0 : nr);
    sync_block();
    j0 = r0;
    if (sh.qr_done) break;
  }
}

// Jacobi with the smallest row class that holds R rows (the element loops
// run over all E = 4 RPL elements of a lane, so a smaller class saves work).
template <int RPL>
__device__ int jacobi_fit(z2* X, int R, int C, Shared& sh, z2* Jl, double stop, double skip) {
  if constexpr (RPL > 1) {
    if (R <= 32 * RPL) return jacobi_fit<RPL / 2>(X, R, C, sh, Jl, stop, skip);
  }
  return jacobi<RPL>(X, R, C, sh, Jl, stop, skip);
}

// Left singular vectors of M (R x C, column-major in Y0): Z = M^H is
// factored as Z P = Q Rz (in W), one-sided Jacobi orthogonalises the m
// columns of X = Rz^H (R x m, m = min(R, C), in the buffer X), and since
// M = P X Q^H, the columns of X with their rows put back by P are the left
// singular vectors of M times the singular values; they are written to W
// (R x m, column-major).  The pivoted QR concentrates the norm in the leading
// columns, which cuts the number of Jacobi sweeps (Drmac and Veselic's QR
// preconditioning of one-sided Jacobi).  Returns the sweeps (-1 at the cap).
template <int RPL, bool MIX>
__device__ int svd_cols(z2* W, const z2* Y0, z2* X, int R, int C, Shared& sh, z2* Jl,
                         double stop, double skip) {
  // the QR works on complex128 on both paths: its passes are bound by
  // instruction issue, and complex64 storage costs more in conversions than
  // it saves in bytes
  using TZ = z2;
  TZ* Z = (TZ*)W;
  for (int idx = threadIdx.x; idx < R * C; idx += NT) {
    const int c = idx / R, r = idx - c * R;
    Z[(uint64_t)r * C + c] = fromz<TZ>(cconj(Y0[idx]));
  }
  sync_block();
  qrcp<RPL>(W, C, R, sh, Jl, X);      // X holds the QR's panel coefficients until it is built
  const int m = R < C ? R : C;
  for (int idx = threadIdx.x; idx < R * m; idx += NT) {
    const int jj = idx / R, r = idx - jj * R;
    X[idx] = jj <= r ? cconj(toz(Z[(uint64_t)r * C + jj])) : cmk(0.0, 0.0);
  }
  sync_block();
  const int sweeps = jacobi_fit<RPL>(X, R, m, sh, Jl, stop, skip);
  for (int idx = threadIdx.x; idx < R * m; idx += NT) {
    const int jj = idx / R, r = idx - jj * R;
    W[(uint64_t)jj * R + sh.piv[r]] = X[idx];
  }
  sync_block();
  return sweeps;
}

struct Factor {
  int k;          // kept singular values
  double scale;   // 1 / ||sigma_kept||
};

// SVD of M = Y0 (R x C): the columns of W become the left singular vectors
// times the singular values (svd_cols, with X as scratch); sort, choose
// k = min(cap, #{sigma > cutoff sigma_0}), record statistics.  sh.perm[j] is
// the column of W holding the j-th largest sigma.
template <int RPL, bool MIX>
__device__ Factor factorise(z2* W, const z2* Y0, z2* X, int R, int C_, int cap, double cutoff,
                            bool record, Shared& sh, z2* Jl, double stop, double skip) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sweeps = svd_cols<RPL, MIX>(W, Y0, X, R, C_, sh, Jl, stop, skip);
  const int C = R < C_ ? R : C_;     // columns of W from here on
  for (int j = wv; j < C; j += NW) {
    const z2* w = W + (uint64_t)j * R;
    double a = 0.0;
    for (int r = lane; r < R; r += 64) a = fma(w[r].x, w[r].x, fma(w[r].y, w[r].y, a));
    a = wave_sum(a);
    if (lane == 0) sh.sig2[j] = a;
  }
  sync_block();
  for (int j = threadIdx.x; j < C; j += NT) {
    const double v = norm_key(sh.sig2[j]);
    int rank = 0;
    for (int i = 0; i < C; ++i) {
      const double u = norm_key(sh.sig2[i]);
      rank += (u > v) || (u == v && i < j);
    }
    sh.perm[rank] = (uint16_t)j;
  }
  sync_block();
  const double s0 = sh.sig2[sh.perm[0]];
  const double thr = cutoff * cutoff * s0;
  int r = 0;
  double tot = 0.0;
  for (int j = 0; j < C; ++j) {
    const double v = sh.sig2[sh.perm[j]];
    tot += v;
    r += (v > thr && v > 0.0) ? 1 : 0;
  }
  if (r < 1) r = 1;
  const int k = r < cap ? r : cap;
  double kept = 0.0;
  for (int j = 0; j < k; ++j) kept += sh.sig2[sh.perm[j]];
  if (threadIdx.x == 0) {
    sh.sweeps += (sweeps < 0 ? kMaxSweeps : sweeps);
    if (sweeps < 0) {
      sh.nonconv += 1;
      sh.sflags |= TEPAI_SAMPLE_NONCONVERGED;
    }
    if (!isfinite(tot) || !(kept > 0.0)) sh.sflags |= TEPAI_SAMPLE_NONFINITE;
    if (record) {
      const double disc = tot > 0.0 ? (tot - kept) / tot : 0.0;
      sh.discarded += disc;
      if (disc > sh.max_disc) sh.max_disc = disc;
      if (k < r) {   // a cut made by the bond cap
        // near tie: an SVD with backward error eps = u sqrt(R C) (relative
        // to sigma_0) fixes the straddling pair to the angle
        // th = min(1, eps / gap), which moves a unit-norm observable by at
        // most 2 sqrt(2) th sigma_{k-1} / |sigma_kept|; doubled for two SVDs
        const double skm = sqrt(sh.sig2[sh.perm[k - 1]]);
        const double gap = (skm - sqrt(sh.sig2[sh.perm[k]])) / sqrt(s0);
        if (gap < sh.min_gap) sh.min_gap = gap;
        const double eps = 0x1p-53 * sqrt((double)R * (double)C_);
        const double th = gap <= eps ? 1.0 : eps / gap;
        if (4.0 * sqrt(2.0) * th * skm / sqrt(kept) > 1e-10) sh.ties += 1;
      }
    }
  }
  sync_block();
  Factor fr;
  fr.k = k;
  fr.scale = 1.0 / sqrt(kept);
  return fr;
}

// P[j][col] = sum_r conj(yhat_j[r]) Y0[col*R + r] for j < k, where yhat_j is
// column perm[j] of W normalised to unit length.
template <bool MIX>
__device__ void project(const z2* W, const z2* Y0, z2* P, int R, int C, int k,
                        Shared& sh) {
  const gz2* w = (const gz2*)W;
  const gz2* y = (const gz2*)Y0;
  gz2* out = (gz2*)P;
  zgemm_p<MIX>(k, C, R,
        [&](int j, int r) { return cconj((z2)w[(uint64_t)sh.perm[j] * R + r]); },
        [&](int r, int col) { return (z2)y[(uint64_t)col * R + r]; },
        [&](int j, int col, z2 v) { out[(uint64_t)j * C + col] = cscale(v, rsq_nr(sh.sig2[sh.perm[j]])); });
  sync_block();
}

// -------------------------------------------------------- MPS operations
template <bool MIX>
__device__ void apply_local(const Slot& S, int k, const z2 U[4], Shared& sh) {
  using TS = TSite<MIX>;
  TS* A = site<TS>(S, k);
  const int cl = sh.bond[k], cr = sh.bond[k + 1];
  for (int idx = threadIdx.x; idx < cl * cr; idx += NT) {
    const int a = idx / cr, b = idx - a * cr;
    TS* x0 = A + (uint64_t)(a * 2 + 0) * cr + b;
    TS* x1 = A + (uint64_t)(a * 2 + 1) * cr + b;
    const z2 v0 = toz(*x0), v1 = toz(*x1);
    z2 o0 = cmk(0.0, 0.0), o1 = cmk(0.0, 0.0);
    cfma(o0, U[0], v0);
    cfma(o0, U[1], v1);
    cfma(o1, U[2], v0);
    cfma(o1, U[3], v1);
    *x0 = fromz<TS>(o0);
    *x1 = fromz<TS>(o1);
  }
  sync_block();
}

// Move the centre from site c to c+1 (SVD of A_c as a (2 cl) x cr matrix).
// cap > 0 also keeps at most cap singular values and renormalises the kept
// ones (the truncation sweep of a shared start).
template <int RPL, bool MIX>
__device__ void shift_right(const Slot& S, int c, double cutoff, Shared& sh, int cap = 0) {
  using TS = TSite<MIX>;
  TS* A = site<TS>(S, c);
  TS* B = site<TS>(S, c + 1);
  const int cl = sh.bond[c], cr = sh.bond[c + 1], cr2 = sh.bond[c + 2];
  const int R = 2 * cl, C = cr;
  for (int idx = threadIdx.x; idx < R * C; idx += NT) {
    const int row = idx / C, col = idx - row * C;
    S.Y0[(uint64_t)col * R + row] = toz(A[idx]);
  }
  sync_block();
  const Factor f = factorise<RPL, MIX>(S.W, S.Y0, S.P, R, C, cap > 0 ? cap : C, cutoff, false, sh,
                                       S.Jl, S.stop, S.skip);
  const int k = f.k;
  const double sc = cap > 0 ? f.scale : 1.0;
  project<MIX>(S.W, S.Y0, S.P, R, C, k, sh);
  for (int idx = threadIdx.x; idx < R * k; idx += NT) {
    const int row = idx / k, j = idx - row * k;
    const int pj = sh.perm[j];
    A[idx] = fromz<TS>(cscale(S.W[(uint64_t)pj * R + row], 1.0 / sqrt(sh.sig2[pj])));
  }
  // B' = P . B  (k x cr) . (cr x 2 cr2) into W, then back
  sync_block();
  const int nb = 2 * cr2;
  {
    const gz2* pp = (const gz2*)S.P;
    const glob<TS>* bb = (const glob<TS>*)B;
    gz2* ww = (gz2*)S.W;
    zgemm_p<MIX>(k, nb, cr, [&](int j, int b) { return (z2)pp[(uint64_t)j * C + b]; },
          [&](int b, int col) { return toz((TS)bb[(uint64_t)b * nb + col]); },
          [&](int j, int col, z2 v) { ww[(uint64_t)j * nb + col] = v; });
  }
  sync_block();
  for (int idx = threadIdx.x; idx < k * nb; idx += NT) B[idx] = fromz<TS>(cscale(S.W[idx], sc));
  if (threadIdx.x == 0) {
    sh.bond[c + 1] = (uint16_t)k;
    sh.centre = c + 1;
    sh.shifts += 1;
  }
  sync_block();
}

// Move the centre from site c to c-1 (SVD of A_c as a cl x (2 cr) matrix).
template <int RPL, bool MIX>
__device__ void shift_left(const Slot& S, int c, double cutoff, Shared& sh) {
  using TS = TSite<MIX>;
  TS* A = site<TS>(S, c);
  TS* B = site<TS>(S, c - 1);
  const int cl = sh.bond[c], cr = sh.bond[c + 1], cl0 = sh.bond[c - 1];
  const int R = 2 * cr, C = cl;
  for (int idx = threadIdx.x; idx < R * C; idx += NT) {
    S.Y0[idx] = cconj(toz(A[idx]));      // Y = A^H, same memory order
  }
  sync_block();
  const Factor f = factorise<RPL, MIX>(S.W, S.Y0, S.P, R, C, C, cutoff, false, sh, S.Jl, S.stop, S.skip);
  const int k = f.k;
  project<MIX>(S.W, S.Y0, S.P, R, C, k, sh);
  for (int idx = threadIdx.x; idx < k * R; idx += NT) {
    const int j = idx / R, col = idx - j * R;
    const int pj = sh.perm[j];
    A[idx] = fromz<TS>(cconj(cscale(S.W[(uint64_t)pj * R + col], 1.0 / sqrt(sh.sig2[pj]))));
  }
  sync_block();
  // B' [x, s, j] = sum_a B[x, s, a] conj(P[j, a])
  const int nrow = 2 * cl0;
  {
    const gz2* pp = (const gz2*)S.P;
    const glob<TS>* bb = (const glob<TS>*)B;
    gz2* ww = (gz2*)S.W;
    zgemm_p<MIX>(nrow, k, cl, [&](int xs, int a) { return toz((TS)bb[(uint64_t)xs * cl + a]); },
          [&](int a, int j) { return cconj((z2)pp[(uint64_t)j * C + a]); },
          [&](int xs, int j, z2 v) { ww[(uint64_t)xs * k + j] = v; });
  }
  sync_block();
  for (int idx = threadIdx.x; idx < nrow * k; idx += NT) B[idx] = fromz<TS>(S.W[idx]);
  if (threadIdx.x == 0) {
    sh.bond[c] = (uint16_t)k;
    sh.centre = c - 1;
    sh.shifts += 1;
  }
  sync_block();
}

template <int RPL, bool MIX>
__device__ void move_centre_to(const Slot& S, int i, Shared& sh) {
  while (sh.centre < i) shift_right<RPL, MIX>(S, sh.centre, S.cutoff, sh);
  while (sh.centre > i + 1) shift_left<RPL, MIX>(S, sh.centre, S.cutoff, sh);
}

// Truncated two-site update of sites (i, i+1) with operator G (site order,
// index s_i * 2 + s_{i+1}).  right: centre ends on i+1, else on i.
template <int RPL, bool MIX>
__device__ void two_site(const Slot& S, int i, bool right, bool is_swap, Shared& sh) {
  move_centre_to<RPL, MIX>(S, i, sh);
  using TS = TSite<MIX>;
  const z2* G = sh.G;
  TS* A = site<TS>(S, i);
  TS* B = site<TS>(S, i + 1);
  const int cl = sh.bond[i], cm = sh.bond[i + 1], cr = sh.bond[i + 2];
  const int M = 2 * cl, N = 2 * cr;
  const int R = right ? M : N, C = right ? N : M;
  // theta[(a,s),(t,c)] = sum_b A[a,s,b] B[b,t,c] into W (row-major, M x N),
  // then theta'[(a,u),(v,c)] = sum_{s,t} G[uv][st] theta[(a,s),(t,c)] into Y0
  {
    const glob<TS>* aa = (const glob<TS>*)A;
    const glob<TS>* bb = (const glob<TS>*)B;
    gz2* ww = (gz2*)S.W;
    zgemm_p<MIX>(M, N, cm, [&](int i, int b) { return toz((TS)aa[(uint64_t)i * cm + b]); },
          [&](int b, int j) { return toz((TS)bb[(uint64_t)b * N + j]); },
          [&](int i, int j, z2 v) { ww[(uint64_t)i * N + j] = v; });
  }
  sync_block();
  for (int idx = threadIdx.x; idx < cl * cr; idx += NT) {
    const int a = idx / cr, c = idx - a * cr;
    z2 tv[4];
#pragma unroll
    for (int st = 0; st < 4; ++st)
      tv[st] = S.W[(uint64_t)(a * 2 + (st >> 1)) * N + (st & 1) * cr + c];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        z2 o = cmk(0, 0);
#pragma unroll
        for (int st = 0; st < 4; ++st) cfma(o, G[(u * 2 + v) * 4 + st], tv[st]);
        const int row = a * 2 + u, col = v * cr + c;
        uint64_t at;
        if (right) {
          at = (uint64_t)col * R + row;
        } else {
          at = (uint64_t)row * R + col;
          o = cconj(o);
        }
        S.Y0[at] = o;
      }
    }
  }
  sync_block();
  const Factor f = factorise<RPL, MIX>(S.W, S.Y0, S.P, R, C, (int)S.chi, S.cutoff, true, sh, S.Jl, S.stop, S.skip);
  const int k = f.k;
  project<MIX>(S.W, S.Y0, S.P, R, C, k, sh);
  if (right) {
    // A_i[(a,u), j] = yhat_j ; A_{i+1}[j, (v,c)] = P[j, col] / ||sigma||
    for (int idx = threadIdx.x; idx < R * k; idx += NT) {
      const int row = idx / k, j = idx - row * k;
      const int pj = sh.perm[j];
      A[idx] = fromz<TS>(cscale(S.W[(uint64_t)pj * R + row], 1.0 / sqrt(sh.sig2[pj])));
    }
    for (int idx = threadIdx.x; idx < k * C; idx += NT) B[idx] = fromz<TS>(cscale(S.P[idx], f.scale));
  } else {
    // A_{i+1}[j, (v,c)] = conj(yhat_j) ; A_i[(a,u), j] = conj(P[j, (a,u)]) / ||sigma||
    for (int idx = threadIdx.x; idx < k * R; idx += NT) {
      const int j = idx / R, col = idx - j * R;
      const int pj = sh.perm[j];
      B[idx] = fromz<TS>(cconj(cscale(S.W[(uint64_t)pj * R + col], 1.0 / sqrt(sh.sig2[pj]))));
    }
    for (int idx = threadIdx.x; idx < C * k; idx += NT) {
      const int row = idx / k, j = idx - row * k;
      A[idx] = fromz<TS>(cconj(cscale(S.P[(uint64_t)j * C + row], f.scale)));
    }
  }
  sync_block();
  if (threadIdx.x == 0) {
    sh.bond[i + 1] = (uint16_t)k;
    sh.centre = right ? i + 1 : i;
    sh.updates += 1;
    if (is_swap) sh.swap_updates += 1;
    sh.sum_chi3 += (double)cm * cm * cm;
    sh.flops += 8.0 * M * cm * N + svd_flops(M, N);
    if ((uint32_t)k > sh.max_bond) sh.max_bond = k;
  }
  sync_block();
}

template <int RPL, bool MIX>
__device__ void swap_sites(const Slot& S, int i, bool right, Shared& sh) {
  if (threadIdx.x < 16) {
    const int r = threadIdx.x >> 2, c = threadIdx.x & 3;
    // SWAP |s_i s_{i+1}> = |s_{i+1} s_i>
    const int sw = ((c & 1) << 1) | (c >> 1);
    sh.G[threadIdx.x] = cmk(r == sw ? 1.0 : 0.0, 0.0);
  }
  sync_block();
  two_site<RPL, MIX>(S, i, right, true, sh);
  if (threadIdx.x == 0) {
    const int a = sh.qubit_at[i], b = sh.qubit_at[i + 1];
    sh.qubit_at[i] = (uint16_t)b;
    sh.qubit_at[i + 1] = (uint16_t)a;
    sh.site_of[a] = (uint16_t)(i + 1);
    sh.site_of[b] = (uint16_t)i;
  }
  sync_block();
}

// Apply the pending same-pair run (if any) and clear it.
template <int RPL, bool MIX>
__device__ void flush(const Slot& S, Shared& sh) {
  if (!sh.p_active) return;
  const int qa = sh.p_qa, qb = sh.p_qb;
  if (!sh.p_has) {
    z2 Ua[4], Ub[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Ua[e] = cmul(sh.pPhase, sh.pLa[e]);
      Ub[e] = sh.pLb[e];
    }
    apply_local<MIX>(S, sh.site_of[qa], Ua, sh);
    apply_local<MIX>(S, sh.site_of[qb], Ub, sh);
  } else {
    // Non-adjacent pair (the two ends of a ring kept as a chain): carry the
    // end qubit nearer the centre across, the last step being SWAP . G on
    // the pair; the chain keeps its new order (a rotation of the ring).
    int ia = sh.site_of[qa], ib = sh.site_of[qb];
    const int lo = ia < ib ? ia : ib, hi = ia < ib ? ib : ia;
    int at = lo;
    const bool carry = hi - lo > 1;
    if (carry) {
      if (2 * sh.centre >= lo + hi) {
        for (int s = hi - 1; s > lo; --s) swap_sites<RPL, MIX>(S, s, false, sh);
        at = lo;
      } else {
        for (int s = lo; s < hi - 1; ++s) swap_sites<RPL, MIX>(S, s, true, sh);
        at = hi - 1;
      }
      ia = sh.site_of[qa];
      ib = sh.site_of[qb];
    }
    if (threadIdx.x < 16) {
      int r = threadIdx.x >> 2;
      const int c = threadIdx.x & 3;
      if (carry) r = ((r & 1) << 1) | (r >> 1);   // rows of SWAP . G
      // exchange tensor factors when qa sits on the right site
      const int rr = ia < ib ? r : ((r & 1) << 1 | (r >> 1));
      const int cc = ia < ib ? c : ((c & 1) << 1 | (c >> 1));
      sh.G[threadIdx.x] = sh.pM[rr * 4 + cc];
    }
    sync_block();
    two_site<RPL, MIX>(S, at, true, false, sh);
    if (carry && threadIdx.x == 0) {
      const int a = sh.qubit_at[at], b = sh.qubit_at[at + 1];
      sh.qubit_at[at] = (uint16_t)b;
      sh.qubit_at[at + 1] = (uint16_t)a;
      sh.site_of[a] = (uint16_t)(at + 1);
      sh.site_of[b] = (uint16_t)at;
    }
    sync_block();
  }
  if (threadIdx.x == 0) sh.p_active = 0;
  sync_block();
}

// Process one sampled non-identity gate (setting 1 = B, 2 = C) of row r.
template <int RPL, bool MIX>
__device__ void process_gate(const Slot& S, const DevRow& row, int setting, int layer_unused,
                             Shared& sh) {
  (void)layer_unused;
  if (row.nq == 1) {
    const int q = row.q0;
    if (sh.p_active && (q == sh.p_qa || q == sh.p_qb)) flush<RPL, MIX>(S, sh);
    z2 U[4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const z2 P = pauli_el(row.p0, r, c);
        // B: cb I - i sb P ;  C: -i P
        const double cb = setting == 1 ? row.cb : 0.0, sb = setting == 1 ? row.sb : 1.0;
        U[r * 2 + c] = cmk((r == c ? cb : 0.0) + sb * P.y, -sb * P.x);
      }
    }
    apply_local<MIX>(S, sh.site_of[q], U, sh);
    return;
  }
  const int qa = row.q0, qb = row.q1;
  if (sh.p_active && !((qa == sh.p_qa && qb == sh.p_qb) || (qa == sh.p_qb && qb == sh.p_qa)))
    flush<RPL, MIX>(S, sh);
  if (threadIdx.x == 0) {
    if (!sh.p_active) {
      sh.p_active = 1;
      sh.p_has = 0;
      sh.p_qa = qa;
      sh.p_qb = qb;
      for (int e = 0; e < 16; ++e) sh.pM[e] = cmk((e % 5 == 0) ? 1.0 : 0.0, 0.0);
      for (int e = 0; e < 4; ++e) {
        sh.pLa[e] = cmk((e % 3 == 0) ? 1.0 : 0.0, 0.0);
        sh.pLb[e] = sh.pLa[e];
      }
      sh.pPhase = cmk(1.0, 0.0);
    }
    // Paulis in the pending pair's order
    const bool same = (qa == sh.p_qa);
    const uint32_t pa = same ? row.p0 : row.p1, pb = same ? row.p1 : row.p0;
    const double cb = setting == 1 ? row.cb : 0.0, sb = setting == 1 ? row.sb : 1.0;
    z2 G[16];
    for (int r = 0; r < 4; ++r) {
      for (int c = 0; c < 4; ++c) {
        const z2 P = cmul(pauli_el(pa, r >> 1, c >> 1), pauli_el(pb, r & 1, c & 1));
        G[r * 4 + c] = cmk((r == c ? cb : 0.0) + sb * P.y, -sb * P.x);
      }
    }
    z2 Mn[16];
    for (int r = 0; r < 4; ++r) {
      for (int c = 0; c < 4; ++c) {
        z2 acc = cmk(0, 0);
        for (int m = 0; m < 4; ++m) cfma(acc, G[r * 4 + m], sh.pM[m * 4 + c]);
        Mn[r * 4 + c] = acc;
      }
    }
    for (int e = 0; e < 16; ++e) sh.pM[e] = Mn[e];
    if (setting == 1) {
      sh.p_has = 1;
    } else {
      z2 La[4], Lb[4];
      for (int r = 0; r < 2; ++r) {
        for (int c = 0; c < 2; ++c) {
          z2 a = cmk(0, 0), b = cmk(0, 0);
          for (int m = 0; m < 2; ++m) {
            cfma(a, pauli_el(pa, r, m), sh.pLa[m * 2 + c]);
            cfma(b, pauli_el(pb, r, m), sh.pLb[m * 2 + c]);
          }
          La[r * 2 + c] = a;
          Lb[r * 2 + c] = b;
        }
      }
      for (int e = 0; e < 4; ++e) {
        sh.pLa[e] = La[e];
        sh.pLb[e] = Lb[e];
      }
      sh.pPhase = cmul(sh.pPhase, cmk(0.0, -1.0));
    }
  }
  sync_block();
  if (S.per_gate) flush<RPL, MIX>(S, sh);   // the run holds this one gate
}

__device__ void load_state(const EngineArgs& a, int slot, Shared& sh) {
  const SampleState* st = a.states + slot;
  for (int k = threadIdx.x; k <= (int)a.n; k += NT) sh.bond[k] = st->bond[k];
  for (int k = threadIdx.x; k < (int)a.n; k += NT) {
    const uint16_t q = st->qubit_at[k];
    sh.qubit_at[k] = q;
    sh.site_of[q] = (uint16_t)k;
  }
  if (threadIdx.x == 0) {
    sh.centre = st->centre;
    sh.updates = st->updates;
    sh.swap_updates = st->swap_updates;
    sh.shifts = st->shifts;
    sh.sweeps = st->sweeps;
    sh.nonconv = st->nonconverged;
    sh.ties = st->ties;
    sh.n_gates = st->n_gates;
    sh.sum_chi3 = st->sum_chi3;
    sh.flops = st->nominal_flops;
    sh.discarded = st->discarded;
    sh.max_disc = st->max_discarded;
    sh.min_gap = st->min_gap;
    sh.max_bond = st->max_bond;
    sh.n_c = st->sign < 0 ? 1 : 0;
    sh.sflags = st->flags;
    sh.qr_panel = a.qr_panel >= 1 ? (int)a.qr_panel : 32;
    sh.p_active = 0;
  }
  sync_block();
}

__device__ void store_state(const EngineArgs& a, int slot, Shared& sh, uint32_t layer) {
  SampleState* st = a.states + slot;
  for (int k = threadIdx.x; k <= (int)a.n; k += NT) st->bond[k] = sh.bond[k];
  for (int k = threadIdx.x; k < (int)a.n; k += NT) st->qubit_at[k] = sh.qubit_at[k];
  if (threadIdx.x == 0) {
    st->centre = sh.centre;
    st->updates = sh.updates;
    st->swap_updates = sh.swap_updates;
    st->shifts = sh.shifts;
    st->sweeps = sh.sweeps;
    st->nonconverged = sh.nonconv;
    st->ties = sh.ties;
    st->n_gates = sh.n_gates;
    st->sum_chi3 = sh.sum_chi3;
    st->nominal_flops = sh.flops;
    st->discarded = sh.discarded;
    st->max_discarded = sh.max_disc;
    st->min_gap = sh.min_gap;
    st->max_bond = sh.max_bond;
    st->sign = (sh.n_c & 1) ? -1 : 1;
    st->flags = sh.sflags;
    st->layer = layer;
  }
}

template <bool MIX>
__device__ Slot make_slot(const EngineArgs& a, int slot, z2* Jl) {
  Slot S;
  S.Jl = Jl;
  S.ss = a.site_stride;
  S.T = reinterpret_cast<TSite<MIX>*>(a.tensors) + (uint64_t)slot * a.n * a.site_stride;
  const uint64_t q = a.work_stride / 3;
  S.Y0 = reinterpret_cast<z2*>(a.work) + (uint64_t)slot * a.work_stride;
  S.W = S.Y0 + q;
  S.P = S.W + q;
  S.cutoff = a.cutoff;
  S.stop = a.stop_cos;
  S.skip = a.skip_tol;
  S.chi = a.states[slot].chi_cap;
  S.n = a.n;
  S.per_gate = a.per_gate;
  return S;
}

// queue.hip compiles the engine above a second time, with TEPAI_ENGINE_ONLY
// defined, for the work-queue form of the evolve kernel; the kernels and
// launchers below belong to this translation unit only.
#ifndef TEPAI_ENGINE_ONLY

// ---------------------------------------------------------------- kernels
template <bool MIX>
__global__ __launch_bounds__(NT) void init_kernel(EngineArgs a) {
  using TS = TSite<MIX>;
  const int slot = blockIdx.x;
  SampleState* st = a.states + slot;
  TS* T = reinterpret_cast<TS*>(a.tensors) + (uint64_t)slot * a.n * a.site_stride;
  if (a.init_tensors) {
    // every slot starts from the shared MPS (copy-on-start)
    for (int k = 0; k < (int)a.n; ++k) {
      const uint64_t o = a.init_off[k], len = a.init_off[k + 1] - o;
      TS* dst = T + (uint64_t)k * a.site_stride;
      for (uint64_t i = threadIdx.x; i < len; i += NT) {
        const double2 v = a.init_tensors[o + i];
        dst[i] = fromz<TS>(cmk(v.x, v.y));
      }
    }
    for (int k = threadIdx.x; k <= (int)a.n; k += NT) st->bond[k] = (uint16_t)a.init_bond[k];
    for (int k = threadIdx.x; k < (int)a.n; k += NT) st->qubit_at[k] = a.init_qubit[k];
  } else {
    for (int k = threadIdx.x; k < (int)a.n; k += NT) {
      const int bit = a.init_bits[k] ? 1 : 0;
      T[(uint64_t)k * a.site_stride + 0] = fromz<TS>(cmk(bit ? 0.0 : 1.0, 0.0));
      T[(uint64_t)k * a.site_stride + 1] = fromz<TS>(cmk(bit ? 1.0 : 0.0, 0.0));
    }
    for (int k = threadIdx.x; k <= (int)a.n; k += NT) st->bond[k] = 1;
    for (int k = threadIdx.x; k < (int)a.n; k += NT) st->qubit_at[k] = (uint16_t)k;
  }
  if (threadIdx.x == 0) {
    st->centre = a.init_tensors ? a.init_centre : 0;
    st->chi_cap = a.chi_caps[slot];
    st->sign = 1;
    st->layer = 0;
    st->flags = 0;
    uint32_t mb = 1;
    if (a.init_tensors)
      for (uint32_t k = 0; k <= a.n; ++k) mb = a.init_bond[k] > mb ? a.init_bond[k] : mb;
    st->max_bond = mb;
    st->n_gates = st->updates = st->swap_updates = st->shifts = st->sweeps = 0;
    st->nonconverged = st->ties = 0;
    st->sum_chi3 = st->nominal_flops = st->discarded = st->max_discarded = 0.0;
    st->min_gap = INFINITY;
  }
}

// Truncation on copy: a slot whose cap is below the shared start's largest
// bond brings its copy to the cap before any step: the centre moves to the
// first site by exact shifts, then sweeps to the last site, each shift
// keeping at most cap singular values, renormalised (the state each step
// leaves is truncated optimally across the next cut).  Other slots return
// at once.
template <int RPL, bool MIX>
__global__ __launch_bounds__(NT) void start_kernel(EngineArgs a) {
  __shared__ Shared sh;
  __shared__ z2 Jl[jl_size<RPL>()];
  const int slot = (int)a.launch_order[blockIdx.x];
  if (a.chi_caps[slot] >= a.init_max_bond) return;    // the whole workgroup
  const Slot S = make_slot<MIX>(a, slot, Jl);
  load_state(a, slot, sh);
  while (sh.centre > 0) shift_left<RPL, MIX>(S, sh.centre, S.cutoff, sh);
  for (int c = 0; c + 1 < (int)a.n; ++c) shift_right<RPL, MIX>(S, c, S.cutoff, sh, (int)S.chi);
  if (threadIdx.x == 0) {     // the copy's largest bond, no longer the shared state's
    uint32_t mb = 1;
    for (int k = 0; k <= (int)a.n; ++k) mb = sh.bond[k] > mb ? sh.bond[k] : mb;
    sh.max_bond = mb;
  }
  sync_block();
  store_state(a, slot, sh, 0);
}

template <int RPL, bool MIX>
__global__ __launch_bounds__(NT) void evolve_kernel(EngineArgs a, uint32_t n_layers) {
  __shared__ Shared sh;
  __shared__ z2 Jl[jl_size<RPL>()];
  const int slot = (int)a.launch_order[blockIdx.x];
  const Slot S = make_slot<MIX>(a, slot, Jl);
  load_state(a, slot, sh);
  const uint32_t sample = (uint32_t)(a.first_sample + slot);
  const uint32_t L = a.l_eff;
  const uint32_t layer0 = a.states[slot].layer;
  for (uint32_t layer = layer0; layer < layer0 + n_layers; ++layer) {
    const uint64_t g0 = (uint64_t)layer * L;
    int nz = 0, nc = 0;
    for (uint32_t r = threadIdx.x; r < L; r += NT) {
      const uint8_t c = draw_setting(a.rows[r], a.seed, sample, g0 + r);
      sh.choice[r] = c;
      nz += c != 0;
      nc += c == 2;
    }
    const double tz = block_sum((double)nz, sh.red);
    const double tc = block_sum((double)nc, sh.red);
    if (threadIdx.x == 0) {
      sh.n_gates += (uint64_t)tz;
      sh.n_c += (int)tc;
    }
    sync_block();
    for (uint32_t r = 0; r < L; ++r) {
      const int c = sh.choice[r];
      if (c == 0) continue;
      process_gate<RPL, MIX>(S, a.rows[r], c, (int)layer, sh);
    }
    flush<RPL, MIX>(S, sh);     // runs end at Trotter-step boundaries
    sync_block();  // every thread is done reading this step's settings
  }
  store_state(a, slot, sh, layer0 + n_layers);
}

// ------------------------------------------------------------ observables
// One-site operator of a Pauli string at a site (identity if the string has
// no factor there).
struct Op2 {
  z2 m[4];
  bool id;
};

__device__ Op2 string_op(const DevString& str, int site, const Shared& sh) {
  Op2 o;
  o.id = true;
  o.m[0] = cmk(1, 0);
  o.m[1] = cmk(0, 0);
  o.m[2] = cmk(0, 0);
  o.m[3] = cmk(1, 0);
  for (uint32_t t = 0; t < str.n_ops; ++t) {
    if (sh.site_of[str.q[t]] != site) continue;
    z2 n[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        z2 v = cmk(0, 0);
        for (int m = 0; m < 2; ++m) cfma(v, pauli_el(str.p[t], r, m), o.m[m * 2 + c]);
        n[r * 2 + c] = v;
      }
    for (int e = 0; e < 4; ++e) o.m[e] = n[e];
    o.id = false;
  }
  return o;
}

// Left environment through site A (kl x 2 x kr) with operator O:
// E'[b'][b] = sum conj(A[a',s',b']) O[s'][s] E[a'][a] A[a,s,b]  (bra first).
// F (kl x 2kr) is scratch; all matrices row-major in global memory.
template <bool MIX>
__device__ void env_left(const TSite<MIX>* A_, int kl, int kr, const z2* E_, z2* F_, z2* Eo_,
                         const Op2& O) {
  using TS = TSite<MIX>;
  const glob<TS>* A = (const glob<TS>*)A_;
  const gz2* E = (const gz2*)E_;
  gz2* F = (gz2*)F_;
  gz2* Eo = (gz2*)Eo_;
  const int n2 = 2 * kr;
  zgemm_p<MIX>(kl, n2, kl, [&](int i, int k) { return (z2)E[(uint64_t)i * kl + k]; },
               [&](int k, int j) { return toz((TS)A[(uint64_t)k * n2 + j]); },
               [&](int i, int j, z2 v) { F[(uint64_t)i * n2 + j] = v; });
  sync_block();
  if (!O.id) {
    for (int idx = threadIdx.x; idx < kl * kr; idx += NT) {
      const int a = idx / kr, b = idx - a * kr;
      const z2 f0 = F[(uint64_t)a * n2 + b], f1 = F[(uint64_t)a * n2 + kr + b];
      z2 g0 = cmk(0, 0), g1 = cmk(0, 0);
      cfma(g0, O.m[0], f0);
      cfma(g0, O.m[1], f1);
      cfma(g1, O.m[2], f0);
      cfma(g1, O.m[3], f1);
      F[(uint64_t)a * n2 + b] = g0;
      F[(uint64_t)a * n2 + kr + b] = g1;
    }
    sync_block();
  }
  // rows r = (a', s') of A and F, kr columns each
  zgemm_p<MIX>(kr, kr, 2 * kl, [&](int bp, int r) { return cconj(toz((TS)A[(uint64_t)r * kr + bp])); },
               [&](int r, int b) { return (z2)F[(uint64_t)r * kr + b]; },
               [&](int bp, int b, z2 v) { Eo[(uint64_t)bp * kr + b] = v; });
  sync_block();
}

// Right environment through site A: R'[a][a'] = sum A[a,s,b] R[b][b'] conj(A[a',s,b'])
// (ket first).
template <bool MIX>
__device__ void env_right(const TSite<MIX>* A_, int kl, int kr, const z2* R_, z2* F_, z2* Ro_) {
  using TS = TSite<MIX>;
  const glob<TS>* A = (const glob<TS>*)A_;
  const gz2* R = (const gz2*)R_;
  gz2* F = (gz2*)F_;
  gz2* Ro = (gz2*)Ro_;
  zgemm_p<MIX>(2 * kl, kr, kr, [&](int r, int b) { return toz((TS)A[(uint64_t)r * kr + b]); },
               [&](int b, int bp) { return (z2)R[(uint64_t)b * kr + bp]; },
               [&](int r, int bp, z2 v) { F[(uint64_t)r * kr + bp] = v; });
  sync_block();
  const int n2 = 2 * kr;
  zgemm_p<MIX>(kl, kl, n2, [&](int a, int j) { return (z2)F[(uint64_t)a * n2 + j]; },
               [&](int j, int ap) { return cconj(toz((TS)A[(uint64_t)ap * n2 + j])); },
               [&](int a, int ap, z2 v) { Ro[(uint64_t)a * kl + ap] = v; });
  sync_block();
}

__device__ void set_identity(z2* M, int d) {
  for (int idx = threadIdx.x; idx < d * d; idx += NT) M[idx] = cmk((idx / d) == (idx % d) ? 1.0 : 0.0, 0.0);
  sync_block();
}

__device__ void copy_mat(z2* dst, const z2* src, int len) {
  for (int idx = threadIdx.x; idx < len; idx += NT) dst[idx] = src[idx];
  sync_block();
}

// Re sum_{b,b'} E[b'][b] R[b][b'] (R = null: the identity), all threads get it.
__device__ double env_trace(const z2* E, const z2* R, int d, Shared& sh) {
  double t = 0.0;
  for (int idx = threadIdx.x; idx < d * d; idx += NT) {
    const int bp = idx / d, b = idx - bp * d;
    if (R) {
      const z2 e = E[idx], r = R[(uint64_t)b * d + bp];
      t += e.x * r.x - e.y * r.y;
    } else if (b == bp) {
      t += E[idx].x;
    }
  }
  return block_sum(t, sh.red);
}

// Observables of every slot, contracted around the orthogonality centre c:
// the sites left of c are left-canonical and those right of it
// right-canonical, so the environment is the identity on the left bond of
// any site <= c and on the right bond of any site >= c.  A Pauli string on
// sites first..last is the transfer from an identity (or from the left
// environment of the sweep, when first > c) through its sites with its
// factors inserted, closed by the identity (last >= c) or by the right
// environment of the sweep (last < c); normalised by |A_c|^2.  Transfers are
// GEMMs on the path's matrix cores; the state is not changed.
template <int RPL, bool MIX>
__global__ __launch_bounds__(NT) void observe_kernel(EngineArgs a, double* values,
                                                     double* weights) {
  using TS = TSite<MIX>;
  __shared__ Shared sh;
  __shared__ double acc_obs[256];
  const int slot = blockIdx.x;
  const Slot S = make_slot<MIX>(a, slot, nullptr);
  load_state(a, slot, sh);
  for (int o = threadIdx.x; o < 256; o += NT) acc_obs[o] = 0.0;
  const int n = (int)a.n, c = sh.centre;
  double nn = 0.0;
  {
    const TS* Ac = site<TS>(S, c);
    const int len = sh.bond[c] * 2 * sh.bond[c + 1];
    for (int idx = threadIdx.x; idx < len; idx += NT) {
      const z2 v = toz(Ac[idx]);
      nn += v.x * v.x + v.y * v.y;
    }
  }
  const double norm2 = block_sum(nn, sh.red);
  const uint64_t chi2 = (uint64_t)a.chi_max * a.chi_max;
  z2* env = S.Y0;                  // environment of the sweep
  z2* F = S.W;                     // GEMM scratch (chi x 2 chi)
  z2* ea = S.P;                    // a string's environment, ping-pong
  z2* eb = S.P + chi2;
  z2* et = S.P + 2 * chi2;         // new sweep environment
  const Op2 ident = {{cmk(1, 0), cmk(0, 0), cmk(0, 0), cmk(1, 0)}, true};

  // value of string str from site f (environment `start` on the left bond of
  // f, identity when null) to its last site l, closed by `close` (null: identity)
  auto string_value = [&](const DevString& str, int f, int l, const z2* start, const z2* close) {
    z2* cur = ea;
    z2* nxt = eb;
    if (start)
      copy_mat(cur, start, sh.bond[f] * sh.bond[f]);
    else
      set_identity(cur, sh.bond[f]);
    for (int k = f; k <= l; ++k) {
      const Op2 o = string_op(str, k, sh);
      env_left<MIX>(site<TS>(S, k), sh.bond[k], sh.bond[k + 1], cur, F, nxt, o);
      z2* t = cur;
      cur = nxt;
      nxt = t;
    }
    return env_trace(cur, close, sh.bond[l + 1], sh);
  };
  auto span = [&](const DevString& str, int& f, int& l) {
    f = n;
    l = -1;
    for (uint32_t t = 0; t < str.n_ops; ++t) {
      const int q = sh.site_of[str.q[t]];
      f = q < f ? q : f;
      l = q > l ? q : l;
    }
  };
  auto add = [&](const DevString& str, double v) {
    if (threadIdx.x == 0) acc_obs[str.observable] += str.coeff * v / norm2;
    sync_block();
  };

  // strings that start at or right of the centre: left-to-right sweep
  set_identity(env, sh.bond[c]);
  for (int k = c; k < n; ++k) {
    for (uint32_t si = 0; si < a.n_strings; ++si) {
      const DevString str = a.strings[si];
      int f, l;
      span(str, f, l);
      if (f == k) add(str, string_value(str, f, l, env, nullptr));
    }
    if (k + 1 < n) {
      env_left<MIX>(site<TS>(S, k), sh.bond[k], sh.bond[k + 1], env, F, et, ident);
      copy_mat(env, et, sh.bond[k + 1] * sh.bond[k + 1]);
    }
  }
  // strings that start left of the centre and reach it: identity at both ends
  for (uint32_t si = 0; si < a.n_strings; ++si) {
    const DevString str = a.strings[si];
    int f, l;
    span(str, f, l);
    if (f < c && l >= c) add(str, string_value(str, f, l, nullptr, nullptr));
  }
  // strings that end left of the centre: right-to-left sweep of R
  set_identity(env, sh.bond[c + 1]);
  for (int k = c; k >= 1; --k) {
    env_right<MIX>(site<TS>(S, k), sh.bond[k], sh.bond[k + 1], env, F, et);
    copy_mat(env, et, sh.bond[k] * sh.bond[k]);          // R on the left bond of k
    for (uint32_t si = 0; si < a.n_strings; ++si) {
      const DevString str = a.strings[si];
      int f, l;
      span(str, f, l);
      if (l == k - 1) add(str, string_value(str, f, l, nullptr, env));
    }
  }
  sync_block();
  const SampleState* st = a.states + slot;
  for (uint32_t o = threadIdx.x; o < a.n_obs; o += NT)
    values[(uint64_t)slot * a.n_obs + o] = acc_obs[o];
  if (threadIdx.x == 0) weights[slot] = (double)st->sign * exp((double)st->layer * a.log_g1_step);
}

// Weighted reduction: one block per observable, fixed summation order.
__global__ __launch_bounds__(NT) void reduce_kernel(uint64_t count, uint32_t n_obs,
                                                    const double* v, const double* w,
                                                    double* mean, double* se) {
  __shared__ double red[NW * 4];
  const uint32_t o = blockIdx.x;
  double s = 0.0;
  for (uint64_t i = threadIdx.x; i < count; i += NT) s += w[i] * v[i * n_obs + o];
  const double m = block_sum(s, red) / (double)count;
  double q = 0.0;
  for (uint64_t i = threadIdx.x; i < count; i += NT) {
    const double d = w[i] * v[i * n_obs + o] - m;
    q = fma(d, d, q);
  }
  const double ss = block_sum(q, red);
  if (threadIdx.x == 0) {
    mean[o] = m;
    se[o] = count > 1 ? sqrt(ss / (double)(count - 1) / (double)count) : NAN;
  }
}

// Sampler: per-sample counts of non-identity gates and the sign.
__global__ __launch_bounds__(NT) void sample_count_kernel(const DevRow* rows, uint32_t L,
                                                          uint64_t seed, uint64_t first,
                                                          uint64_t n_draws, uint64_t* counts,
                                                          int8_t* signs) {
  __shared__ double red[NW * 4];
  const uint32_t sample = (uint32_t)(first + blockIdx.x);
  double nz = 0.0, nc = 0.0;
  for (uint64_t g = threadIdx.x; g < n_draws; g += NT) {
    const uint8_t c = draw_setting(rows[g % L], seed, sample, g);
    nz += c != 0;
    nc += c == 2;
  }
  const double tz = block_sum(nz, red);
  const double tc = block_sum(nc, red);
  if (threadIdx.x == 0) {
    counts[blockIdx.x] = (uint64_t)tz;
    signs[blockIdx.x] = (((uint64_t)tc) & 1) ? -1 : 1;
  }
}

// Sampler: ordered compaction of the non-identity gates into words.
__global__ __launch_bounds__(NT) void sample_write_kernel(const DevRow* rows, uint32_t L,
                                                          uint64_t seed, uint64_t first,
                                                          uint64_t n_draws,
                                                          const uint64_t* offsets,
                                                          uint32_t* words) {
  __shared__ int scan[NT];
  const uint32_t sample = (uint32_t)(first + blockIdx.x);
  uint64_t base = offsets[blockIdx.x];
  for (uint64_t g0 = 0; g0 < n_draws; g0 += NT) {
    const uint64_t g = g0 + threadIdx.x;
    uint8_t c = 0;
    if (g < n_draws) c = draw_setting(rows[g % L], seed, sample, g);
    scan[threadIdx.x] = c != 0;
    sync_block();
    // inclusive Hillis-Steele scan over the block
    for (int off = 1; off < NT; off <<= 1) {
      const int v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
      sync_block();
      scan[threadIdx.x] += v;
      sync_block();
    }
    if (c != 0) words[base + scan[threadIdx.x] - 1] = (uint32_t)(g * 4 + c);
    base += scan[NT - 1];
    sync_block();
  }
}

#endif  // TEPAI_ENGINE_ONLY
}  // namespace

#ifndef TEPAI_ENGINE_ONLY
hipError_t launch_init(const EngineArgs& a, hipStream_t s) {
  (void)hipGetLastError();   // an earlier call's error was reported by that call
  if (a.mixed)
    hipLaunchKernelGGL(init_kernel<true>, dim3(a.count), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL(init_kernel<false>, dim3(a.count), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <bool MIX>
static void evolve_rpl(const EngineArgs& a, uint32_t n_layers, hipStream_t s) {
  switch (rows_per_lane(a.chi_max)) {
    case 1: hipLaunchKernelGGL((evolve_kernel<1, MIX>), dim3(a.count), dim3(NT), 0, s, a, n_layers); break;
    case 2: hipLaunchKernelGGL((evolve_kernel<2, MIX>), dim3(a.count), dim3(NT), 0, s, a, n_layers); break;
    case 4: hipLaunchKernelGGL((evolve_kernel<4, MIX>), dim3(a.count), dim3(NT), 0, s, a, n_layers); break;
    default: hipLaunchKernelGGL((evolve_kernel<8, MIX>), dim3(a.count), dim3(NT), 0, s, a, n_layers); break;
  }
}

hipError_t launch_evolve(const EngineArgs& a, uint32_t n_layers, hipStream_t s) {
  (void)hipGetLastError();
  if (a.mixed)
    evolve_rpl<true>(a, n_layers, s);
  else
    evolve_rpl<false>(a, n_layers, s);
  return hipGetLastError();
}

template <bool MIX>
static void observe_rpl(const EngineArgs& a, double* v, double* w, hipStream_t s) {
  switch (rows_per_lane(a.chi_max)) {
    case 1: hipLaunchKernelGGL((observe_kernel<1, MIX>), dim3(a.count), dim3(NT), 0, s, a, v, w); break;
    case 2: hipLaunchKernelGGL((observe_kernel<2, MIX>), dim3(a.count), dim3(NT), 0, s, a, v, w); break;
    case 4: hipLaunchKernelGGL((observe_kernel<4, MIX>), dim3(a.count), dim3(NT), 0, s, a, v, w); break;
    default: hipLaunchKernelGGL((observe_kernel<8, MIX>), dim3(a.count), dim3(NT), 0, s, a, v, w); break;
  }
}

template <bool MIX>
static void start_rpl(const EngineArgs& a, hipStream_t s) {
  switch (rows_per_lane(a.chi_max)) {
    case 1: hipLaunchKernelGGL((start_kernel<1, MIX>), dim3(a.count), dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((start_kernel<2, MIX>), dim3(a.count), dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((start_kernel<4, MIX>), dim3(a.count), dim3(NT), 0, s, a); break;
    default: hipLaunchKernelGGL((start_kernel<8, MIX>), dim3(a.count), dim3(NT), 0, s, a); break;
  }
}

hipError_t launch_start(const EngineArgs& a, hipStream_t s) {
  (void)hipGetLastError();
  if (a.mixed)
    start_rpl<true>(a, s);
  else
    start_rpl<false>(a, s);
  return hipGetLastError();
}

hipError_t launch_observe(const EngineArgs& a, double* d_values, double* d_weights,
                          hipStream_t s) {
  (void)hipGetLastError();
  if (a.mixed)
    observe_rpl<true>(a, d_values, d_weights, s);
  else
    observe_rpl<false>(a, d_values, d_weights, s);
  return hipGetLastError();
}

hipError_t launch_reduce(uint64_t count, uint32_t n_obs, const double* v, const double* w,
                         double* mean, double* se, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(reduce_kernel, dim3(n_obs), dim3(NT), 0, s, count, n_obs, v, w, mean, se);
  return hipGetLastError();
}

hipError_t launch_sample_count(const DevRow* rows, uint32_t l_eff, uint64_t seed,
                               uint64_t first_sample, uint64_t count, uint64_t n_draws,
                               uint64_t* d_counts, int8_t* d_signs, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(sample_count_kernel, dim3((uint32_t)count), dim3(NT), 0, s, rows, l_eff,
                     seed, first_sample, n_draws, d_counts, d_signs);
  return hipGetLastError();
}

hipError_t launch_sample_write(const DevRow* rows, uint32_t l_eff, uint64_t seed,
                               uint64_t first_sample, uint64_t count, uint64_t n_draws,
                               const uint64_t* d_offsets, uint32_t* d_words, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(sample_write_kernel, dim3((uint32_t)count), dim3(NT), 0, s, rows, l_eff,
                     seed, first_sample, n_draws, d_offsets, d_words);
  return hipGetLastError();
}

#endif  // TEPAI_ENGINE_ONLY

}  // namespace tepai
