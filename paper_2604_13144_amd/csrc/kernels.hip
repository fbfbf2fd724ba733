// Device side of libtepai: TE-PAI sampling, the per-sample MPS engine,
// observables and the weighted reduction, written for gfx950 (wave64).
//
// One workgroup owns one sample for the whole launch.  It draws the sample's
// gate settings itself (Philox4x32-10, counter = (g_lo, g_hi, sample, 1),
// key = seed), so no gate stream is ever materialised, and applies them to
// the sample's MPS, which lives in HBM in the caller's workspace:
//   site k of slot b: tensors + (b * n + k) * site_stride, layout A[a][s][c]
//   (row-major, actual bond dimensions), complex128 as double2.
// Every factorisation is a one-sided (Hestenes) Jacobi SVD done by the four
// waves of the workgroup: columns are rotated pairwise in round-robin order,
// one column pair per wave, with the wave's 64 lanes striding over the rows
// and the pair held in registers between the dot products and the rotation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tepai_internal.h"

namespace tepai {
namespace {

constexpr int NT = kThreads;
constexpr int NW = kThreads / 64;
constexpr int kMaxRowsPerLane = (2 * kMaxChi + 63) / 64;   // rows of a column per lane

// ---------------------------------------------------------------- complex
__device__ __forceinline__ double2 cmk(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
// acc += a * b
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__device__ __forceinline__ void cfmac(double2& acc, double2 a, double2 b) {
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

// Fixed-order block sum (deterministic); all threads get the result.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NW; ++w) t += red[w];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------- Paulis
// Element (r, c) of Pauli p (1 = X, 2 = Y, 3 = Z).
__device__ __forceinline__ double2 pauli_el(uint32_t p, int r, int c) {
  if (p == 1) return cmk(r != c ? 1.0 : 0.0, 0.0);
  if (p == 2) return r == c ? cmk(0.0, 0.0) : cmk(0.0, r == 0 ? -1.0 : 1.0);
  if (p == 3) return cmk(r == c ? (r == 0 ? 1.0 : -1.0) : 0.0, 0.0);
  return cmk(r == c ? 1.0 : 0.0, 0.0);
}

// -------------------------------------------------------- shared memory
struct Shared {
  double2 pM[16];             // pending two-site operator, (qa, qb) order
  double2 pLa[4], pLb[4];     // its local factors while it holds only C settings
  double2 pPhase;
  double sig2[2 * kMaxChi];   // squared column norms after Jacobi
  double red[NW * 4];
  uint16_t perm[2 * kMaxChi]; // columns by descending norm
  uint16_t bond[kMaxQubits + 1];
  uint16_t qubit_at[kMaxQubits];
  uint16_t site_of[kMaxQubits];
  uint8_t choice[kMaxRows];
  int flag;
  int p_active, p_has, p_qa, p_qb;
  int centre;
  // statistics (thread 0 writes)
  uint64_t updates, swap_updates, shifts, sweeps, nonconv, ties, n_gates;
  double sum_chi3, flops, discarded, max_disc, min_gap;
  int n_c;
  uint32_t max_bond;
};

struct Slot {
  double2* T;      // site tensors of this sample
  double2* Y0;     // scratch: factorised matrix (kept)
  double2* W;      // scratch: Jacobi working copy
  double2* P;      // scratch: projections
  uint64_t ss;     // site stride
  double cutoff;
  uint32_t chi;
  uint32_t n;
};

__device__ __forceinline__ double2* site(const Slot& s, int k) { return s.T + (uint64_t)k * s.ss; }

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

// One-sided Jacobi on the columns of W (R x C, column-major): on return the
// columns are mutually orthogonal (W <- W V).  Returns the number of sweeps,
// or -1 when the sweep cap was reached.
__device__ int jacobi(double2* W, int R, int C, Shared& sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (C < 2) return 0;
  const int Cp = C + (C & 1);
  // scale for "numerically zero" columns: sigma_j^2 < 1e-32 ||W||_F^2
  double f = 0.0;
  for (int i = threadIdx.x; i < R * C; i += NT) {
    const double2 x = W[i];
    f += x.x * x.x + x.y * x.y;
  }
  const double fro2 = block_sum(f, sh.red);
  const double tiny = 1e-32 * fro2;
  const double tol = 1e-15 * sqrt((double)R);
  for (int sweep = 1; sweep <= kMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) sh.flag = 0;
    __syncthreads();
    for (int round = 0; round < Cp - 1; ++round) {
      for (int k = wv; k < Cp / 2; k += NW) {
        int p, q;
        rr_pair(round, k, Cp, p, q);
        if (q >= C) continue;
        double2* wp = W + (uint64_t)p * R;
        double2* wq = W + (uint64_t)q * R;
        double2 xs[kMaxRowsPerLane], ys[kMaxRowsPerLane];
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
        for (int t = 0; t < kMaxRowsPerLane; ++t) {
          const int r = lane + 64 * t;
          if (r < R) {
            const double2 x = wp[r], y = wq[r];
            xs[t] = x;
            ys[t] = y;
            al = fma(x.x, x.x, fma(x.y, x.y, al));
            be = fma(y.x, y.x, fma(y.y, y.y, be));
            gr = fma(x.x, y.x, fma(x.y, y.y, gr));
            gi = fma(x.x, y.y, fma(-x.y, y.x, gi));
          }
        }
        al = wave_sum(al);
        be = wave_sum(be);
        gr = wave_sum(gr);
        gi = wave_sum(gi);
        const double g = sqrt(gr * gr + gi * gi);
        if (al <= tiny || be <= tiny || !(g > tol * sqrt(al * be))) continue;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        const double er = gr / g, ei = gi / g;   // e^{i phi} = gamma / |gamma|
        // w_p <- c w_p - s e^{-i phi} w_q ;  w_q <- s e^{i phi} w_p + c w_q
#pragma unroll
        for (int t2 = 0; t2 < kMaxRowsPerLane; ++t2) {
          const int r = lane + 64 * t2;
          if (r < R) {
            const double2 x = xs[t2], y = ys[t2];
            const double2 ey = cmk(er * y.x + ei * y.y, er * y.y - ei * y.x);
            const double2 ex = cmk(er * x.x - ei * x.y, er * x.y + ei * x.x);
            wp[r] = cmk(c * x.x - s * ey.x, c * x.y - s * ey.y);
            wq[r] = cmk(s * ex.x + c * y.x, s * ex.y + c * y.y);
          }
        }
        if (lane == 0) sh.flag = 1;
      }
      __syncthreads();
    }
    const int rotated = sh.flag;
    __syncthreads();
    if (!rotated) return sweep;
  }
  return -1;
}

struct Factor {
  int k;          // kept singular values
  double scale;   // 1 / ||sigma_kept||
};

// Jacobi SVD of W (R x C), sort, choose k = min(cap, #{sigma > cutoff sigma_0}),
// record statistics.  sh.perm[j] is the column of the j-th largest sigma.
__device__ Factor factorise(double2* W, int R, int C, int cap, double cutoff, bool record,
                            Shared& sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sweeps = jacobi(W, R, C, sh);
  for (int j = wv; j < C; j += NW) {
    const double2* w = W + (uint64_t)j * R;
    double a = 0.0;
    for (int r = lane; r < R; r += 64) a = fma(w[r].x, w[r].x, fma(w[r].y, w[r].y, a));
    a = wave_sum(a);
    if (lane == 0) sh.sig2[j] = a;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < C; j += NT) {
    const double v = sh.sig2[j];
    int rank = 0;
    for (int i = 0; i < C; ++i) {
      const double u = sh.sig2[i];
      rank += (u > v) || (u == v && i < j);
    }
    sh.perm[rank] = (uint16_t)j;
  }
  __syncthreads();
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
    if (sweeps < 0) sh.nonconv += 1;
    if (record) {
      const double disc = tot > 0.0 ? (tot - kept) / tot : 0.0;
      sh.discarded += disc;
      if (disc > sh.max_disc) sh.max_disc = disc;
      if (k < r) {   // a cut made by the bond cap
        const double sk = sh.sig2[sh.perm[k]];
        const double gap = (sqrt(sh.sig2[sh.perm[k - 1]]) - sqrt(sk)) / sqrt(s0);
        if (gap < sh.min_gap) sh.min_gap = gap;
        if (gap <= 1e-10) sh.ties += 1;
      }
    }
  }
  __syncthreads();
  Factor fr;
  fr.k = k;
  fr.scale = 1.0 / sqrt(kept);
  return fr;
}

// P[j][col] = sum_r conj(yhat_j[r]) Y0[col*R + r] for j < k, where yhat_j is
// column perm[j] of W normalised to unit length.
__device__ void project(const double2* W, const double2* Y0, double2* P, int R, int C, int k,
                        Shared& sh) {
  for (int idx = threadIdx.x; idx < k * C; idx += NT) {
    const int j = idx / C, col = idx - j * C;
    const int pj = sh.perm[j];
    const double2* w = W + (uint64_t)pj * R;
    const double2* y = Y0 + (uint64_t)col * R;
    double2 acc = cmk(0.0, 0.0);
    for (int r = 0; r < R; ++r) cfmac(acc, w[r], y[r]);
    P[idx] = cscale(acc, 1.0 / sqrt(sh.sig2[pj]));
  }
  __syncthreads();
}

// -------------------------------------------------------- MPS operations
__device__ void apply_local(const Slot& S, int k, const double2 U[4], Shared& sh) {
  double2* A = site(S, k);
  const int cl = sh.bond[k], cr = sh.bond[k + 1];
  for (int idx = threadIdx.x; idx < cl * cr; idx += NT) {
    const int a = idx / cr, b = idx - a * cr;
    double2* x0 = A + (uint64_t)(a * 2 + 0) * cr + b;
    double2* x1 = A + (uint64_t)(a * 2 + 1) * cr + b;
    const double2 v0 = *x0, v1 = *x1;
    double2 o0 = cmk(0.0, 0.0), o1 = cmk(0.0, 0.0);
    cfma(o0, U[0], v0);
    cfma(o0, U[1], v1);
    cfma(o1, U[2], v0);
    cfma(o1, U[3], v1);
    *x0 = o0;
    *x1 = o1;
  }
  __syncthreads();
}

// Move the centre from site c to c+1 (SVD of A_c as a (2 cl) x cr matrix).
__device__ void shift_right(const Slot& S, int c, double cutoff, Shared& sh) {
  double2* A = site(S, c);
  double2* B = site(S, c + 1);
  const int cl = sh.bond[c], cr = sh.bond[c + 1], cr2 = sh.bond[c + 2];
  const int R = 2 * cl, C = cr;
  for (int idx = threadIdx.x; idx < R * C; idx += NT) {
    const int row = idx / C, col = idx - row * C;
    const double2 v = A[idx];
    S.Y0[(uint64_t)col * R + row] = v;
    S.W[(uint64_t)col * R + row] = v;
  }
  __syncthreads();
  const Factor f = factorise(S.W, R, C, C, cutoff, false, sh);
  const int k = f.k;
  project(S.W, S.Y0, S.P, R, C, k, sh);
  for (int idx = threadIdx.x; idx < R * k; idx += NT) {
    const int row = idx / k, j = idx - row * k;
    const int pj = sh.perm[j];
    A[idx] = cscale(S.W[(uint64_t)pj * R + row], 1.0 / sqrt(sh.sig2[pj]));
  }
  // B' = P . B  (k x cr) . (cr x 2 cr2) into W, then back
  __syncthreads();
  const int nb = 2 * cr2;
  for (int idx = threadIdx.x; idx < k * nb; idx += NT) {
    const int j = idx / nb, col = idx - j * nb;
    double2 acc = cmk(0.0, 0.0);
    for (int b = 0; b < cr; ++b) cfma(acc, S.P[j * C + b], B[(uint64_t)b * nb + col]);
    S.W[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * nb; idx += NT) B[idx] = S.W[idx];
  if (threadIdx.x == 0) {
    sh.bond[c + 1] = (uint16_t)k;
    sh.centre = c + 1;
    sh.shifts += 1;
  }
  __syncthreads();
}

// Move the centre from site c to c-1 (SVD of A_c as a cl x (2 cr) matrix).
__device__ void shift_left(const Slot& S, int c, double cutoff, Shared& sh) {
  double2* A = site(S, c);
  double2* B = site(S, c - 1);
  const int cl = sh.bond[c], cr = sh.bond[c + 1], cl0 = sh.bond[c - 1];
  const int R = 2 * cr, C = cl;
  for (int idx = threadIdx.x; idx < R * C; idx += NT) {
    const double2 v = cconj(A[idx]);      // Y = A^H, same memory order
    S.Y0[idx] = v;
    S.W[idx] = v;
  }
  __syncthreads();
  const Factor f = factorise(S.W, R, C, C, cutoff, false, sh);
  const int k = f.k;
  project(S.W, S.Y0, S.P, R, C, k, sh);
  for (int idx = threadIdx.x; idx < k * R; idx += NT) {
    const int j = idx / R, col = idx - j * R;
    const int pj = sh.perm[j];
    A[idx] = cconj(cscale(S.W[(uint64_t)pj * R + col], 1.0 / sqrt(sh.sig2[pj])));
  }
  __syncthreads();
  // B' [x, s, j] = sum_a B[x, s, a] conj(P[j, a])
  const int nrow = 2 * cl0;
  for (int idx = threadIdx.x; idx < nrow * k; idx += NT) {
    const int xs = idx / k, j = idx - xs * k;
    double2 acc = cmk(0.0, 0.0);
    for (int a = 0; a < cl; ++a) cfma(acc, B[(uint64_t)xs * cl + a], cconj(S.P[j * C + a]));
    S.W[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nrow * k; idx += NT) B[idx] = S.W[idx];
  if (threadIdx.x == 0) {
    sh.bond[c] = (uint16_t)k;
    sh.centre = c - 1;
    sh.shifts += 1;
  }
  __syncthreads();
}

__device__ void move_centre_to(const Slot& S, int i, Shared& sh) {
  while (sh.centre < i) shift_right(S, sh.centre, S.cutoff, sh);
  while (sh.centre > i + 1) shift_left(S, sh.centre, S.cutoff, sh);
}

// Truncated two-site update of sites (i, i+1) with operator G (site order,
// index s_i * 2 + s_{i+1}).  right: centre ends on i+1, else on i.
__device__ void two_site(const Slot& S, int i, const double2* G, bool right, bool is_swap,
                         Shared& sh) {
  move_centre_to(S, i, sh);
  double2* A = site(S, i);
  double2* B = site(S, i + 1);
  const int cl = sh.bond[i], cm = sh.bond[i + 1], cr = sh.bond[i + 2];
  const int M = 2 * cl, N = 2 * cr;
  const int R = right ? M : N, C = right ? N : M;
  // theta'[(a,u),(v,c)] = sum_{s,t} G[uv][st] sum_b A[a,s,b] B[b,t,c]
  double2 g[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) g[e] = G[e];
  for (int idx = threadIdx.x; idx < cl * cr; idx += NT) {
    const int a = idx / cr, c = idx - a * cr;
    double2 t00 = cmk(0, 0), t01 = cmk(0, 0), t10 = cmk(0, 0), t11 = cmk(0, 0);
    const double2* a0 = A + (uint64_t)(a * 2 + 0) * cm;
    const double2* a1 = A + (uint64_t)(a * 2 + 1) * cm;
    for (int b = 0; b < cm; ++b) {
      const double2 x0 = a0[b], x1 = a1[b];
      const double2 y0 = B[(uint64_t)(b * 2 + 0) * cr + c], y1 = B[(uint64_t)(b * 2 + 1) * cr + c];
      cfma(t00, x0, y0);
      cfma(t01, x0, y1);
      cfma(t10, x1, y0);
      cfma(t11, x1, y1);
    }
    const double2 tv[4] = {t00, t01, t10, t11};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        double2 o = cmk(0, 0);
#pragma unroll
        for (int st = 0; st < 4; ++st) cfma(o, g[(u * 2 + v) * 4 + st], tv[st]);
        const int row = a * 2 + u, col = v * cr + c;
        uint64_t at;
        if (right) {
          at = (uint64_t)col * R + row;
        } else {
          at = (uint64_t)row * R + col;
          o = cconj(o);
        }
        S.Y0[at] = o;
        S.W[at] = o;
      }
    }
  }
  __syncthreads();
  const Factor f = factorise(S.W, R, C, (int)S.chi, S.cutoff, true, sh);
  const int k = f.k;
  project(S.W, S.Y0, S.P, R, C, k, sh);
  if (right) {
    // A_i[(a,u), j] = yhat_j ; A_{i+1}[j, (v,c)] = P[j, col] / ||sigma||
    for (int idx = threadIdx.x; idx < R * k; idx += NT) {
      const int row = idx / k, j = idx - row * k;
      const int pj = sh.perm[j];
      A[idx] = cscale(S.W[(uint64_t)pj * R + row], 1.0 / sqrt(sh.sig2[pj]));
    }
    for (int idx = threadIdx.x; idx < k * C; idx += NT) B[idx] = cscale(S.P[idx], f.scale);
  } else {
    // A_{i+1}[j, (v,c)] = conj(yhat_j) ; A_i[(a,u), j] = conj(P[j, (a,u)]) / ||sigma||
    for (int idx = threadIdx.x; idx < k * R; idx += NT) {
      const int j = idx / R, col = idx - j * R;
      const int pj = sh.perm[j];
      B[idx] = cconj(cscale(S.W[(uint64_t)pj * R + col], 1.0 / sqrt(sh.sig2[pj])));
    }
    for (int idx = threadIdx.x; idx < C * k; idx += NT) {
      const int row = idx / k, j = idx - row * k;
      A[idx] = cconj(cscale(S.P[(uint64_t)j * C + row], f.scale));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sh.bond[i + 1] = (uint16_t)k;
    sh.centre = right ? i + 1 : i;
    sh.updates += 1;
    if (is_swap) sh.swap_updates += 1;
    sh.sum_chi3 += (double)cm * cm * cm;
    sh.flops += 8.0 * M * cm * N + svd_flops(M, N);
    if ((uint32_t)k > sh.max_bond) sh.max_bond = k;
  }
  __syncthreads();
}

__device__ void swap_sites(const Slot& S, int i, bool right, Shared& sh) {
  double2 G[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) G[e] = cmk(0, 0);
  G[0 * 4 + 0] = cmk(1, 0);
  G[1 * 4 + 2] = cmk(1, 0);
  G[2 * 4 + 1] = cmk(1, 0);
  G[3 * 4 + 3] = cmk(1, 0);
  two_site(S, i, G, right, true, sh);
  if (threadIdx.x == 0) {
    const int a = sh.qubit_at[i], b = sh.qubit_at[i + 1];
    sh.qubit_at[i] = (uint16_t)b;
    sh.qubit_at[i + 1] = (uint16_t)a;
    sh.site_of[a] = (uint16_t)(i + 1);
    sh.site_of[b] = (uint16_t)i;
  }
  __syncthreads();
}

// Apply the pending same-pair run (if any) and clear it.
__device__ void flush(const Slot& S, Shared& sh) {
  if (!sh.p_active) return;
  const int qa = sh.p_qa, qb = sh.p_qb;
  if (!sh.p_has) {
    double2 Ua[4], Ub[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Ua[e] = cmul(sh.pPhase, sh.pLa[e]);
      Ub[e] = sh.pLb[e];
    }
    apply_local(S, sh.site_of[qa], Ua, sh);
    apply_local(S, sh.site_of[qb], Ub, sh);
  } else {
    int ia = sh.site_of[qa], ib = sh.site_of[qb];
    const int lo = ia < ib ? ia : ib, hi = ia < ib ? ib : ia;
    for (int s = hi - 1; s > lo; --s) swap_sites(S, s, false, sh);
    ia = sh.site_of[qa];
    ib = sh.site_of[qb];
    double2 G[16];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        // exchange tensor factors when qa sits on the right site
        const int rr = ia < ib ? r : ((r & 1) << 1 | (r >> 1));
        const int cc = ia < ib ? c : ((c & 1) << 1 | (c >> 1));
        G[r * 4 + c] = sh.pM[rr * 4 + cc];
      }
    }
    two_site(S, lo, G, true, false, sh);
    for (int s = lo + 1; s < hi; ++s) swap_sites(S, s, true, sh);
  }
  if (threadIdx.x == 0) sh.p_active = 0;
  __syncthreads();
}

// Process one sampled non-identity gate (setting 1 = B, 2 = C) of row r.
__device__ void process_gate(const Slot& S, const DevRow& row, int setting, int layer_unused,
                             Shared& sh) {
  (void)layer_unused;
  if (row.nq == 1) {
    const int q = row.q0;
    if (sh.p_active && (q == sh.p_qa || q == sh.p_qb)) flush(S, sh);
    double2 U[4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double2 P = pauli_el(row.p0, r, c);
        // B: cb I - i sb P ;  C: -i P
        const double cb = setting == 1 ? row.cb : 0.0, sb = setting == 1 ? row.sb : 1.0;
        U[r * 2 + c] = cmk((r == c ? cb : 0.0) + sb * P.y, -sb * P.x);
      }
    }
    apply_local(S, sh.site_of[q], U, sh);
    return;
  }
  const int qa = row.q0, qb = row.q1;
  if (sh.p_active && !((qa == sh.p_qa && qb == sh.p_qb) || (qa == sh.p_qb && qb == sh.p_qa)))
    flush(S, sh);
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
    double2 G[16];
    for (int r = 0; r < 4; ++r) {
      for (int c = 0; c < 4; ++c) {
        const double2 P = cmul(pauli_el(pa, r >> 1, c >> 1), pauli_el(pb, r & 1, c & 1));
        G[r * 4 + c] = cmk((r == c ? cb : 0.0) + sb * P.y, -sb * P.x);
      }
    }
    double2 Mn[16];
    for (int r = 0; r < 4; ++r) {
      for (int c = 0; c < 4; ++c) {
        double2 acc = cmk(0, 0);
        for (int m = 0; m < 4; ++m) cfma(acc, G[r * 4 + m], sh.pM[m * 4 + c]);
        Mn[r * 4 + c] = acc;
      }
    }
    for (int e = 0; e < 16; ++e) sh.pM[e] = Mn[e];
    if (setting == 1) {
      sh.p_has = 1;
    } else {
      double2 La[4], Lb[4];
      for (int r = 0; r < 2; ++r) {
        for (int c = 0; c < 2; ++c) {
          double2 a = cmk(0, 0), b = cmk(0, 0);
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
  __syncthreads();
}

__device__ void load_state(const EngineArgs& a, int slot, Shared& sh) {
  const SampleState* st = a.states + slot;
  for (int k = threadIdx.x; k <= (int)a.n; k += NT) sh.bond[k] = st->bond[k];
  for (int k = threadIdx.x; k < (int)a.n; k += NT) {
    sh.qubit_at[k] = (uint16_t)k;
    sh.site_of[k] = (uint16_t)k;
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
    sh.p_active = 0;
  }
  __syncthreads();
}

__device__ void store_state(const EngineArgs& a, int slot, Shared& sh, uint32_t layer) {
  SampleState* st = a.states + slot;
  for (int k = threadIdx.x; k <= (int)a.n; k += NT) st->bond[k] = sh.bond[k];
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
    st->layer = layer;
  }
}

__device__ Slot make_slot(const EngineArgs& a, int slot) {
  Slot S;
  S.ss = a.site_stride;
  S.T = a.tensors + (uint64_t)slot * a.n * a.site_stride;
  const uint64_t q = a.work_stride / 3;
  S.Y0 = a.work + (uint64_t)slot * a.work_stride;
  S.W = S.Y0 + q;
  S.P = S.W + q;
  S.cutoff = a.cutoff;
  S.chi = a.states[slot].chi_cap;
  S.n = a.n;
  return S;
}

// ---------------------------------------------------------------- kernels
__global__ __launch_bounds__(NT) void init_kernel(EngineArgs a) {
  const int slot = blockIdx.x;
  SampleState* st = a.states + slot;
  double2* T = a.tensors + (uint64_t)slot * a.n * a.site_stride;
  for (int k = threadIdx.x; k < (int)a.n; k += NT) {
    const int bit = a.init_bits[k] ? 1 : 0;
    T[(uint64_t)k * a.site_stride + 0] = cmk(bit ? 0.0 : 1.0, 0.0);
    T[(uint64_t)k * a.site_stride + 1] = cmk(bit ? 1.0 : 0.0, 0.0);
  }
  for (int k = threadIdx.x; k <= (int)a.n; k += NT) st->bond[k] = 1;
  if (threadIdx.x == 0) {
    st->centre = 0;
    st->chi_cap = a.chi_caps[slot];
    st->sign = 1;
    st->layer = 0;
    st->flags = 0;
    st->max_bond = 1;
    st->n_gates = st->updates = st->swap_updates = st->shifts = st->sweeps = 0;
    st->nonconverged = st->ties = 0;
    st->sum_chi3 = st->nominal_flops = st->discarded = st->max_discarded = 0.0;
    st->min_gap = INFINITY;
  }
}

__global__ __launch_bounds__(NT) void evolve_kernel(EngineArgs a, uint32_t n_layers) {
  __shared__ Shared sh;
  const int slot = blockIdx.x;
  const Slot S = make_slot(a, slot);
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
    __syncthreads();
    for (uint32_t r = 0; r < L; ++r) {
      const int c = sh.choice[r];
      if (c == 0) continue;
      process_gate(S, a.rows[r], c, (int)layer, sh);
    }
    flush(S, sh);     // runs end at Trotter-step boundaries
    __syncthreads();  // every thread is done reading this step's settings
  }
  store_state(a, slot, sh, layer0 + n_layers);
}

// Observables of every slot: sweep the centre from site 0 to n-1; at site c
// evaluate every Pauli string whose first site is c by a transfer-matrix
// contraction from c (left part left-canonical) to its last site (right part
// right-canonical), normalised by the centre's squared norm.
__global__ __launch_bounds__(NT) void observe_kernel(EngineArgs a, double* values,
                                                     double* weights) {
  __shared__ Shared sh;
  __shared__ double acc_obs[256];
  const int slot = blockIdx.x;
  const Slot S = make_slot(a, slot);
  load_state(a, slot, sh);
  const double obs_cut = 1e-30;    // gauge-only shifts
  for (int o = threadIdx.x; o < 256; o += NT) acc_obs[o] = 0.0;
  while (sh.centre > 0) shift_left(S, sh.centre, obs_cut, sh);
  double2* E = S.Y0;
  double2* F = S.W;
  for (int c = 0; c < (int)a.n; ++c) {
    const double2* Ac = site(S, c);
    const int cl = sh.bond[c], cr = sh.bond[c + 1];
    double nn = 0.0;
    for (int idx = threadIdx.x; idx < cl * 2 * cr; idx += NT)
      nn += Ac[idx].x * Ac[idx].x + Ac[idx].y * Ac[idx].y;
    const double norm2 = block_sum(nn, sh.red);
    for (uint32_t si = 0; si < a.n_strings; ++si) {
      const DevString str = a.strings[si];
      int first = (int)a.n, last = -1;
      for (uint32_t t = 0; t < str.n_ops; ++t) {
        const int q = sh.site_of[str.q[t]];
        first = q < first ? q : first;
        last = q > last ? q : last;
      }
      if (first != c) continue;
      // E = identity on the left bond of site c
      int dl = cl;
      for (int idx = threadIdx.x; idx < dl * dl; idx += NT)
        E[idx] = cmk((idx / dl) == (idx % dl) ? 1.0 : 0.0, 0.0);
      __syncthreads();
      for (int k = c; k <= last; ++k) {
        const double2* A = site(S, k);
        const int kl = sh.bond[k], kr = sh.bond[k + 1];
        // operator on this site (product of the string's factors here)
        double2 O[4] = {cmk(1, 0), cmk(0, 0), cmk(0, 0), cmk(1, 0)};
        for (uint32_t t = 0; t < str.n_ops; ++t) {
          if (sh.site_of[str.q[t]] != k) continue;
          double2 On[4];
          for (int r = 0; r < 2; ++r)
            for (int cc = 0; cc < 2; ++cc) {
              double2 v = cmk(0, 0);
              for (int m = 0; m < 2; ++m) cfma(v, pauli_el(str.p[t], r, m), O[m * 2 + cc]);
              On[r * 2 + cc] = v;
            }
          for (int e = 0; e < 4; ++e) O[e] = On[e];
        }
        // F[a', s, b] = sum_a E[a', a] A[a, s, b]
        for (int idx = threadIdx.x; idx < kl * 2 * kr; idx += NT) {
          const int ap = idx / (2 * kr), sb = idx - ap * 2 * kr;
          double2 v = cmk(0, 0);
          for (int aa = 0; aa < kl; ++aa) cfma(v, E[ap * kl + aa], A[(uint64_t)aa * 2 * kr + sb]);
          F[idx] = v;
        }
        __syncthreads();
        // E'[b', b] = sum_{a', s', s} conj(A[a', s', b']) O[s', s] F[a', s, b]
        for (int idx = threadIdx.x; idx < kr * kr; idx += NT) {
          const int bp = idx / kr, b = idx - bp * kr;
          double2 v = cmk(0, 0);
          for (int ap = 0; ap < kl; ++ap) {
            const double2 f0 = F[(uint64_t)ap * 2 * kr + 0 * kr + b];
            const double2 f1 = F[(uint64_t)ap * 2 * kr + 1 * kr + b];
            double2 of0 = cmk(0, 0), of1 = cmk(0, 0);
            cfma(of0, O[0], f0);
            cfma(of0, O[1], f1);
            cfma(of1, O[2], f0);
            cfma(of1, O[3], f1);
            cfmac(v, A[(uint64_t)ap * 2 * kr + 0 * kr + bp], of0);
            cfmac(v, A[(uint64_t)ap * 2 * kr + 1 * kr + bp], of1);
          }
          F[kl * 2 * kr + idx] = v;     // stage after F's live part
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < kr * kr; idx += NT) E[idx] = F[kl * 2 * kr + idx];
        __syncthreads();
        dl = kr;
      }
      double tr = 0.0;
      for (int b = threadIdx.x; b < dl; b += NT) tr += E[b * dl + b].x;
      tr = block_sum(tr, sh.red);
      if (threadIdx.x == 0) acc_obs[str.observable] += str.coeff * tr / norm2;
      __syncthreads();
    }
    if (c + 1 < (int)a.n) shift_right(S, c, obs_cut, sh);
  }
  __syncthreads();
  const SampleState* st = a.states + slot;
  for (uint32_t o = threadIdx.x; o < a.n_obs; o += NT)
    values[(uint64_t)slot * a.n_obs + o] = acc_obs[o];
  if (threadIdx.x == 0) {
    weights[slot] = (double)st->sign * exp((double)st->layer * a.log_g1_step);
    a.states[slot].centre = sh.centre;
    a.states[slot].shifts = sh.shifts;
  }
  for (int k = threadIdx.x; k <= (int)a.n; k += NT) a.states[slot].bond[k] = sh.bond[k];
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
    __syncthreads();
    // inclusive Hillis-Steele scan over the block
    for (int off = 1; off < NT; off <<= 1) {
      const int v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (c != 0) words[base + scan[threadIdx.x] - 1] = (uint32_t)(g * 4 + c);
    base += scan[NT - 1];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_init(const EngineArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(a.count), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_evolve(const EngineArgs& a, uint32_t n_layers, hipStream_t s) {
  hipLaunchKernelGGL(evolve_kernel, dim3(a.count), dim3(NT), 0, s, a, n_layers);
  return hipGetLastError();
}

hipError_t launch_observe(const EngineArgs& a, double* d_values, double* d_weights,
                          hipStream_t s) {
  hipLaunchKernelGGL(observe_kernel, dim3(a.count), dim3(NT), 0, s, a, d_values, d_weights);
  return hipGetLastError();
}

hipError_t launch_reduce(uint64_t count, uint32_t n_obs, const double* v, const double* w,
                         double* mean, double* se, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(n_obs), dim3(NT), 0, s, count, n_obs, v, w, mean, se);
  return hipGetLastError();
}

hipError_t launch_sample_count(const DevRow* rows, uint32_t l_eff, uint64_t seed,
                               uint64_t first_sample, uint64_t count, uint64_t n_draws,
                               uint64_t* d_counts, int8_t* d_signs, hipStream_t s) {
  hipLaunchKernelGGL(sample_count_kernel, dim3((uint32_t)count), dim3(NT), 0, s, rows, l_eff,
                     seed, first_sample, n_draws, d_counts, d_signs);
  return hipGetLastError();
}

hipError_t launch_sample_write(const DevRow* rows, uint32_t l_eff, uint64_t seed,
                               uint64_t first_sample, uint64_t count, uint64_t n_draws,
                               const uint64_t* d_offsets, uint32_t* d_words, hipStream_t s) {
  hipLaunchKernelGGL(sample_write_kernel, dim3((uint32_t)count), dim3(NT), 0, s, rows, l_eff,
                     seed, first_sample, n_draws, d_offsets, d_words);
  return hipGetLastError();
}

}  // namespace tepai
