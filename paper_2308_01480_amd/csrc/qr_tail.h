// Work-group (256-thread) factorisations of a small s x s Gram matrix (s <= SMAX <= 64)
// that turn a block into an orthonormal basis: the rank-revealing pivoted Cholesky (first
// pass) and the Cholesky inverse (second pass).  Lane l of every wave holds row l of the
// Schur complement, wave w its columns [w SMAX/4, (w+1) SMAX/4), so one elimination step
// costs each wave a quarter of the row update and a single barrier.  Used by the
// stand-alone transform kernels and by the last work-group of the fused block
// orthonormalisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "wave_ops.h"

namespace ttr {

// Argmax over the wave of (v, i) where i is the lane's own index or (1 << 30): the
// largest value, ties to the lowest lane (so to the smaller index); every lane gets the
// same pair.
__device__ inline void wave_argmax(double& v, int& i) {
  const double mx = max64(v);
  const uint64_t hit = __ballot(v == mx);
  const int lane = hit ? __builtin_ctzll(hit) : 0;
  i = __builtin_amdgcn_readlane(i, lane);
  v = mx;
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by three Newton steps (quadratic
// convergence from the estimate's relative error to float64 rounding level).
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  r = r * fma(-hx * r, r, 1.5);
  r = r * fma(-hx * r, r, 1.5);
  r = r * fma(-hx * r, r, 1.5);
  return r;
}

// Shared memory of the work-group QR tails below.
template <int SMAX>
struct alignas(16) QrTailSmem {
  static constexpr int P = SMAX + 1;
  alignas(16) double prow[2][SMAX];  // pivot row, double buffered across steps
  double rinv[SMAX];
  double Rm[SMAX * P];  // R rows in pivot order, columns in original order
  double Rt[SMAX * P];  // R_11 in pivot order (upper triangular, zero elsewhere)
  int rowid[SMAX];
  int keep[SMAX], pos[SMAX];
};
template <int SMAX>
constexpr size_t qr_tail_lds_bytes() { return sizeof(QrTailSmem<SMAX>) + (size_t)SMAX * SMAX * sizeof(double); }

// Column c of X = Rt^{-1} (Rt upper triangular k x k, pitch P, zero below the diagonal
// and beyond k; rinv[i] = 1 / Rt[i][i] or 0) by back substitution with the column in
// registers: x[i] = -(sum_{l > i} Rt[i][l] x[l]) rinv[i] for i < c, x[c] = rinv[c].
template <int SMAX, int P>
__device__ inline void tri_inverse_col(const double* Rt, const double* rinv, int k, int c, double (&x)[SMAX]) {
#pragma unroll
  for (int i = SMAX - 1; i >= 0; --i) {
    double acc = 0.0;
#pragma unroll
    for (int l = i + 1; l < SMAX; ++l) acc = fma(Rt[i * P + l], x[l], acc);
    x[i] = (i < k && i <= c) ? (i == c ? rinv[i] : -acc * rinv[i]) : 0.0;
  }
}

// Rank-revealing first pass: pivoted Cholesky of the s x s block Gram (pitch ldg).  Step j
// picks the largest remaining diagonal (ties to the smaller index; every wave finds the
// same pivot from its identical copy of the diagonal), the pivot row is exchanged through
// LDS and the remaining rows are updated; it stops at the first pivot <= thr or
// <= s 2^-52 d_0.  T (s x s) = E R_11^{-1}: row rowid[i], column c holds
// (R_11^{-1})[i][c]; *kept = k, the number of pivots taken.  All 256 threads call it.
template <int SMAX>
__device__ inline void qrcp_block(const double* Gm, int ldg, int s, double thr, double* __restrict__ T, int* kept,
                                  QrTailSmem<SMAX>& sm) {
  constexpr int P = QrTailSmem<SMAX>::P, CW = SMAX / 4;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, c0 = w * CW;
  double r[CW];
#pragma unroll
  for (int t = 0; t < CW; ++t) r[t] = (l < s && c0 + t < s) ? Gm[l * ldg + c0 + t] : 0.0;
  double diag = l < s ? Gm[l * ldg + l] : 0.0;
  bool remaining = l < s;
  for (int e = tid; e < SMAX * P; e += 256) { sm.Rm[e] = 0.0; sm.Rt[e] = 0.0; }
  if (tid < SMAX) sm.rinv[tid] = 0.0;
  __syncthreads();
  double d0 = 0.0;
  int k = 0;
  for (int j = 0; j < s; ++j) {
    double best = remaining ? diag : -1.0;
    int bi = remaining ? l : (1 << 30);
    wave_argmax(best, bi);
    if (j == 0) d0 = best;
    if (!(best > 0.0 && best > thr && best > (double)s * 0x1p-52 * d0)) break;
    const int pv = bi;
    double* pb = sm.prow[j & 1];
    if (l == pv) {
#pragma unroll
      for (int t = 0; t < CW; ++t) pb[c0 + t] = r[t];
    }
    __syncthreads();
    const double rinv = rsqrt_nr(best);
    if (l == pv) remaining = false;
    const double pl = l < SMAX ? pb[l] : 0.0;
    const double rl = remaining ? pl * rinv : (l == pv ? best * rinv : 0.0);
    if (w == 0 && l < SMAX) sm.Rm[j * P + l] = rl;
    if (tid == 0) { sm.rowid[j] = pv; sm.rinv[j] = rinv; }
    // rows already pivoted (and lanes beyond s) take a zero factor: no divergent update
    const double f = remaining ? -rl * rinv : 0.0;
#pragma unroll
    for (int t = 0; t < CW; ++t) r[t] = fma(f, pb[c0 + t], r[t]);
    diag = remaining ? fma(-rl, rl, diag) : diag;
    k = j + 1;
  }
  __syncthreads();
  // R_11 in pivot order, then column l of its inverse in registers (wave 0)
  for (int e = tid; e < k * k; e += 256) {
    const int i = e / k, c = e % k;
    if (c >= i) sm.Rt[i * P + c] = sm.Rm[i * P + sm.rowid[c]];
  }
  for (int e = tid; e < s * s; e += 256) T[e] = 0.0;
  __syncthreads();
  if (w == 0) {
    double x[SMAX];
    tri_inverse_col<SMAX, P>(sm.Rt, sm.rinv, k, l, x);
    if (l < k) {
#pragma unroll
      for (int i = 0; i < SMAX; ++i)
        if (i <= l) T[sm.rowid[i] * s + l] = x[i];
    }
    if (l == 0) *kept = k;
  }
}

// Second orthonormalisation pass: Gm (s x s, pitch ldg) = Q^T Q of a basis whose first
// k_in columns are non-zero and nearly orthonormal.  Cholesky of that leading block,
// Gm = R^T R; a column whose pivot is <= thresh is dropped (its row of R is zero, so it
// takes no part in the remaining factorisation).  T (s x s) = R^{-1} with the surviving
// columns packed first, zeros after; *kept_out = their number.  All 256 threads call it.
template <int SMAX>
__device__ inline void chol_inv_block(const double* Gm, int ldg, int s, int k_in, double thresh, double* __restrict__ T,
                                      int* kept_out, QrTailSmem<SMAX>& sm) {
  constexpr int P = QrTailSmem<SMAX>::P, CW = SMAX / 4;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, c0 = w * CW;
  const int k = k_in < s ? k_in : s;
  double r[CW];
#pragma unroll
  for (int t = 0; t < CW; ++t) r[t] = (l < k && c0 + t < k) ? Gm[l * ldg + c0 + t] : 0.0;
  for (int e = tid; e < SMAX * P; e += 256) sm.Rt[e] = 0.0;
  if (tid < SMAX) sm.rinv[tid] = 0.0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double* pb = sm.prow[j & 1];
    if (l == j) {
#pragma unroll
      for (int t = 0; t < CW; ++t) pb[c0 + t] = r[t];
    }
    __syncthreads();
    const double d = pb[j];
    const bool ok = d > thresh;
    const double rinv = ok ? rsqrt_nr(d) : 0.0;
    const double pl = l < SMAX ? pb[l] : 0.0;
    const double rl = (ok && l > j && l < k) ? pl * rinv : 0.0;
    if (w == 0 && l >= j && l < k) sm.Rt[j * P + l] = l == j ? (ok ? d * rinv : 0.0) : rl;
    if (tid == 0) { sm.keep[j] = ok; sm.rinv[j] = rinv; }
    const double f = -rl * rinv;  // zero for rows at or above j and for dropped pivots
#pragma unroll
    for (int t = 0; t < CW; ++t) r[t] = fma(f, pb[c0 + t], r[t]);
  }
  for (int e = tid; e < s * s; e += 256) T[e] = 0.0;
  __syncthreads();
  if (w == 0) {
    // packed positions of the surviving columns
    const bool kl = l < k && sm.keep[l];
    const uint64_t kb = __ballot(kl);
    const int c_out = __popcll(kb);
    if (l < k) sm.pos[l] = kl ? __popcll(kb & ((1ull << l) - 1ull)) : -1;
    if (l == 0) *kept_out = c_out;
    __builtin_amdgcn_wave_barrier();
    double x[SMAX];
    tri_inverse_col<SMAX, P>(sm.Rt, sm.rinv, k, l, x);
    if (l < k && sm.keep[l]) {
      const int pc = sm.pos[l];
#pragma unroll
      for (int i = 0; i < SMAX; ++i)
        if (i <= l && sm.keep[i]) T[i * s + pc] = x[i];
    }
  }
}

}  // namespace ttr
