// Block orthonormalisation of one Krylov block (Algorithm 3, steps 4-5) in a few
// row-parallel launches.
//
// Every kernel splits the m rows into chunks of RB rows (64, or 32 / 16 when the operands
// would not fit in LDS; 16 for the output kernel, which writes no partials and takes one
// work-group per chunk); work-group g takes chunks g, g + G, ... (G <= kOrthMaxGroups),
// stages each chunk in LDS with all of its global loads in flight at once, forms its
// products with float64 matrix-core instructions and writes one partial result.  The last work-group to finish (an
// atomic counter, reset by that work-group) sums the partials in group order, so the
// result does not depend on scheduling, and then runs the small s x s step:
//
//   orth_project   h = Q^T Y (and ||Y||_F^2)                         Q: m x js, Y: m x s
//   orth_update    P = S - Q h; then either h2 = Q^T P, or Gm = P^T P and the
//                  pivoted Cholesky T1 = E R_11^{-1} (rank-revealing first pass)
//   orth_tgram     U = P T1; Gm = U^T U and T2 = R^{-1} of its Cholesky (second pass)
//   orth_out       Q_j = U T2, also rounded into the zero-padded stream copy
//
// With S = Y this is block classical Gram-Schmidt run twice (P = Y - Q Q^T Y, then
// P -= Q Q^T P), followed by the rank-revealing QR of the projected block.
#include <hip/hip_runtime.h>

#include "common.h"
#include "convert.h"
#include "kernels.h"
#include "qr_tail.h"
#include "wave_ops.h"

namespace ttr {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kOrthThreads = 256;
constexpr int kOrthWaves = kOrthThreads / 64;

__device__ inline d4_t mma64(double a, double b, d4_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline d4_t zero4() { return d4_t{0.0, 0.0, 0.0, 0.0}; }

// Signals that this work-group has published its partial results; true in the last one
// to do so, which then sees every other group's partials.
__device__ inline bool last_group(int* counter) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (last) __threadfence();
  return last;
}

__device__ inline void release_counter(int* counter) {
  if (threadIdx.x == 0) atomicExch(counter, 0);
}

// Stages rows [r0, r0 + RB) x columns [0, kc) of src (ld lds) into Ds (pitch ldd), zero
// for rows >= r1.  All loads of a thread are issued before its LDS stores.
__device__ inline void stage_rows(const double* __restrict__ src, int64_t lds, int kc, int64_t r0, int64_t r1, int RB,
                                  double* __restrict__ Ds, int ldd) {
  const int total = RB * kc;
  for (int e0 = 0; e0 < total; e0 += 16 * kOrthThreads) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + u * kOrthThreads + (int)threadIdx.x;
      const int lr = e / kc, c = e - lr * kc;
      v[u] = (e < total && r0 + lr < r1) ? src[(r0 + lr) * lds + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + u * kOrthThreads + (int)threadIdx.x;
      const int lr = e / kc, c = e - lr * kc;
      if (e < total) Ds[lr * ldd + c] = v[u];
    }
  }
}

// Copies the ka x kb matrix W (row-major, pitch kb) into Ws (pitch kb).
__device__ inline void stage_matrix(const double* __restrict__ W, int len, double* __restrict__ Ws) {
  for (int e = threadIdx.x; e < len; e += kOrthThreads) Ws[e] = W[e];
}

__device__ inline void store_rows_global(const double* __restrict__ Ds, int ldd, int kb, int64_t r0, int64_t r1, int RB,
                                         double* __restrict__ dst, int64_t ldo) {
  for (int e = threadIdx.x; e < RB * kb; e += kOrthThreads) {
    const int lr = e / kb, c = e - lr * kb;
    if (r0 + lr < r1) dst[(r0 + lr) * ldo + c] = Ds[lr * ldd + c];
  }
}

// acc[t] (tile t = wave + kOrthWaves * i of the ka x kb output, 16 x 16 each) +=
// Xs^T Ys over the RB staged rows (pitches ldx, ldy; rows beyond the chunk are zero).
template <int MAXT>
__device__ inline void tn_tiles(const double* __restrict__ Xs, int ldx, int ka, const double* __restrict__ Ys, int ldy,
                                int kb, int RB, d4_t (&acc)[MAXT]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ta = (ka + 15) / 16, tb = (kb + 15) / 16;
  const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int tile = wave + kOrthWaves * t;
    if (tile >= ta * tb) break;
    const int a = (tile / tb) * 16 + i16, b = (tile % tb) * 16 + i16;
    const bool aok = a < ka, bok = b < kb;
    d4_t c = acc[t];
    for (int k0 = 0; k0 < RB; k0 += 16) {
      double xa[4], yv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = k0 + 4 * u + k4;
        xa[u] = aok ? Xs[row * ldx + a] : 0.0;
        yv[u] = bok ? Ys[row * ldy + b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) c = mma64(xa[u], yv[u], c);
    }
    acc[t] = c;
  }
}

// Ds (RB x kb, pitch ldd) = base - Xs W (SUB, base = Ds itself) or Xs W, with Xs the
// staged RB x ka rows (pitch ldx) and W (ka x kb, pitch kb) in LDS or global memory.
// Every output element is read (as base) and written by the same lane.
template <bool SUB>
__device__ inline void nn_rows(const double* __restrict__ Xs, int ldx, int ka, const double* W, int kb, int RB,
                               double* Ds, int ldd) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tb = (kb + 15) / 16;
  const int i16 = lane & 15, k4 = lane >> 4;
  for (int tile = wave; tile < (RB / 16) * tb; tile += kOrthWaves) {
    const int rt = tile / tb, ct = tile % tb;
    const int lrow = rt * 16 + i16;
    const int col = ct * 16 + i16;
    d4_t c = zero4();
    for (int k0 = 0; k0 < ka; k0 += 16) {
      double xa[4], wb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + k4;
        xa[u] = k < ka ? Xs[lrow * ldx + k] : 0.0;
        wb[u] = (k < ka && col < kb) ? W[k * kb + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) c = mma64(xa[u], wb[u], c);
    }
    if (col < kb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = rt * 16 + k4 + 4 * r;
        Ds[lr * ldd + col] = SUB ? Ds[lr * ldd + col] - c[r] : c[r];
      }
    }
  }
}

// Writes the tiles of acc into out (ka x kb, row-major).
template <int MAXT>
__device__ inline void store_tiles(const d4_t (&acc)[MAXT], int ka, int kb, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ta = (ka + 15) / 16, tb = (kb + 15) / 16;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int tile = wave + kOrthWaves * t;
    if (tile >= ta * tb) break;
    const int b = (tile % tb) * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = (tile / tb) * 16 + (lane >> 4) + 4 * r;
      if (a < ka && b < kb) out[(int64_t)a * kb + b] = acc[t][r];
    }
  }
}

// out[e] = sum over the G partials part[g * len + e], in group order.  Each thread keeps
// the G partials of four elements in flight at once (after the acquire in last_group
// these reads go past the cache, so the round trips, not the bytes, set the time).
__device__ inline void sum_partials(const double* __restrict__ part, int G, int len, double* __restrict__ out) {
  constexpr int U = 4;
  for (int e0 = 0; e0 < len; e0 += U * kOrthThreads) {
    double v[U][kOrthMaxGroups];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kOrthThreads + (int)threadIdx.x;
#pragma unroll
      for (int g = 0; g < kOrthMaxGroups; ++g) v[u][g] = (e < len && g < G) ? part[(int64_t)g * len + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kOrthThreads + (int)threadIdx.x;
      double acc = 0.0;
#pragma unroll
      for (int g = 0; g < kOrthMaxGroups; ++g) acc += v[u][g];
      if (e < len) out[e] = acc;
    }
  }
}

__device__ inline double block_total(double v) {
  __shared__ double red[kOrthWaves];
  v = sum64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------------------------
// orth_project: h (js x s) = Q^T Y; *ref = ||Y||_F^2 when ref is given.
// LDS: Q rows (RB x js+1), Y rows (RB x s+1).
// ---------------------------------------------------------------------------------
template <int MAXT, bool BIG = false>
__global__ __launch_bounds__(kOrthThreads) void k_orth_project(OrthArgs a, const double* __restrict__ Y, int64_t ldy,
                                                               int RB) {
  extern __shared__ __align__(16) double dsm[];
  const int lq = a.js + 1, ly = a.s + 1;
  double* Qs = dsm;
  double* Ys = Qs + RB * lq;
  const int G = gridDim.x;
  d4_t acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = zero4();
  double nrm = 0.0;
  const int64_t nchunks = (a.m + RB - 1) / RB;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += G) {
    const int64_t r0 = ch * RB, r1 = r0 + RB < a.m ? r0 + RB : a.m;
    stage_rows(a.Q, a.ldq, a.js, r0, r1, RB, Qs, lq);
    stage_rows(Y, ldy, a.s, r0, r1, RB, Ys, ly);
    __syncthreads();
    tn_tiles<MAXT>(Qs, lq, a.js, Ys, ly, a.s, RB, acc);
    if (a.ref)
      for (int e = threadIdx.x; e < RB * a.s; e += kOrthThreads) {
        const double v = Ys[(e / a.s) * ly + e % a.s];
        nrm = fma(v, v, nrm);
      }
    __syncthreads();
  }
  const int len = a.js * a.s;
  store_tiles<MAXT>(acc, a.js, a.s, a.part + (int64_t)blockIdx.x * len);
  if (a.ref) {
    const double t = block_total(nrm);
    if (threadIdx.x == 0) a.norm_part[blockIdx.x] = t;
  }
  if constexpr (BIG) return;
  if (!last_group(a.counter)) return;
  sum_partials(a.part, G, len, a.h);
  if (a.ref && threadIdx.x == 0) {
    double v[kOrthMaxGroups];
#pragma unroll
    for (int g = 0; g < kOrthMaxGroups; ++g) v[g] = g < G ? a.norm_part[g] : 0.0;
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < kOrthMaxGroups; ++g) t += v[g];
    *a.ref = t;
  }
  release_counter(a.counter);
}

// ---------------------------------------------------------------------------------
// orth_update: P = S - Q W (js >= 1) or P = S (js = 0), written to a.P; then
//   NEXT_PROJ: h2 = Q^T P into a.h2;
//   else     : Gm = P^T P, *ref = trace(Gm) when ref_from_gram, and the pivoted
//              Cholesky T1 = E R_11^{-1} (pivots <= coef * (*ref) dropped), kept1.
// LDS: W (js x s, when w_lds), Q rows (RB x js+1), P rows (RB x s+1).
// ---------------------------------------------------------------------------------
template <int SMAX, int MAXT, bool NEXT_PROJ, bool BIG = false>
__global__ __launch_bounds__(kOrthThreads) void k_orth_update(OrthArgs a, const double* __restrict__ S, int64_t lds_,
                                                              const double* __restrict__ W, int RB, int w_lds) {
  extern __shared__ __align__(16) double dsm[];
  const int lq = a.js + 1, lp = a.s + 1;
  double* Ws = dsm;
  double* Qs = Ws + (w_lds ? a.js * a.s : 0);
  double* Ps = Qs + (a.js > 0 ? RB * lq : 0);
  const double* Wp = w_lds ? Ws : W;
  const int G = gridDim.x;
  if (w_lds && a.js > 0) stage_matrix(W, a.js * a.s, Ws);
  d4_t acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = zero4();
  const int64_t nchunks = (a.m + RB - 1) / RB;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += G) {
    const int64_t r0 = ch * RB, r1 = r0 + RB < a.m ? r0 + RB : a.m;
    if (a.js > 0) stage_rows(a.Q, a.ldq, a.js, r0, r1, RB, Qs, lq);
    stage_rows(S, lds_, a.s, r0, r1, RB, Ps, lp);
    __syncthreads();
    if (a.js > 0) {
      nn_rows<true>(Qs, lq, a.js, Wp, a.s, RB, Ps, lp);
      __syncthreads();
    }
    store_rows_global(Ps, lp, a.s, r0, r1, RB, a.P, a.ldp);
    if (NEXT_PROJ) tn_tiles<MAXT>(Qs, lq, a.js, Ps, lp, a.s, RB, acc);
    else tn_tiles<MAXT>(Ps, lp, a.s, Ps, lp, a.s, RB, acc);
    __syncthreads();
  }
  const int ka = NEXT_PROJ ? a.js : a.s;
  const int len = ka * a.s;
  store_tiles<MAXT>(acc, ka, a.s, a.part + (int64_t)blockIdx.x * len);
  if constexpr (BIG) return;
  if (!last_group(a.counter)) return;
  if (NEXT_PROJ) {
    sum_partials(a.part, G, len, a.h2);
    release_counter(a.counter);
    return;
  }
  __shared__ double Gs[SMAX * SMAX];
  __shared__ QrTailSmem<SMAX> sm;
  sum_partials(a.part, G, len, Gs);
  __syncthreads();
  double thr;
  if (a.ref_from_gram) {
    double tr = 0.0;
    for (int i = 0; i < a.s; ++i) tr += Gs[i * a.s + i];
    if (threadIdx.x == 0) *a.ref = tr;
    thr = a.coef * tr;
  } else {
    thr = a.coef * (*a.ref);
  }
  qrcp_block<SMAX>(Gs, a.s, a.s, thr, a.T1, a.kept1, sm);
  release_counter(a.counter);
}

// ---------------------------------------------------------------------------------
// orth_tgram: U = P T1 (written to a.U); Gm = U^T U; T2 = R^{-1} of its Cholesky over
// the first kept1 columns (pivots <= thresh dropped, survivors packed), kept2;
// Tprod = T1 T2 when asked.  LDS: T1 (s x s), P rows, U rows (RB x s+1 each).
// ---------------------------------------------------------------------------------
template <int SMAX, int MAXT, bool BIG = false>
__global__ __launch_bounds__(kOrthThreads) void k_orth_tgram(OrthArgs a, int RB) {
  extern __shared__ __align__(16) double dsm[];
  const int lp = a.s + 1;
  double* Ts = dsm;
  double* Ps = Ts + a.s * a.s;
  double* Us = Ps + RB * lp;
  const int G = gridDim.x;
  stage_matrix(a.T1, a.s * a.s, Ts);
  d4_t acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = zero4();
  const int64_t nchunks = (a.m + RB - 1) / RB;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += G) {
    const int64_t r0 = ch * RB, r1 = r0 + RB < a.m ? r0 + RB : a.m;
    stage_rows(a.P, a.ldp, a.s, r0, r1, RB, Ps, lp);
    __syncthreads();
    nn_rows<false>(Ps, lp, a.s, Ts, a.s, RB, Us, lp);
    __syncthreads();
    store_rows_global(Us, lp, a.s, r0, r1, RB, a.U, a.ldu);
    tn_tiles<MAXT>(Us, lp, a.s, Us, lp, a.s, RB, acc);
    __syncthreads();
  }
  const int len = a.s * a.s;
  store_tiles<MAXT>(acc, a.s, a.s, a.part + (int64_t)blockIdx.x * len);
  if constexpr (BIG) return;
  if (!last_group(a.counter)) return;
  __shared__ double Gs[SMAX * SMAX];
  __shared__ QrTailSmem<SMAX> sm;
  sum_partials(a.part, G, len, Gs);
  __syncthreads();
  chol_inv_block<SMAX>(Gs, a.s, a.s, *a.kept1, a.thresh2, a.T2, a.kept2, sm);
  if (a.Tprod) {
    __threadfence();
    __syncthreads();
    for (int e = threadIdx.x; e < a.s * a.s; e += kOrthThreads) {
      const int i = e / a.s, j = e % a.s;
      double acc2 = 0.0;
      for (int l = 0; l < a.s; ++l) acc2 = fma(Ts[i * a.s + l], a.T2[l * a.s + j], acc2);
      a.Tprod[e] = acc2;
    }
  }
  release_counter(a.counter);
}

// ---------------------------------------------------------------------------------
// orth_out: Q_j = U T2 into a.Qout (ld ldqo) and, when zs is given, rounded into the
// stream copy zs (m_pad x Sz, dtype zdt; rows >= m and columns >= s are zero).
// LDS: T2 (s x s), U rows, Q rows (RB x s+1 each).
// ---------------------------------------------------------------------------------
template <typename TZ>
__global__ __launch_bounds__(kOrthThreads) void k_orth_out(OrthArgs a, int RB) {
  extern __shared__ __align__(16) double dsm[];
  const int lp = a.s + 1;
  double* Ts = dsm;
  double* Us = Ts + a.s * a.s;
  double* Os = Us + RB * lp;
  const int G = gridDim.x;
  stage_matrix(a.T2, a.s * a.s, Ts);
  const int64_t rows_z = a.zs ? a.m_pad : a.m;
  const int64_t nchunks = (rows_z + RB - 1) / RB;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += G) {
    const int64_t r0 = ch * RB, r1 = r0 + RB < a.m ? r0 + RB : a.m;
    stage_rows(a.U, a.ldu, a.s, r0, r1, RB, Us, lp);
    __syncthreads();
    nn_rows<false>(Us, lp, a.s, Ts, a.s, RB, Os, lp);
    __syncthreads();
    store_rows_global(Os, lp, a.s, r0, r1, RB, a.Qout, a.ldqo);
    if (a.zs) {
      TZ* z = static_cast<TZ*>(a.zs);
      for (int e = threadIdx.x; e < RB * a.Sz; e += kOrthThreads) {
        const int lr = e / a.Sz, c = e - lr * a.Sz;
        const int64_t row = r0 + lr;
        if (row < a.m_pad) z[row * a.Sz + c] = (row < a.m && c < a.s) ? round_from_f64<TZ>(Os[lr * lp + c]) : TZ(0);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------
// Split reduction of tall blocks: out[e] = sum over the G row-group partials
// part[g * len + e] for e < len; each output's G partials are summed by eight thread
// slices over contiguous group ranges, combined in slice order (a fixed order).  The last
// work-group then runs the block's s x s step on the sum:
//   TAIL_NONE  nothing (h = Q^T Y, h2 = Q^T P)
//   TAIL_NORM  *ref = ||Y||_F^2 from the groups' partial norms
//   TAIL_QRCP  rank-revealing pivoted Cholesky of Gm = P^T P (as orth_update's tail)
//   TAIL_CHOL  Cholesky inverse of Gm = U^T U, and T1 T2 when asked (as orth_tgram's tail)
// ---------------------------------------------------------------------------------
enum { TAIL_NONE = 0, TAIL_NORM = 1, TAIL_QRCP = 2, TAIL_CHOL = 3 };
constexpr int kRedSegO = 8;
constexpr int kRedOutsO = kOrthThreads / kRedSegO;

template <int SMAX, int TAIL>
__global__ __launch_bounds__(kOrthThreads) void k_orth_reduce(OrthArgs a, int G, int len, double* __restrict__ out) {
  __shared__ double red[kRedSegO][kRedOutsO];
  const int o = threadIdx.x % kRedOutsO, seg = threadIdx.x / kRedOutsO;
  const int e = blockIdx.x * kRedOutsO + o;
  const int per = (G + kRedSegO - 1) / kRedSegO;
  const int g0 = seg * per, g1 = g0 + per < G ? g0 + per : G;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < len) {
    int g = g0;
    for (; g + 4 <= g1; g += 4)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += a.part[(int64_t)(g + u) * len + e];
    for (int u = 0; g < g1; ++g, ++u) acc[u] += a.part[(int64_t)g * len + e];
  }
  red[seg][o] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (seg == 0 && e < len) {
    double t = red[0][o];
#pragma unroll
    for (int k = 1; k < kRedSegO; ++k) t += red[k][o];
    out[e] = t;
  }
  if (TAIL == TAIL_NONE) return;
  if (!last_group(a.counter)) return;
  if constexpr (TAIL == TAIL_NORM) {
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int g = 0; g < G; ++g) t += a.norm_part[g];
      *a.ref = t;
    }
  } else {
    __shared__ double Gs[SMAX * SMAX];
    __shared__ QrTailSmem<SMAX> sm;
    for (int i = threadIdx.x; i < len; i += kOrthThreads) Gs[i] = out[i];
    __syncthreads();
    if constexpr (TAIL == TAIL_QRCP) {
      double thr;
      if (a.ref_from_gram) {
        double tr = 0.0;
        for (int i = 0; i < a.s; ++i) tr += Gs[i * a.s + i];
        if (threadIdx.x == 0) *a.ref = tr;
        thr = a.coef * tr;
      } else {
        thr = a.coef * (*a.ref);
      }
      qrcp_block<SMAX>(Gs, a.s, a.s, thr, a.T1, a.kept1, sm);
    } else {
      chol_inv_block<SMAX>(Gs, a.s, a.s, *a.kept1, a.thresh2, a.T2, a.kept2, sm);
      if (a.Tprod) {
        __threadfence();
        __syncthreads();
        for (int q = threadIdx.x; q < a.s * a.s; q += kOrthThreads) {
          const int i = q / a.s, j = q % a.s;
          double acc2 = 0.0;
          for (int l = 0; l < a.s; ++l) acc2 = fma(a.T1[i * a.s + l], a.T2[l * a.s + j], acc2);
          a.Tprod[q] = acc2;
        }
      }
    }
  }
  release_counter(a.counter);
}

__global__ void k_zero_int(int* p) { *p = 0; }

// ---------------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------------
static int orth_groups(int64_t rows, int RB, bool big = false) {
  const int64_t c = (rows + RB - 1) / RB;
  const int64_t cap = big ? kOrthBigGroups : kOrthMaxGroups;
  return (int)(c < cap ? (c < 1 ? 1 : c) : cap);
}

template <int SMAX, int TAIL>
static hipError_t reduce_launch(const OrthArgs& a, int G, int len, double* out) {
  hipLaunchKernelGGL((k_orth_reduce<SMAX, TAIL>), dim3((unsigned)((len + kRedOutsO - 1) / kRedOutsO)),
                     dim3(kOrthThreads), 0, a.st, a, G, len, out);
  return hipGetLastError();
}

// The split reduction of a tall block's partials (see k_orth_reduce).
static hipError_t orth_reduce(const OrthArgs& a, int G, int len, double* out, int tail) {
  if (tail == TAIL_NONE) return reduce_launch<16, TAIL_NONE>(a, G, len, out);
  if (tail == TAIL_NORM) return reduce_launch<16, TAIL_NORM>(a, G, len, out);
  if (!a.gsum) return hipErrorInvalidValue;
#define TTR_RED_TAIL(SM)                                                                       \
  if (a.s <= SM) return tail == TAIL_QRCP ? reduce_launch<SM, TAIL_QRCP>(a, G, len, a.gsum)    \
                                          : reduce_launch<SM, TAIL_CHOL>(a, G, len, a.gsum);
  TTR_RED_TAIL(16) TTR_RED_TAIL(32) TTR_RED_TAIL(48) TTR_RED_TAIL(64)
#undef TTR_RED_TAIL
  return hipErrorInvalidValue;
}

template <typename F>
static hipError_t orth_set_lds(F kernel, size_t bytes) {
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

// Largest row chunk RB in {64, 32, 16} whose dynamic LDS (doubles: fixed + RB * per_row)
// fits next to `static_bytes`; 0 if none does.
static int pick_rows(size_t fixed, size_t per_row, size_t static_bytes, size_t* bytes) {
  for (int rb = 64; rb >= 16; rb /= 2) {
    const size_t b = (fixed + (size_t)rb * per_row) * sizeof(double);
    if (b + static_bytes + 1024 <= (size_t)kLdsBytes) { *bytes = b; return rb; }
  }
  return 0;
}

hipError_t orth_reset_counter(int* counter, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, counter);
  return hipGetLastError();
}

static bool orth_args_ok(const OrthArgs& a) {
  return a.m > 0 && a.s >= 1 && a.s <= 64 && a.js >= 0 && a.counter && a.part;
}
static bool part_ok(const OrthArgs& a, int G, int ka) {
  return (size_t)G * (size_t)(ka > 0 ? ka : 1) * a.s * sizeof(double) <= a.part_bytes;
}

template <int MAXT>
static hipError_t project_t(const OrthArgs& a, const double* Y, int64_t ldy, int RB, size_t lds) {
  auto kern = a.big ? k_orth_project<MAXT, true> : k_orth_project<MAXT, false>;
  hipError_t e = orth_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int G = orth_groups(a.m, RB, a.big);
  hipLaunchKernelGGL(kern, dim3(G), dim3(kOrthThreads), lds, a.st, a, Y, ldy, RB);
  if ((e = hipGetLastError()) != hipSuccess || !a.big) return e;
  return orth_reduce(a, G, a.js * a.s, a.h, a.ref ? TAIL_NORM : TAIL_NONE);
}

hipError_t orth_project(const OrthArgs& a, const double* Y, int64_t ldy) {
  if (!orth_args_ok(a) || a.js < 1 || !a.h || (a.ref && !a.norm_part)) return hipErrorInvalidValue;
  size_t lds = 0;
  const int RB = pick_rows(0, (size_t)(a.js + 1) + (a.s + 1), 0, &lds);
  if (!RB || !part_ok(a, orth_groups(a.m, RB, a.big), a.js)) return hipErrorInvalidValue;
  const int tiles = ((a.js + 15) / 16) * ((a.s + 15) / 16);
  if (tiles <= 4 * kOrthWaves) return project_t<4>(a, Y, ldy, RB, lds);
  if (tiles <= 8 * kOrthWaves) return project_t<8>(a, Y, ldy, RB, lds);
  if (tiles <= 16 * kOrthWaves) return project_t<16>(a, Y, ldy, RB, lds);
  return hipErrorInvalidValue;
}

template <int SMAX, int MAXT, bool NP>
static hipError_t update_launch(const OrthArgs& a, const double* S, int64_t lds_, const double* W) {
  const size_t tail = (NP || a.big) ? 0 : qr_tail_lds_bytes<SMAX>();
  const size_t per_row = (size_t)(a.js > 0 ? a.js + 1 : 0) + (a.s + 1);
  size_t lds = 0;
  int w_lds = a.js > 0 ? 1 : 0;
  int RB = pick_rows(w_lds ? (size_t)a.js * a.s : 0, per_row, tail, &lds);
  if (!RB && w_lds) { w_lds = 0; RB = pick_rows(0, per_row, tail, &lds); }
  const int G = orth_groups(a.m, RB, a.big);
  if (!RB || !part_ok(a, G, NP ? a.js : a.s)) return hipErrorInvalidValue;
  auto kern = a.big ? k_orth_update<SMAX, MAXT, NP, true> : k_orth_update<SMAX, MAXT, NP, false>;
  hipError_t e = orth_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(G), dim3(kOrthThreads), lds, a.st, a, S, lds_, W, RB, w_lds);
  if ((e = hipGetLastError()) != hipSuccess || !a.big) return e;
  return NP ? orth_reduce(a, G, a.js * a.s, a.h2, TAIL_NONE) : orth_reduce(a, G, a.s * a.s, nullptr, TAIL_QRCP);
}

template <int SMAX, bool NP>
static hipError_t update_t(const OrthArgs& a, const double* S, int64_t lds_, const double* W) {
  const int ka = NP ? a.js : a.s;
  const int tiles = ((ka + 15) / 16) * ((a.s + 15) / 16);
  if (tiles <= 4 * kOrthWaves) return update_launch<SMAX, 4, NP>(a, S, lds_, W);
  if (tiles <= 8 * kOrthWaves) return update_launch<SMAX, 8, NP>(a, S, lds_, W);
  if (tiles <= 16 * kOrthWaves) return update_launch<SMAX, 16, NP>(a, S, lds_, W);
  return hipErrorInvalidValue;
}

hipError_t orth_update(const OrthArgs& a, const double* S, int64_t lds_, const double* W, bool next_proj) {
  if (!orth_args_ok(a) || (next_proj && (a.js < 1 || !a.h2)) || !a.P || !S) return hipErrorInvalidValue;
  if (a.js > 0 && !W) return hipErrorInvalidValue;
  if (!next_proj && (!a.T1 || !a.kept1 || !a.ref)) return hipErrorInvalidValue;
  if (a.s <= 16) return next_proj ? update_t<16, true>(a, S, lds_, W) : update_t<16, false>(a, S, lds_, W);
  if (a.s <= 32) return next_proj ? update_t<32, true>(a, S, lds_, W) : update_t<32, false>(a, S, lds_, W);
  if (a.s <= 48) return next_proj ? update_t<48, true>(a, S, lds_, W) : update_t<48, false>(a, S, lds_, W);
  return next_proj ? update_t<64, true>(a, S, lds_, W) : update_t<64, false>(a, S, lds_, W);
}

template <int SMAX>
static hipError_t tgram_t(const OrthArgs& a) {
  size_t lds = 0;
  const int RB = pick_rows((size_t)a.s * a.s, 2 * (size_t)(a.s + 1), a.big ? 0 : qr_tail_lds_bytes<SMAX>(), &lds);
  const int G = orth_groups(a.m, RB, a.big);
  if (!RB || !part_ok(a, G, a.s)) return hipErrorInvalidValue;
  auto kern = a.big ? k_orth_tgram<SMAX, 4, true> : k_orth_tgram<SMAX, 4, false>;
  hipError_t e = orth_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(G), dim3(kOrthThreads), lds, a.st, a, RB);
  if ((e = hipGetLastError()) != hipSuccess || !a.big) return e;
  return orth_reduce(a, G, a.s * a.s, nullptr, TAIL_CHOL);
}

hipError_t orth_tgram(const OrthArgs& a) {
  if (!orth_args_ok(a) || !a.P || !a.U || !a.T1 || !a.T2 || !a.kept1 || !a.kept2) return hipErrorInvalidValue;
  if (a.s <= 16) return tgram_t<16>(a);
  if (a.s <= 32) return tgram_t<32>(a);
  if (a.s <= 48) return tgram_t<48>(a);
  return tgram_t<64>(a);
}

// The output has no partials, so it is not held to kOrthMaxGroups: one work-group per
// 16-row chunk.
template <typename TZ>
static hipError_t out_t(const OrthArgs& a) {
  constexpr int RB = 16;
  const size_t lds = ((size_t)a.s * a.s + (size_t)RB * 2 * (a.s + 1)) * sizeof(double);
  if (lds + 1024 > (size_t)kLdsBytes) return hipErrorInvalidValue;
  auto kern = k_orth_out<TZ>;
  hipError_t e = orth_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int64_t rows = a.zs ? a.m_pad : a.m;
  hipLaunchKernelGGL(kern, dim3((unsigned)((rows + RB - 1) / RB)), dim3(kOrthThreads), lds, a.st, a, RB);
  return hipGetLastError();
}

hipError_t orth_out(const OrthArgs& a) {
  if (a.m <= 0 || a.s < 1 || a.s > 64 || !a.U || !a.T2 || !a.Qout) return hipErrorInvalidValue;
  if (a.zs && (a.m_pad < a.m || a.Sz < a.s)) return hipErrorInvalidValue;
  if (!a.zs || a.zdt == TTR_F64) return out_t<double>(a);
  if (a.zdt == TTR_F32) return out_t<float>(a);
  return out_t<__bf16>(a);
}

}  // namespace ttr
