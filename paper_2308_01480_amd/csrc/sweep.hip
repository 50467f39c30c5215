// Host driver of the TT-RBKI sweep (Algorithm 3) and the C-ABI entry points.
//
// Everything is enqueued on the caller's stream; the host never waits inside a call,
// because every shape is fixed by the plan: dropped Krylov directions become zero
// columns and counts live in device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"
#include "driver.h"
#include "kernels.h"

namespace ttr {

#define TTR_CHECK(expr)                                                        \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      (void)hipGetLastError();                                                 \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
      return TTR_EHIP;                                                         \
    }                                                                          \
  } while (0)

// Carving of the `small` workspace region: square n_e x n_e float64 matrices,
// split-K partials, per-block scalars and counters.
struct SmallBufs {
  double* gram;   // Gram / Rayleigh-Ritz matrix
  double* vecs;   // eigenvectors
  double* vals;   // eigenvalues
  double* tmat;   // SVQB transform, Ritz selection U
  double* hmat;   // projection coefficients Q_prev^T P
  double* eigw;   // eigen work (n > 128)
  double* splitk; // split-K partials of X^T Y products
  double* scal;   // ||Y_j||_F^2 per block
  int* ints;      // kept counts
  size_t splitk_bytes = 0;     // bytes of splitk (also the block orthonormalisation partials)
  double* norm_part = nullptr; // kOrthMaxGroups partial norms
  int* counter = nullptr;      // last-work-group counter of the block orthonormalisation
  // tall blocks: partials of up to kOrthBigGroups row work-groups, their norms, the s x s sum
  double* big_part = nullptr;
  size_t big_part_bytes = 0;
  double* big_norm = nullptr;
  double* big_gsum = nullptr;
};

static SmallBufs carve_small(char* base, size_t bytes, int ne) {
  SmallBufs b;
  const size_t sq = (size_t)ne * ne;
  double* p = reinterpret_cast<double*>(base);
  b.gram = p; p += sq;
  b.vecs = p; p += sq;
  b.tmat = p; p += sq;
  b.hmat = p; p += sq;
  b.eigw = p; p += 2 * sq + 3 * kMaxSmall;  // eigen work when n > 128: (n + 3) rows of pitch 256
  b.splitk = p; p += 15 * sq;
  b.vals = p; p += 512;
  b.scal = p; p += 512;
  b.ints = reinterpret_cast<int*>(p); p += 512;
  b.splitk_bytes = 15 * sq * sizeof(double);
  b.norm_part = b.scal + 448;
  b.counter = b.ints + 1023;
  (void)bytes;
  return b;
}

struct ModeCtx {
  const ModeTape* tape = nullptr;
  const void* A;
  int adt;
  const ModeGeom* g;
  int q;
  uint64_t seed;
  double tau;
  double* core;   // m x r float64 output (core k)
  void* carry;    // r x n output, dtype cdt
  int cdt;
  char* ws;
  const Layout* lay;
  SmallBufs sb;
  hipStream_t st;
  int* status;    // non-finite flag of the call
  const ModeGeom* next = nullptr;  // geometry of mode k + 1 (nullptr for the last carry)
  bool sketch_ready = false;       // Y0 of this mode already in pbuf (formed with the last carry)
  bool* fused_next = nullptr;      // set when this mode's carry also formed mode k + 1's Y0
};

// Rank-revealing orthonormal basis of P (m x s), the economy QR of Algorithm 3
// step 5 with column pivoting: the block Gram's pivoted Cholesky keeps the leading
// pivots with |R_jj|^2 > coef * (*ref) and gives Q1 = P R_11^{-1} (scattered), then a
// Cholesky QR pass restores the orthogonality lost to the Gram's squared
// conditioning.  Q (ld ldq) gets the kept columns first, zeros after; *kept2 is
// their number.  Uses `tmp` (m x s) as the intermediate basis.
// Common fields of the block orthonormalisation launches.
static OrthArgs orth_args(int64_t m, int s, double coef, const SmallBufs& sb, hipStream_t st) {
  OrthArgs a;
  a.m = m; a.s = s; a.coef = coef; a.thresh2 = 1e-6;
  a.part = sb.splitk; a.part_bytes = sb.splitk_bytes; a.norm_part = sb.norm_part; a.counter = sb.counter;
  if (orth_big_rows(m) && sb.big_part) {
    a.big = true;
    a.part = sb.big_part; a.part_bytes = sb.big_part_bytes; a.norm_part = sb.big_norm; a.gsum = sb.big_gsum;
  }
  a.h = sb.vecs; a.h2 = sb.gram; a.T1 = sb.tmat; a.T2 = sb.hmat;
  a.st = st;
  return a;
}

// Rank-revealing orthonormal basis Q (ld ldq) of the m x s block Src (ld s), with drops
// relative to *ref: the pivoted Cholesky of P^T P (first pass) then a Cholesky-QR pass;
// P (m x s) receives a copy of Src (may be Src itself), tmp the first-pass basis, and
// tprod = T1 T2 when given.
// ref_from_gram: *ref is written with ||Src||_F^2 (the trace of the block Gram) before use.
static int orth_block(const double* Src, double* P, int64_t m, int s, double* ref, double coef, double* Q, int64_t ldq,
                      double* tmp, int* kept1, int* kept2, const SmallBufs& sb, hipStream_t st,
                      double* tprod = nullptr, bool ref_from_gram = false) {
  OrthArgs a = orth_args(m, s, coef, sb, st);
  a.P = P; a.ldp = s; a.U = tmp; a.ldu = s; a.ref = ref; a.kept1 = kept1; a.kept2 = kept2; a.Tprod = tprod;
  a.ref_from_gram = ref_from_gram;
  a.Qout = Q; a.ldqo = ldq;
  TTR_CHECK(orth_update(a, Src, s, nullptr, false));
  TTR_CHECK(orth_tgram(a));
  TTR_CHECK(orth_out(a));
  return TTR_OK;
}

// Eigenpairs of a small symmetric Gram / Rayleigh-Ritz matrix.  The sweep keeps only the
// r leading pairs; the gradient's forward pass records the full decomposition (its
// adjoint couples kept and discarded directions), and both use the same vectors for G.
static hipError_t eigen(const ModeCtx& c, const double* a, int n, int r, double* vecs, double* vals) {
  if (c.tape) return sym_eig(a, n, vecs, vals, c.sb.eigw, c.st);
  return sym_eig_top(a, n, r, vecs, vals, c.sb.eigw, c.st);
}

// Float32 streams of tall, wide unfoldings multiply on the bf16 matrix cores with three-way
// split operands, which keeps float32 accuracy (split_f32_mode; launch_aw_split,
// launch_atz_split).
static bool split_products(const ModeCtx& c) { return split_f32_mode(c.adt, c.g->m_pad, c.g->n); }

// Whether mode k + 1's sketch Y0 = A_{k+1} Omega_{k+1} (Algorithm 3, step 3) can be formed in
// the pass that writes the carry: a bfloat16 short unfolding with a float32 carry, followed by
// a regular Rayleigh-Ritz mode that would sketch its float32 unfolding from HBM.
static bool fuse_next_sketch(const ModeCtx& c) {
  const ModeGeom& g = *c.g;
  const ModeGeom* nx = c.next;
  if (!nx || c.tape || !c.fused_next || c.adt != TTR_BF16 || c.cdt != TTR_F32) return false;
  if (nx->kind != TTR_MODE_REGULAR || nx->method != TTR_METHOD_RBKI || nx->literal || nx->gram_first) return false;
  if (nx->n <= 0 || g.n % nx->n != 0 || nx->m != (int64_t)g.r * (g.n / nx->n) || nx->s > nx->S) return false;
  if (!carry_sketch_fits(c.adt, g.m_pad, pad16(g.r), g.n, nx->n, nx->S)) return false;
  return carry_sketch_part_bytes(g.n, nx->n, pad16(g.r), nx->S) <= c.lay->partials_bytes;
}

// Carry C = G^T A (r x n) through the A^T Z kernel with Z = G rounded to A's dtype; when
// fuse_next_sketch holds, the same pass also forms the next mode's Y0 into pbuf, with its
// Omega drawn (transposed, float32) into wbuf first.
static int carry_pass(const ModeCtx& c) {
  const ModeGeom& g = *c.g;
  const int R = pad16(g.r);
  char* zs = c.ws + c.lay->zs;
  TTR_CHECK(convert_pad(c.core, TTR_F64, g.m, g.r, g.r, zs, c.adt, g.m_pad, R, R, c.st));
  StreamArgs sa;
  sa.A = c.A; sa.dtype = c.adt; sa.m = g.m; sa.n = g.n; sa.m_pad = g.m_pad;
  sa.Z = zs; sa.S = R; sa.s = g.r; sa.stream = c.st;
  sa.part = c.ws + c.lay->partials; sa.part_bytes = c.lay->partials_bytes;  // row-split partials of short unfoldings
  sa.split_f32 = split_products(c);
  if (fuse_next_sketch(c)) {
    const ModeGeom& nx = *c.next;
    float* omt = reinterpret_cast<float*>(c.ws + c.lay->wbuf);
    double* y0 = reinterpret_cast<double*>(c.ws + c.lay->pbuf);
    TTR_CHECK(launch_omega_t(c.seed, nx.k, nx.n, nx.s, nx.S, nx.n, omt, c.st));
    TTR_CHECK(launch_carry_sketch_bf16(sa, static_cast<float*>(c.carry), g.n, g.r, omt, nx.n, nx.S, nx.s, y0, nx.s));
    *c.fused_next = true;
    return TTR_OK;
  }
  TTR_CHECK(launch_atz(sa, c.carry, c.cdt, g.n, g.r, 1));
  return TTR_OK;
}

// Sketch Y = A Omega_k (Algorithm 3, step 3) into sa.y: for short unfoldings (one row block
// of the A W kernel) Omega_k is drawn inside the streaming kernel; taller ones materialise
// it (n x width, stream dtype) in wbuf, where the A W kernel's row blocks share it.
static hipError_t sketch_pass(StreamArgs sa, uint64_t seed, int k, int width, void* wbuf) {
  if (sa.m_pad <= kAwRows) {
    sa.seed = seed; sa.kmode = k;
    return launch_aw_omega(sa);
  }
  hipError_t e = launch_omega(seed, k, 0, sa.n, sa.s, width, wbuf, sa.dtype, sa.stream);
  if (e != hipSuccess) return e;
  sa.W = wbuf;
  sa.w_f32 = true;  // Omega materialised as float32 n x width
  return launch_aw(sa);
}

static int run_regular(const ModeCtx& c) {
  const ModeGeom& g = *c.g;
  const int64_t m = g.m;
  const int s = g.s, S = g.S, w = g.w, q = c.q;
  char* ws = c.ws;
  const Layout& L = *c.lay;
  const SmallBufs& sb = c.sb;
  double* ybuf = reinterpret_cast<double*>(ws + L.ybuf);
  double* pbuf = reinterpret_cast<double*>(ws + L.pbuf);
  double* yall = c.tape ? c.tape->Yall : reinterpret_cast<double*>(ws + L.yall);
  double* qbuf = c.tape ? c.tape->Q : reinterpret_cast<double*>(ws + L.qbuf);
  int* kept = c.tape ? c.tape->ints : nullptr;
  void* wbuf = ws + L.wbuf;
  void* zs = ws + L.zs;
  const double coef = c.tau * c.tau;

  StreamArgs sa;
  sa.A = c.A; sa.dtype = c.adt; sa.m = m; sa.n = g.n; sa.m_pad = g.m_pad;
  sa.part = ws + L.partials; sa.part_bytes = L.partials_bytes; sa.S = S; sa.s = s; sa.stream = c.st;
  sa.split_f32 = split_products(c);

  // Gram-first (short unfoldings): A A^T (m x m, float64) in one streaming pass; every
  // Krylov product below is then (A A^T) Q_{j-1} in float64 (the taped forward sweep of the
  // gradient entry streams, as its reverse sweep does).
  const bool gram = g.gram_first && !c.tape;
  double* gm = reinterpret_cast<double*>(ws + L.gram);

  // Sketch Y0 = A Omega_k (Algorithm 3, step 3) and its orthonormal basis Q_0; every
  // basis block is also written, rounded and zero padded, into zs for the next product.
  sa.y = pbuf; sa.ldy = s;
  if (gram) {
    // The Gram and the sketch in one pass, Omega_k drawn inside the kernel.  float32 input
    // takes float64 Gram products (exact) and sums, so the Gram's rounding stays far below
    // what its small eigen-directions can absorb; bfloat16 and float64 input keep their own
    // matrix-core products (float32 and float64 sums).
    sa.seed = c.seed; sa.kmode = g.k;
    TTR_CHECK(launch_gram_sketch(sa, gm));
  } else if (!c.sketch_ready) {
    TTR_CHECK(sketch_pass(sa, c.seed, g.k, S, wbuf));
  }  // else Y0 was formed in pbuf by the previous mode's carry pass
  // every entry of A reaches Y0 through a dense Omega row: a NaN or infinity in A (or an
  // overflow of the products) leaves a non-finite entry here
  TTR_CHECK(flag_nonfinite(pbuf, m * s, c.status, c.st));
  OrthArgs oa = orth_args(m, s, coef, sb, c.st);
  oa.Q = qbuf; oa.ldq = w; oa.P = pbuf; oa.ldp = s; oa.U = ybuf; oa.ldu = s;
  oa.zs = zs; oa.zdt = c.adt; oa.m_pad = g.m_pad; oa.Sz = S;
  oa.js = 0; oa.ref = sb.scal + 0; oa.ref_from_gram = true;
  oa.kept1 = sb.ints + 0; oa.kept2 = kept ? kept : sb.ints + 1;
  oa.Tprod = c.tape ? c.tape->T : nullptr;
  oa.Qout = qbuf; oa.ldqo = w;
  TTR_CHECK(orth_update(oa, pbuf, s, nullptr, false));
  TTR_CHECK(orth_tgram(oa));
  TTR_CHECK(orth_out(oa));

  // Krylov blocks Y_j = A A^T Q_{j-1}, j = 1..q+1 (the last one only feeds Rayleigh-Ritz).
  for (int j = 1; j <= q + 1; ++j) {
    double* yj = yall + (j - 1) * s;
    sa.Z = zs; sa.y = yj; sa.ldy = w;
    if (gram) {
      TTR_CHECK(gemm_nn(m, (int)m, s, gm, TTR_F64, m, qbuf + (j - 1) * s, w, 1.0, 0.0, yj, w, c.st));
    } else if (!g.two_pass) {
      TTR_CHECK(launch_fused(sa));
    } else {
      TTR_CHECK(launch_atz(sa, wbuf, c.adt, S, S, 0));
      sa.W = wbuf;
      TTR_CHECK(launch_aw(sa));
    }
    if (j > q) break;
    // P = Y_j - Q Q^T Y_j, then P -= Q Q^T P (Q = Q_0..Q_{j-1}), orthonormalised with
    // drops relative to ||Y_j||_F.
    oa.js = j * s; oa.ref = sb.scal + j; oa.ref_from_gram = false;
    oa.kept1 = sb.ints + 2 * j; oa.kept2 = kept ? kept + j : sb.ints + 2 * j + 1;
    oa.Tprod = c.tape ? c.tape->T + (size_t)j * s * s : nullptr;
    oa.Qout = qbuf + j * s;
    TTR_CHECK(orth_project(oa, yj, w));
    TTR_CHECK(orth_update(oa, yj, w, oa.h, true));
    TTR_CHECK(orth_update(oa, pbuf, s, oa.h2, false));
    TTR_CHECK(orth_tgram(oa));
    TTR_CHECK(orth_out(oa));
  }

  // Rayleigh-Ritz: M = Q^T A A^T Q = Q^T [Y_1 .. Y_{q+1}], top-r eigenvectors, G = Q U.
  TTR_CHECK(gemm_tn_sym(m, w, qbuf, w, yall, w, sb.gram, w, sb.splitk, c.st));
  double* evec = c.tape ? c.tape->U : sb.vecs;
  double* eval = c.tape ? c.tape->lam : sb.vals;
  TTR_CHECK(eigen(c, sb.gram, w, g.r, evec, eval));
  int* nv = c.tape ? c.tape->ints + q + 1 : sb.ints + 1020;
  TTR_CHECK(gemm_nn_ritz(m, w, g.r, qbuf, w, evec, eval, c.core, g.r, nv, c.st));
  TTR_CHECK(complete_columns(c.core, m, g.r, nv, ybuf, c.st));
  return carry_pass(c);
}

// TT-rSI (Algorithm 4), TT-rSVD (Algorithm 2) and the printed first-r-columns forms of all
// three drivers.  One block of b columns (b = s for Rayleigh-Ritz, b = r for the printed
// truncation): the sketch Y = A Omega_b, then `iters` products Y = A (A^T Q) of the
// renormalised block, each followed by the rank-revealing orthonormalisation (the printed
// n-side QR between the two halves of a product only rescales the block by a triangular
// factor, so the spans agree).  The printed truncation takes the final basis itself (any
// orthonormal basis of the span of the first r columns gives the same tensor); the
// Rayleigh-Ritz form takes the r leading Ritz directions of one more product.
static int run_power(const ModeCtx& c) {
  const ModeGeom& g = *c.g;
  const int64_t m = g.m;
  const int b = g.b, B = pad16(b);
  char* ws = c.ws;
  const Layout& L = *c.lay;
  const SmallBufs& sb = c.sb;
  double* ybuf = reinterpret_cast<double*>(ws + L.ybuf);
  double* pbuf = reinterpret_cast<double*>(ws + L.pbuf);
  double* yall = reinterpret_cast<double*>(ws + L.yall);
  double* qbuf = reinterpret_cast<double*>(ws + L.qbuf);
  void* wbuf = ws + L.wbuf;
  void* zs = ws + L.zs;

  StreamArgs sa;
  sa.A = c.A; sa.dtype = c.adt; sa.m = m; sa.n = g.n; sa.m_pad = g.m_pad;
  sa.part = ws + L.partials; sa.part_bytes = L.partials_bytes; sa.S = B; sa.s = b; sa.stream = c.st;
  sa.split_f32 = split_products(c);

  sa.y = pbuf; sa.ldy = b;
  TTR_CHECK(sketch_pass(sa, c.seed, g.k, B, wbuf));
  TTR_CHECK(flag_nonfinite(pbuf, m * b, c.status, c.st));
  OrthArgs oa = orth_args(m, b, c.tau * c.tau, sb, c.st);
  oa.Q = qbuf; oa.ldq = b; oa.P = pbuf; oa.ldp = b; oa.U = ybuf; oa.ldu = b;
  oa.zs = zs; oa.zdt = c.adt; oa.m_pad = g.m_pad; oa.Sz = B;
  oa.js = 0; oa.ref = sb.scal + 0; oa.ref_from_gram = true;
  oa.kept1 = sb.ints + 0; oa.kept2 = sb.ints + 1;
  const int* nv = sb.ints + 1;
  const bool last_is_core = g.literal;  // the printed truncation keeps the final basis itself
  for (int it = 0; it <= g.iters; ++it) {
    if (it > 0) {
      sa.Z = zs; sa.y = yall; sa.ldy = b;
      if (!g.two_pass) {
        TTR_CHECK(launch_fused(sa));
      } else {
        TTR_CHECK(launch_atz(sa, wbuf, c.adt, B, B, 0));
        sa.W = wbuf;
        TTR_CHECK(launch_aw(sa));
      }
    }
    const bool last = it == g.iters;
    oa.Qout = (last && last_is_core) ? c.core : qbuf;
    oa.ldqo = b;
    TTR_CHECK(orth_update(oa, it == 0 ? pbuf : yall, b, nullptr, false));
    TTR_CHECK(orth_tgram(oa));
    TTR_CHECK(orth_out(oa));
  }
  if (!last_is_core) {
    // Rayleigh-Ritz on span(Q): M = Q^T A A^T Q, top-r eigenvectors, G = Q U
    sa.Z = zs; sa.y = yall; sa.ldy = b;
    if (!g.two_pass) {
      TTR_CHECK(launch_fused(sa));
    } else {
      TTR_CHECK(launch_atz(sa, wbuf, c.adt, B, B, 0));
      sa.W = wbuf;
      TTR_CHECK(launch_aw(sa));
    }
    TTR_CHECK(gemm_tn_sym(m, b, qbuf, b, yall, b, sb.gram, b, sb.splitk, c.st));
    TTR_CHECK(sym_eig_top(sb.gram, b, g.r, sb.vecs, sb.vals, sb.eigw, c.st));
    int* nvr = sb.ints + 1020;
    TTR_CHECK(gemm_nn_ritz(m, b, g.r, qbuf, b, sb.vecs, sb.vals, c.core, g.r, nvr, c.st));
    nv = nvr;
  }
  TTR_CHECK(complete_columns(c.core, m, g.r, nv, ybuf, c.st));
  return carry_pass(c);
}

static int run_saturated(const ModeCtx& c) {
  const ModeGeom& g = *c.g;
  const SmallBufs& sb = c.sb;
  int* nv = c.tape ? c.tape->ints + c.q + 1 : sb.ints + 1020;
  double* evec = c.tape ? c.tape->U : sb.vecs;
  double* eval = c.tape ? c.tape->lam : sb.vals;
  double* pbuf = reinterpret_cast<double*>(c.ws + c.lay->pbuf);
  double* ybuf = reinterpret_cast<double*>(c.ws + c.lay->ybuf);
  if (g.m <= g.n) {
    // Exact truncated SVD through the m x m Gram A A^T.
    StreamArgs sa;
    sa.A = c.A; sa.dtype = c.adt; sa.m = g.m; sa.n = g.n; sa.m_pad = g.m_pad;
    sa.part = c.ws + c.lay->partials; sa.part_bytes = c.lay->partials_bytes; sa.stream = c.st;
    TTR_CHECK(launch_gram(sa, sb.gram));
    TTR_CHECK(flag_nonfinite(sb.gram, g.m * g.m, c.status, c.st));  // A A^T sees every entry of A
    TTR_CHECK(eigen(c, sb.gram, (int)g.m, g.r, evec, eval));
    TTR_CHECK(sat_select(evec, eval, (int)g.m, g.r, c.tau, c.core, nv, c.st));
    TTR_CHECK(complete_columns(c.core, g.m, g.r, nv, ybuf, c.st));
    return carry_pass(c);
  }
  // n < m: right singular vectors from the n x n Gram A^T A, then G = orth(A V_r).
  const int n = (int)g.n;
  TTR_CHECK(gemm_tn(g.m, n, n, c.A, c.adt, n, c.A, c.adt, n, 1.0, 0.0, sb.gram, TTR_F64, n, sb.splitk, c.st));
  TTR_CHECK(flag_nonfinite(sb.gram, (int64_t)n * n, c.status, c.st));  // A^T A sees every entry of A
  TTR_CHECK(eigen(c, sb.gram, n, g.r, evec, eval));
  TTR_CHECK(gemm_nn(g.m, n, g.r, c.A, c.adt, n, evec, n, 1.0, 0.0, pbuf, g.r, c.st));
  int rc = orth_block(pbuf, pbuf, g.m, g.r, sb.scal + 400, c.tau * c.tau, c.core, g.r, ybuf, sb.ints + 1021, nv, sb, c.st,
                      c.tape ? c.tape->T : nullptr, true);
  if (rc) return rc;
  TTR_CHECK(complete_columns(c.core, g.m, g.r, nv, ybuf, c.st));
  TTR_CHECK(gemm_tn(g.m, g.r, n, c.core, TTR_F64, g.r, c.A, c.adt, n, 1.0, 0.0, c.carry, c.cdt, n, sb.splitk, c.st));
  return TTR_OK;
}

static int check_ptr_align(const void* p, const char* what) {
  if ((reinterpret_cast<uintptr_t>(p) & 255) != 0) {
    set_error(std::string(what) + " must be 256-byte aligned");
    return TTR_EINVAL;
  }
  return TTR_OK;
}

int sweep(const void* x, const Plan& pl, uint64_t seed, double* const* cores, char* ws, hipStream_t st,
          const ModeTape* tapes) {
  const ttr_plan_t& P = pl.pub;
  const int d = P.d;
  SmallBufs sb = carve_small(ws + pl.lay.small, pl.lay.small_bytes, pl.lay.small_ne);
  if (pl.lay.orth_big_bytes) {
    // kOrthBigGroups partials of the longest step, then the groups' norms, then the s x s sum
    const size_t gsum_bytes = (size_t)64 * 64 * 8, norm_bytes = (size_t)kOrthBigGroups * 8;
    sb.big_part = reinterpret_cast<double*>(ws + pl.lay.orth_big);
    sb.big_part_bytes = pl.lay.orth_big_bytes - gsum_bytes - norm_bytes;
    sb.big_norm = sb.big_part + sb.big_part_bytes / 8;
    sb.big_gsum = sb.big_norm + kOrthBigGroups;
  }
  int* status = reinterpret_cast<int*>(ws + kStatusOffset);
  TTR_CHECK(orth_reset_counter(sb.counter, st));
  TTR_CHECK(orth_reset_counter(status, st));
  const void* A = x;
  int adt = P.x_dtype;
  int ping = 0;
  bool next_ready = false;  // this mode's Y0 was formed by the previous carry pass
  for (int k = 1; k < d; ++k) {
    const ModeGeom& g = pl.modes[k - 1];
    ModeCtx c;
    bool fused = false;
    c.next = k + 1 < d ? &pl.modes[k] : nullptr;
    c.sketch_ready = next_ready;
    c.fused_next = &fused;
    next_ready = false;
    c.tape = tapes ? &tapes[k - 1] : nullptr;
    c.A = A; c.adt = adt; c.g = &g; c.q = P.q; c.seed = seed; c.tau = g.tau;
    c.core = cores[k - 1]; c.cdt = P.carry_dtype; c.ws = ws; c.lay = &pl.lay; c.sb = sb; c.st = st;
    c.status = status;
    c.carry = c.tape ? c.tape->carry : ws + pl.lay.carry[ping];
    int rc = TTR_OK;
    if (g.kind == TTR_MODE_IDENTITY) {
      TTR_CHECK(identity(c.core, g.m, st));
      continue;  // the carry is A itself: same memory, same dtype
    } else if (g.kind == TTR_MODE_SATURATED) {
      rc = run_saturated(c);
    } else {
      rc = (g.method == TTR_METHOD_RBKI && !g.literal) ? run_regular(c) : run_power(c);
    }
    if (rc) return rc;
    next_ready = fused;
    A = c.carry;
    adt = P.carry_dtype;
    ping ^= 1;
  }
  // Last core (Algorithm 3, step 12): the final carry, r_{d-1} x I_d, in float64.
  const int64_t rl = P.ranks[d - 1], Id = P.dims[d - 1];
  TTR_CHECK(convert_pad(A, adt, rl * Id, 1, 1, cores[d - 1], TTR_F64, rl * Id, 1, 1, st));
  // non-finite values created anywhere in the sweep reach the last core through the carries
  TTR_CHECK(flag_nonfinite(cores[d - 1], rl * Id, status, st));
  return TTR_OK;
}

// Streaming reconstruction error (Section 4 metrics): out3 <- (||X - Xhat||^2, ||X||^2,
// ||Xhat||_inf) for float64 cores (host array of device pointers).  The trailing cores
// are contracted into R (r_s x prod_{k>s} I_k), then every slab of the leading indices is
// formed on chip against R and X; partial sums are reduced in a fixed order.
hipError_t tt_error_run(const void* x, int x_dtype, int d, const int64_t* dims, const int64_t* ranks,
                        const double* const* cores, double* out3, char* ws, hipStream_t st) {
  int64_t inner = 0;
  const int s = error_split(d, dims, &inner);
  int64_t rmax = 1;
  for (int k = s; k <= d; ++k) rmax = std::max(rmax, ranks[k]);
  int64_t outer = 1;
  for (int k = 0; k < s; ++k) outer *= dims[k];
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  double* buf[2] = {reinterpret_cast<double*>(ws), reinterpret_cast<double*>(ws + al((size_t)rmax * inner * 8))};
  double* part = reinterpret_cast<double*>(ws + 2 * al((size_t)rmax * inner * 8));
  // R_{d} = core_d (r_{d-1} x I_d); R_k = G_k (r_{k-1} I_k x r_k) R_{k+1} (r_k x rest)
  const double* R = cores[d - 1];
  int64_t rest = dims[d - 1];
  int which = 0;
  for (int k = d - 2; k >= s; --k) {
    double* out = buf[which];
    hipError_t e = gemm_nn(ranks[k] * dims[k], (int)ranks[k + 1], (int)rest, cores[k], TTR_F64, ranks[k + 1], R,
                           rest, 1.0, 0.0, out, rest, st);
    if (e != hipSuccess) return e;
    rest *= dims[k];
    R = out;
    which ^= 1;
  }
  return tt_error_blocks(x, x_dtype, outer, inner, s, dims, ranks, cores, R, part, out3, st);
}

}  // namespace ttr

using namespace ttr;

// ---- allocation-free sweep: scratch in a file-scope device array ---------------------
// Every GPU that runs ttr_rbki_noalloc holds its own copy of `scratch` (loaded with the
// module, kept until the process ends).  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in): the device address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch_ptr.
static_assert(TTR_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[TTR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up on the first call there.
int static_scratch(void** out, bool lookup) {
  int dev = 0;
  TTR_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) { set_error("device index above 63"); return TTR_EINVAL; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev] && lookup) {
    void* ptr = nullptr;
    TTR_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TTR_OK;
}
}  // namespace

extern "C" {

int ttr_rbki(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims, const int64_t* target_ranks, int32_t q,
             int32_t p, uint64_t seed, const ttr_options* opt, double* const* cores, void* workspace,
             size_t workspace_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(d, dims, target_ranks, q, p, x_dtype, opt, &pl);
  if (rc) return rc;
  if (!x || !cores) { set_error("null tensor or core array"); return TTR_EINVAL; }
  for (int k = 0; k < d; ++k)
    if (!cores[k]) { set_error("null core pointer"); return TTR_EINVAL; }
  if (workspace_bytes < pl.pub.workspace_bytes || !workspace) {
    set_error("workspace needs " + std::to_string(pl.pub.workspace_bytes) + " bytes");
    return TTR_EWORKSPACE;
  }
  if ((rc = check_ptr_align(workspace, "workspace"))) return rc;
  return sweep(x, pl, seed, cores, static_cast<char*>(workspace), static_cast<hipStream_t>(stream), nullptr);
}

int ttr_rbki_noalloc(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims, const int64_t* target_ranks,
                     int32_t q, int32_t p, uint64_t seed, const ttr_options* opt, double* const* cores, void* stream) {
  Plan pl;
  int rc = make_plan(d, dims, target_ranks, q, p, x_dtype, opt, &pl);
  if (rc) return rc;
  if (!x || !cores) { set_error("null tensor or core array"); return TTR_EINVAL; }
  for (int k = 0; k < d; ++k)
    if (!cores[k]) { set_error("null core pointer"); return TTR_EINVAL; }
  if (pl.pub.workspace_bytes > TTR_NOALLOC_SCRATCH_BYTES) {
    set_error("the sweep needs " + std::to_string(pl.pub.workspace_bytes) + " bytes of scratch; the static scratch holds " +
              std::to_string((size_t)TTR_NOALLOC_SCRATCH_BYTES));
    return TTR_EWORKSPACE;
  }
  void* ws = nullptr;
  if ((rc = static_scratch(&ws, true))) return rc;
  return sweep(x, pl, seed, cores, static_cast<char*>(ws), static_cast<hipStream_t>(stream), nullptr);
}

int ttr_check(const void* workspace, void* stream) {
  if (!workspace) {  // the allocation-free entry's scratch on the current device
    void* ws = nullptr;
    int rc = static_scratch(&ws, false);
    if (rc) return rc;
    if (!ws) { set_error("null workspace and no allocation-free call on this device"); return TTR_EINVAL; }
    workspace = ws;
  }
  int flag = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TTR_CHECK(hipMemcpyAsync(&flag, static_cast<const char*>(workspace) + kStatusOffset, sizeof(int),
                           hipMemcpyDeviceToHost, st));
  TTR_CHECK(hipStreamSynchronize(st));
  if (flag) { set_error("non-finite values in the input or the results of the last call"); return TTR_ENUMERIC; }
  return TTR_OK;
}

size_t ttr_sym_eig_workspace(int32_t n) {
  if (n <= 0 || n > kMaxSmall) return 0;
  return std::max<size_t>(256, eig_work_doubles(n) * sizeof(double));
}

static int eig_args(const double* a, int32_t n, double* vecs, double* vals, void* workspace, size_t workspace_bytes) {
  if (!a || !vecs || !vals) { set_error("null pointer"); return TTR_EINVAL; }
  if (n <= 0 || n > kMaxSmall) { set_error("the eigen entries take 1 <= n <= 256"); return TTR_EINVAL; }
  if (eig_work_doubles(n) > 0 && (!workspace || workspace_bytes < ttr_sym_eig_workspace(n))) {
    set_error("workspace needs " + std::to_string(ttr_sym_eig_workspace(n)) + " bytes");
    return TTR_EWORKSPACE;
  }
  return TTR_OK;
}

int ttr_sym_eig(const double* a, int32_t n, double* vecs, double* vals, void* workspace, size_t workspace_bytes,
                void* stream) {
  int rc = eig_args(a, n, vecs, vals, workspace, workspace_bytes);
  if (rc) return rc;
  TTR_CHECK(sym_eig(a, n, vecs, vals, static_cast<double*>(workspace), static_cast<hipStream_t>(stream)));
  return TTR_OK;
}

int ttr_sym_eig_top(const double* a, int32_t n, int32_t r, double* vecs, double* vals, void* workspace,
                    size_t workspace_bytes, void* stream) {
  int rc = eig_args(a, n, vecs, vals, workspace, workspace_bytes);
  if (rc) return rc;
  if (r <= 0 || r > n || r > 64) { set_error("ttr_sym_eig_top takes 1 <= r <= min(n, 64)"); return TTR_EINVAL; }
  TTR_CHECK(sym_eig_top(a, n, r, vecs, vals, static_cast<double*>(workspace), static_cast<hipStream_t>(stream)));
  return TTR_OK;
}

int ttr_omega(uint64_t seed, int32_t k, int64_t beta0, int64_t nrows, int32_t s, double* out, void* stream) {
  if (!out || k < 1 || beta0 < 0 || nrows < 0 || s <= 0) { set_error("bad omega arguments"); return TTR_EINVAL; }
  if (nrows == 0) return TTR_OK;
  TTR_CHECK(launch_omega(seed, k, beta0, nrows, s, s, out, TTR_F64, static_cast<hipStream_t>(stream)));
  return TTR_OK;
}

// ---- building blocks ------------------------------------------------------------
struct BlockWs {
  char* wbuf;
  char* part;
  size_t part_bytes;
  char* zs;
};

static int block_setup(const void* a, int32_t dt, int64_t m, int64_t n, int cols, void* ws, size_t bytes,
                       BlockWs* b) {
  if (!a || !ws) { set_error("null pointer"); return TTR_EINVAL; }
  if (dt != TTR_F64 && dt != TTR_F32 && dt != TTR_BF16) { set_error("unknown dtype"); return TTR_EINVAL; }
  if (m <= 0 || n <= 0 || cols <= 0 || cols > 64) { set_error("bad block shape"); return TTR_EINVAL; }
  if (m > 65536) { set_error("block rows above 65536"); return TTR_EUNSUPPORTED; }
  const size_t need = block_workspace(m, n, cols, dt);
  if (bytes < need) { set_error("workspace needs " + std::to_string(need) + " bytes"); return TTR_EWORKSPACE; }
  int rc = check_ptr_align(ws, "workspace");
  if (rc) return rc;
  const int S = pad16(cols);
  const int64_t m_pad = pad_rows(m, dt);
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  b->wbuf = base + off; off = al(off + (size_t)n * S * dtype_bytes(dt));
  b->part_bytes = stream_partial_bytes(n, m_pad, S, dt, m_pad <= kGramBigM);
  if (m_pad <= kGramBigM) b->part_bytes = std::max(b->part_bytes, gram_sketch_partial_bytes(n, m_pad, S, dt));
  b->part = base + off; off = al(off + b->part_bytes);
  b->zs = base + off;
  return TTR_OK;
}

int ttr_sketch(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k, int32_t s, double* y,
               void* workspace, size_t workspace_bytes, void* stream) {
  BlockWs b;
  int rc = block_setup(a, a_dtype, m, n, s, workspace, workspace_bytes, &b);
  if (rc) return rc;
  if (!y || k < 1) { set_error("bad sketch arguments"); return TTR_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  StreamArgs sa;
  sa.A = a; sa.dtype = a_dtype; sa.m = m; sa.n = n; sa.m_pad = pad_rows(m, a_dtype);
  sa.S = pad16(s); sa.s = s; sa.part = b.part; sa.part_bytes = b.part_bytes; sa.W = b.wbuf; sa.y = y; sa.ldy = s; sa.stream = st;
  TTR_CHECK(sketch_pass(sa, seed, k, sa.S, b.wbuf));
  return TTR_OK;
}

static int krylov_impl(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* z, int32_t s, double* y,
                       int32_t force_two_pass, void* workspace, size_t workspace_bytes, void* stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end, int reps) {
  BlockWs b;
  int rc = block_setup(a, a_dtype, m, n, s, workspace, workspace_bytes, &b);
  if (rc) return rc;
  if (!z || !y) { set_error("null pointer"); return TTR_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  StreamArgs sa;
  sa.A = a; sa.dtype = a_dtype; sa.m = m; sa.n = n; sa.m_pad = pad_rows(m, a_dtype);
  sa.S = pad16(s); sa.s = s; sa.part = b.part; sa.part_bytes = b.part_bytes; sa.Z = b.zs; sa.y = y; sa.ldy = s; sa.stream = st;
  const bool fused = !force_two_pass && fused_fits(sa.m_pad, sa.S, a_dtype);
  if ((ev_begin || ev_end) && !(fused && ev_begin && ev_end)) {
    set_error("timing events need both handles and the one-pass fused product");
    return TTR_EINVAL;
  }
  sa.ev_begin = ev_begin; sa.ev_end = ev_end; sa.reps = reps;
  TTR_CHECK(convert_pad(z, TTR_F64, m, s, s, b.zs, a_dtype, sa.m_pad, sa.S, sa.S, st));
  if (fused) {
    TTR_CHECK(launch_fused(sa));
  } else {
    TTR_CHECK(launch_atz(sa, b.wbuf, a_dtype, sa.S, sa.S, 0));
    sa.W = b.wbuf;
    TTR_CHECK(launch_aw(sa));
  }
  return TTR_OK;
}

int ttr_krylov(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* z, int32_t s, double* y,
               int32_t force_two_pass, void* workspace, size_t workspace_bytes, void* stream) {
  return krylov_impl(a, a_dtype, m, n, z, s, y, force_two_pass, workspace, workspace_bytes, stream, nullptr,
                     nullptr, 1);
}

int ttr_krylov_timed(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* z, int32_t s, double* y,
                     int32_t reps, void* workspace, size_t workspace_bytes, void* ev_begin, void* ev_end,
                     void* stream) {
  if (!ev_begin || !ev_end) { set_error("null event"); return TTR_EINVAL; }
  if (reps < 1 || reps > 1000) { set_error("reps must be in [1, 1000]"); return TTR_EINVAL; }
  return krylov_impl(a, a_dtype, m, n, z, s, y, 0, workspace, workspace_bytes, stream,
                     static_cast<hipEvent_t>(ev_begin), static_cast<hipEvent_t>(ev_end), reps);
}

int ttr_carry(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* g, int32_t s, void* c,
              int32_t c_dtype, void* workspace, size_t workspace_bytes, void* stream) {
  BlockWs b;
  int rc = block_setup(a, a_dtype, m, n, s, workspace, workspace_bytes, &b);
  if (rc) return rc;
  if (!g || !c) { set_error("null pointer"); return TTR_EINVAL; }
  const int want = a_dtype == TTR_F64 ? TTR_F64 : TTR_F32;
  if (c_dtype != want) { set_error("carry dtype must be f64 for f64 input, else f32"); return TTR_EINVAL; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  StreamArgs sa;
  sa.A = a; sa.dtype = a_dtype; sa.m = m; sa.n = n; sa.m_pad = pad_rows(m, a_dtype);
  sa.S = pad16(s); sa.s = s; sa.part = b.part; sa.part_bytes = b.part_bytes; sa.Z = b.zs; sa.stream = st;
  TTR_CHECK(convert_pad(g, TTR_F64, m, s, s, b.zs, a_dtype, sa.m_pad, sa.S, sa.S, st));
  TTR_CHECK(launch_atz(sa, c, c_dtype, n, s, 1));
  return TTR_OK;
}

size_t ttr_orth_workspace(int64_t m, int32_t s) {
  if (m <= 0 || s <= 0 || s > 64) return 0;
  const size_t sq = (size_t)s * s * 8, ms = ((size_t)m * s * 8 + 255) / 256 * 256;
  return 256 + 3 * ((sq + 255) / 256 * 256) + (15 * sq + 255) / 256 * 256 + 2 * ms + 256;
}

int ttr_orth(const double* p, int64_t m, int32_t s, double ref_norm, double tau, double* q, int32_t* kept,
             void* workspace, size_t workspace_bytes, void* stream) {
  if (!p || !q || !kept || !workspace) { set_error("null pointer"); return TTR_EINVAL; }
  if (m <= 0 || s <= 0 || s > 64 || !(tau >= 0.0) || !(ref_norm >= 0.0)) {
    set_error("ttr_orth takes m > 0, 1 <= s <= 64, tau >= 0, ref_norm >= 0");
    return TTR_EINVAL;
  }
  if (workspace_bytes < ttr_orth_workspace(m, s)) {
    set_error("workspace needs " + std::to_string(ttr_orth_workspace(m, s)) + " bytes");
    return TTR_EWORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t sq = (size_t)s * s * 8, sqa = (sq + 255) / 256 * 256;
  char* w = static_cast<char*>(workspace);
  double* ref = reinterpret_cast<double*>(w);
  SmallBufs sb{};
  sb.gram = reinterpret_cast<double*>(w + 256);
  sb.tmat = reinterpret_cast<double*>(w + 256 + sqa);
  sb.hmat = reinterpret_cast<double*>(w + 256 + 2 * sqa);
  sb.splitk = reinterpret_cast<double*>(w + 256 + 3 * sqa);
  sb.splitk_bytes = 15 * sq;
  char* tail = w + 256 + 3 * sqa + (15 * sq + 255) / 256 * 256;
  double* tmp = reinterpret_cast<double*>(tail);
  double* pw = reinterpret_cast<double*>(tail + ((size_t)m * s * 8 + 255) / 256 * 256);
  int* k1 = reinterpret_cast<int*>(pw + (size_t)m * s);
  sb.counter = k1 + 16;
  sb.vecs = sb.gram;  // projection buffers are unused without a previous basis
  TTR_CHECK(set_scalar(ref, ref_norm * ref_norm, st));
  TTR_CHECK(orth_reset_counter(sb.counter, st));
  return orth_block(p, pw, m, s, ref, tau * tau, q, s, tmp, k1, kept, sb, st);
}

int ttr_gram(const void* a, int32_t a_dtype, int64_t m, int64_t n, double* gm, void* workspace,
             size_t workspace_bytes, void* stream) {
  BlockWs b;
  int rc = block_setup(a, a_dtype, m, n, 1, workspace, workspace_bytes, &b);
  if (rc) return rc;
  if (!gm) { set_error("null pointer"); return TTR_EINVAL; }
  if (pad_rows(m, a_dtype) > kGramBigM) { set_error("ttr_gram needs m <= 256"); return TTR_EUNSUPPORTED; }
  StreamArgs sa;
  sa.A = a; sa.dtype = a_dtype; sa.m = m; sa.n = n; sa.m_pad = pad_rows(m, a_dtype);
  sa.part = b.part; sa.part_bytes = b.part_bytes; sa.stream = static_cast<hipStream_t>(stream);
  TTR_CHECK(launch_gram(sa, gm));
  return TTR_OK;
}

static int gram_sketch_impl(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k,
                            int32_t s, double* gm, double* y, void* workspace, size_t workspace_bytes, void* stream,
                            hipEvent_t ev_begin, hipEvent_t ev_end, int reps) {
  BlockWs b;
  int rc = block_setup(a, a_dtype, m, n, s, workspace, workspace_bytes, &b);
  if (rc) return rc;
  if (!gm || !y || k < 1) { set_error("bad gram_sketch arguments"); return TTR_EINVAL; }
  if (pad_rows(m, a_dtype) > kGramBigM) { set_error("ttr_gram_sketch needs m <= 256"); return TTR_EUNSUPPORTED; }
  StreamArgs sa;
  sa.A = a; sa.dtype = a_dtype; sa.m = m; sa.n = n; sa.m_pad = pad_rows(m, a_dtype);
  sa.S = pad16(s); sa.s = s; sa.part = b.part; sa.part_bytes = b.part_bytes; sa.y = y; sa.ldy = s;
  sa.seed = seed; sa.kmode = k; sa.stream = static_cast<hipStream_t>(stream);
  sa.ev_begin = ev_begin; sa.ev_end = ev_end; sa.reps = reps;
  TTR_CHECK(launch_gram_sketch(sa, gm));
  return TTR_OK;
}

int ttr_gram_sketch(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k, int32_t s,
                    double* gm, double* y, void* workspace, size_t workspace_bytes, void* stream) {
  return gram_sketch_impl(a, a_dtype, m, n, seed, k, s, gm, y, workspace, workspace_bytes, stream, nullptr, nullptr,
                          1);
}

int ttr_gram_sketch_timed(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k, int32_t s,
                          double* gm, double* y, int32_t reps, void* workspace, size_t workspace_bytes, void* ev_begin,
                          void* ev_end, void* stream) {
  if (!ev_begin || !ev_end) { set_error("null event"); return TTR_EINVAL; }
  if (reps < 1 || reps > 1000) { set_error("reps must be in [1, 1000]"); return TTR_EINVAL; }
  if (a_dtype != TTR_BF16) { set_error("the timed Gram-and-sketch kernel is the bfloat16 one"); return TTR_EUNSUPPORTED; }
  return gram_sketch_impl(a, a_dtype, m, n, seed, k, s, gm, y, workspace, workspace_bytes, stream,
                          static_cast<hipEvent_t>(ev_begin), static_cast<hipEvent_t>(ev_end), reps);
}

// ---- reconstruction error ---------------------------------------------------------
size_t ttr_tt_error_workspace(int32_t d, const int64_t* dims, const int64_t* ranks) {
  if (d < 2 || d > TTR_MAX_D || !dims || !ranks) return 0;
  return tt_error_ws_bytes(d, dims, ranks);
}

int ttr_tt_error(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims, const int64_t* ranks,
                 const double* const* cores, double* out3, void* workspace, size_t workspace_bytes, void* stream) {
  if (!x || !dims || !ranks || !cores || !out3 || !workspace) { set_error("null pointer"); return TTR_EINVAL; }
  if (d < 2 || d > TTR_MAX_D) { set_error("bad d"); return TTR_EINVAL; }
  if (x_dtype != TTR_F64 && x_dtype != TTR_F32 && x_dtype != TTR_BF16) { set_error("unknown dtype"); return TTR_EINVAL; }
  if (ranks[0] != 1 || ranks[d] != 1) { set_error("ranks[0] and ranks[d] must be 1"); return TTR_EINVAL; }
  for (int k = 0; k < d; ++k) {
    if (dims[k] <= 0 || !cores[k]) { set_error("bad dims or core"); return TTR_EINVAL; }
    if (ranks[k + 1] <= 0 || ranks[k + 1] > 64) { set_error("ranks must be in [1, 64]"); return TTR_EINVAL; }
  }
  const size_t need = tt_error_ws_bytes(d, dims, ranks);
  if (workspace_bytes < need) { set_error("workspace needs " + std::to_string(need) + " bytes"); return TTR_EWORKSPACE; }
  TTR_CHECK(tt_error_run(x, x_dtype, d, dims, ranks, cores, out3, static_cast<char*>(workspace),
                         static_cast<hipStream_t>(stream)));
  return TTR_OK;
}

}  // extern "C"
