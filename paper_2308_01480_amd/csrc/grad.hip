// Gradient of f(X) = ||X - TT_r(X)||_F^2 through the TT-RBKI sweep (Algorithm 3, the
// random matrices Omega_k held fixed).
//
// With left-orthonormal cores the TT approximation is an orthogonal projection of X,
// so f = ||X||^2 - ||C_{d-1}||^2, C_{d-1} the last carry.  The forward sweep keeps,
// per mode, the Krylov basis Q, the products A A^T Q, the block transforms T_j
// (Q_j = P_j T_j, T_j = E R_j^{-1}), the eigen-decomposition behind the truncation and
// every carry.  The reverse sweep starts from Cbar_{d-1} = -2 C_{d-1} and maps the
// adjoint of each carry C_k = G_k^T A_k to the adjoint of A_k (the previous carry):
//
//   Abar = (Kbar + Kbar^T) A + Ybar_0 Omega^T + G Cbar,      K = A A^T,
//
// where the small float64 steps contribute
//   Rayleigh-Ritz  G = Q U_r, U_r = top-r eigenvectors of M = Q^T K Q:
//       Gbar = A Cbar^T, Qbar += Gbar U_r^T, Ubar = Q^T Gbar, Mbar = eigenvector
//       adjoint (kept x discarded pairs), Kbar += Q Mbar Q^T, Qbar += 2 (K Q) Mbar;
//   block QR       Q_j = qr(P_j E):  Pbar = [Qbar + Q copyltu(-Qbar^T Q)] T^T;
//   projection     P_j = Y_j - Q_< Q_<^T Y_j:  Ybar = Pbar - Q_< Q_<^T Pbar,
//                  Qbar_< -= Pbar (Q_<^T Y_j)^T + Y_j (Q_<^T Pbar)^T;
//   Krylov step    Y_j = K Q_{j-1}:  Kbar += Ybar_j Q_{j-1}^T, Qbar_{j-1} += K Ybar_j;
//   sketch         Q_0 = qr(Y_0 E), Y_0 = A Omega.
// Saturated modes (the exact truncated SVD) use the eigenvector adjoint of A A^T
// (m <= n) or, for n < m, G = A V_r Lambda_r^{-1/2} with (V, Lambda) = eig(A^T A).
// Finally df/dX = 2 X + Abar_1.  Everything runs on the caller's stream; the large
// products go through the streaming kernels of the forward sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "driver.h"
#include "kernels.h"

namespace ttr {

#define TTR_GCHECK(expr)                                                       \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      (void)hipGetLastError();                                                 \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
      return TTR_EHIP;                                                         \
    }                                                                          \
  } while (0)

// W (n x R, zero beyond column r) <- Cbar^T, Cbar: r x n.  32 x 32 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_pad(const T* __restrict__ c, int r, int64_t n, int R,
                                                       T* __restrict__ w) {
  __shared__ T tile[32][33];
  const int64_t b0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int row = c0 + yy;
    const int64_t col = b0 + tx;
    tile[yy][tx] = (row < r && col < n) ? c[(int64_t)row * n + col] : (T)0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t row = b0 + yy;
    const int col = c0 + tx;
    if (row < n && col < R) w[row * R + col] = tile[tx][yy];
  }
}

// Abar (m x n) += [Ybar0 | G] (m x (s + r)) [Omega^T ; Cbar] ((s + r) x n).
// A work-group owns 32 rows x 256 columns; the 32 x (s + r) float64 coefficients sit
// in LDS (s + r <= 128) and each lane accumulates its column for the 32 rows in registers.
template <typename T>
__global__ __launch_bounds__(256) void k_rank_update(T* __restrict__ abar, int64_t m, int64_t n,
                                                     const double* __restrict__ y0b, int s,
                                                     const T* __restrict__ om, int S, const double* __restrict__ g,
                                                     int r, const T* __restrict__ cbar) {
  __shared__ double coef[32][128];
  const int64_t i0 = (int64_t)blockIdx.y * 32;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int kk = s + r;
  for (int e = threadIdx.x; e < 32 * kk; e += 256) {
    const int ii = e / kk, c = e % kk;
    const int64_t row = i0 + ii;
    double v = 0.0;
    if (row < m) v = c < s ? y0b[row * s + c] : g[row * r + (c - s)];
    coef[ii][c] = v;
  }
  __syncthreads();
  if (b >= n) return;
  double acc[32];
#pragma unroll
  for (int ii = 0; ii < 32; ++ii) acc[ii] = 0.0;
  for (int c = 0; c < kk; ++c) {
    const double v = c < s ? (double)om[b * S + c] : (double)cbar[(int64_t)(c - s) * n + b];
#pragma unroll
    for (int ii = 0; ii < 32; ++ii) acc[ii] += coef[ii][c] * v;
  }
#pragma unroll
  for (int ii = 0; ii < 32; ++ii) {
    const int64_t row = i0 + ii;
    if (row < m) abar[row * n + b] = (T)((double)abar[row * n + b] + acc[ii]);
  }
}

// out = alpha * c (same dtype, element-wise).
template <typename T>
__global__ __launch_bounds__(256) void k_scale_copy(const T* __restrict__ c, T* __restrict__ out, int64_t n,
                                                    double alpha) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = (T)(alpha * (double)c[i]);
}

static hipError_t scale_copy(const void* c, void* out, int dt, int64_t n, double alpha, hipStream_t st) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  if (dt == TTR_F64)
    hipLaunchKernelGGL(k_scale_copy<double>, dim3(nb), dim3(256), 0, st, (const double*)c, (double*)out, n, alpha);
  else
    hipLaunchKernelGGL(k_scale_copy<float>, dim3(nb), dim3(256), 0, st, (const float*)c, (float*)out, n, alpha);
  return hipGetLastError();
}

struct GradCtx {
  const Plan* pl;
  char* ws;
  hipStream_t st;
  uint64_t seed;
  template <typename F>
  F* at(size_t off) const { return reinterpret_cast<F*>(ws + off); }
  double* d(size_t off) const { return at<double>(off); }
};

// Abar = Kt A for symmetric Kt (m x m float64), one 64-row band at a time through the
// A^T Z kernel: rows b0.. of Kt A are (A^T Kt[:, band])^T, written in carry layout.
static int apply_sym(const GradCtx& c, const void* A, int dt, int64_t m, int64_t n, const double* Kt, void* abar) {
  const GradLayout& G = c.pl->glay;
  const int64_t m_pad = pad_rows(m, dt);
  void* zs = c.ws + G.ktildt;
  for (int64_t b0 = 0; b0 < m; b0 += 64) {
    const int bw = (int)std::min<int64_t>(64, m - b0);
    const int S = pad16(bw);
    TTR_GCHECK(convert_pad(Kt + b0, TTR_F64, m, bw, m, zs, dt, m_pad, S, S, c.st));
    StreamArgs sa;
    sa.A = A; sa.dtype = dt; sa.m = m; sa.n = n; sa.m_pad = m_pad; sa.Z = zs; sa.S = S; sa.s = bw; sa.stream = c.st;
    TTR_GCHECK(launch_atz(sa, static_cast<char*>(abar) + (size_t)b0 * n * dtype_bytes(dt), dt, n, bw, 1));
  }
  return TTR_OK;
}

// Gbar (m x r float64) = A Cbar^T through the A W kernel (Cbar transposed to n x R).
static int a_cbar_t(const GradCtx& c, const void* A, int dt, int64_t m, int64_t n, const void* cbar, int r,
                    double* gbar) {
  const GradLayout& G = c.pl->glay;
  const int R = pad16(r);
  void* wt = c.ws + G.wt;
  const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((R + 31) / 32));
  if (dt == TTR_F64)
    hipLaunchKernelGGL(k_transpose_pad<double>, grid, dim3(256), 0, c.st, (const double*)cbar, r, n, R, (double*)wt);
  else
    hipLaunchKernelGGL(k_transpose_pad<float>, grid, dim3(256), 0, c.st, (const float*)cbar, r, n, R, (float*)wt);
  TTR_GCHECK(hipGetLastError());
  StreamArgs sa;
  sa.A = A; sa.dtype = dt; sa.m = m; sa.n = n; sa.m_pad = pad_rows(m, dt); sa.W = wt; sa.S = R; sa.s = r;
  sa.part = c.ws + G.gpart; sa.part_bytes = G.gpart_bytes; sa.y = gbar; sa.ldy = r; sa.stream = c.st;
  TTR_GCHECK(launch_aw(sa));
  return TTR_OK;
}

// out (m x s float64) = K y = A (A^T y), the forward sweep's Krylov product.
static int krylov_apply(const GradCtx& c, const void* A, int dt, const ModeGeom& g, const double* y, double* out) {
  const Layout& L = c.pl->lay;
  StreamArgs sa;
  sa.A = A; sa.dtype = dt; sa.m = g.m; sa.n = g.n; sa.m_pad = g.m_pad; sa.S = g.S; sa.s = g.s;
  sa.part = c.ws + L.partials; sa.part_bytes = L.partials_bytes; sa.Z = c.ws + L.zs; sa.y = out; sa.ldy = g.s; sa.stream = c.st;
  TTR_GCHECK(convert_pad(y, TTR_F64, g.m, g.s, g.s, c.ws + L.zs, dt, g.m_pad, g.S, g.S, c.st));
  if (!g.two_pass) {
    TTR_GCHECK(launch_fused(sa));
  } else {
    TTR_GCHECK(launch_atz(sa, c.ws + L.wbuf, dt, g.S, g.S, 0));
    sa.W = c.ws + L.wbuf;
    TTR_GCHECK(launch_aw(sa));
  }
  return TTR_OK;
}

// Adjoint of Q = P T (T = E R^{-1}, the kept columns of a column-pivoted QR):
// Pbar (m x s) = [Zb + Q copyltu(-Zb^T Q)] T^T, Zb = Qbar with the dropped columns zeroed.
static int qr_adjoint(const GradCtx& c, int64_t m, int s, const double* Q, int64_t ldq, const double* Qb,
                      int64_t ldqb, const double* T, const int* kept, double* pbar) {
  const GradLayout& G = c.pl->glay;
  double* zb = c.d(G.zb);
  double* cl = c.d(G.cl);
  double* mq = c.d(G.mq);
  TTR_GCHECK(axpby(m, s, 1.0, Qb, ldqb, 0.0, zb, s, kept, c.st));
  TTR_GCHECK(gemm_tn(m, s, s, zb, TTR_F64, s, Q, TTR_F64, ldq, 1.0, 0.0, mq, TTR_F64, s, c.d(G.splitk), c.st));
  TTR_GCHECK(copyltu(mq, s, -1.0, cl, c.st));
  TTR_GCHECK(gemm_nn(m, s, s, Q, TTR_F64, ldq, cl, s, 1.0, 1.0, zb, s, c.st));
  TTR_GCHECK(gemm_nt(m, s, s, zb, s, T, s, 1.0, 0.0, pbar, s, c.st));
  return TTR_OK;
}

static hipError_t rank_update(void* abar, int dt, int64_t m, int64_t n, const double* y0b, int s, const void* om,
                              int S, const double* g, int r, const void* cbar, hipStream_t st) {
  if (s + r > 128) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((m + 31) / 32));
  if (dt == TTR_F64)
    hipLaunchKernelGGL(k_rank_update<double>, grid, dim3(256), 0, st, (double*)abar, m, n, y0b, s, (const double*)om,
                       S, g, r, (const double*)cbar);
  else
    hipLaunchKernelGGL(k_rank_update<float>, grid, dim3(256), 0, st, (float*)abar, m, n, y0b, s, (const float*)om, S,
                       g, r, (const float*)cbar);
  return hipGetLastError();
}

static int backward_regular(const GradCtx& c, const ModeGeom& g, const ModeTape& tp, const double* core,
                            const void* A, int dt, const void* cbar, void* abar) {
  const GradLayout& G = c.pl->glay;
  const int64_t m = g.m;
  const int s = g.s, w = g.w, r = g.r, q = c.pl->pub.q;
  double* gb = c.d(G.gb);
  double* ub = c.d(G.ub);
  double* qb = c.d(G.qb);
  double* mb = c.d(G.mb);
  double* vv = c.d(G.vv);
  double* qmb = c.d(G.qmb);
  double* kbar = c.d(G.kbar);
  double* ktil = c.d(G.ktil);
  double* pb = c.d(G.pb);
  double* hh = c.d(G.hh);
  double* qtpb = c.d(G.qtpb);
  double* yb = c.d(G.yb);
  double* ktmp = c.d(G.ktmp);
  double* sk = c.d(G.splitk);

  int rc = a_cbar_t(c, A, dt, m, g.n, cbar, r, gb);
  if (rc) return rc;
  // Rayleigh-Ritz: U_r is the first r columns of the w x w eigenvector matrix.
  TTR_GCHECK(gemm_tn(m, w, r, tp.Q, TTR_F64, w, gb, TTR_F64, r, 1.0, 0.0, ub, TTR_F64, r, sk, c.st));
  TTR_GCHECK(gemm_nt(m, w, r, gb, r, tp.U, w, 1.0, 0.0, qb, w, c.st));
  TTR_GCHECK(eig_adjoint(tp.U, tp.lam, w, r, ub, tp.ints + q + 1, vv, mb, c.st));
  TTR_GCHECK(gemm_nn(m, w, w, tp.Q, TTR_F64, w, mb, w, 1.0, 0.0, qmb, w, c.st));
  TTR_GCHECK(gemm_nt(m, m, w, qmb, w, tp.Q, w, 1.0, 0.0, kbar, m, c.st));
  TTR_GCHECK(gemm_nn(m, w, w, tp.Yall, TTR_F64, w, mb, w, 2.0, 1.0, qb, w, c.st));
  // Krylov blocks, last first: Qbar_j is complete once every later block is done.
  for (int j = q; j >= 1; --j) {
    rc = qr_adjoint(c, m, s, tp.Q + j * s, w, qb + j * s, w, tp.T + (size_t)j * s * s, tp.ints + j, pb);
    if (rc) return rc;
    const double* Yj = tp.Yall + (j - 1) * s;
    const int js = j * s;
    TTR_GCHECK(gemm_tn(m, js, s, tp.Q, TTR_F64, w, Yj, TTR_F64, w, 1.0, 0.0, hh, TTR_F64, s, sk, c.st));
    TTR_GCHECK(gemm_tn(m, js, s, tp.Q, TTR_F64, w, pb, TTR_F64, s, 1.0, 0.0, qtpb, TTR_F64, s, sk, c.st));
    TTR_GCHECK(axpby(m, s, 1.0, pb, s, 0.0, yb, s, nullptr, c.st));
    TTR_GCHECK(gemm_nn(m, js, s, tp.Q, TTR_F64, w, qtpb, s, -1.0, 1.0, yb, s, c.st));
    TTR_GCHECK(gemm_nt(m, js, s, pb, s, hh, s, -1.0, 1.0, qb, w, c.st));
    TTR_GCHECK(gemm_nt(m, js, s, Yj, w, qtpb, s, -1.0, 1.0, qb, w, c.st));
    TTR_GCHECK(gemm_nt(m, m, s, yb, s, tp.Q + (j - 1) * s, w, 1.0, 1.0, kbar, m, c.st));
    rc = krylov_apply(c, A, dt, g, yb, ktmp);
    if (rc) return rc;
    TTR_GCHECK(axpby(m, s, 1.0, ktmp, s, 1.0, qb + (j - 1) * s, w, nullptr, c.st));
  }
  // Sketch block: Ybar_0 from Q_0 = qr(Y_0 E).
  double* y0b = yb;
  rc = qr_adjoint(c, m, s, tp.Q, w, qb, w, tp.T, tp.ints + 0, y0b);
  if (rc) return rc;
  // Abar = (Kbar + Kbar^T) A + Ybar_0 Omega^T + G Cbar
  TTR_GCHECK(sym_sum(kbar, m, ktil, c.st));
  rc = apply_sym(c, A, dt, m, g.n, ktil, abar);
  if (rc) return rc;
  void* om = c.ws + c.pl->lay.wbuf;
  TTR_GCHECK(launch_omega(c.seed, g.k, 0, g.n, s, g.S, om, dt, c.st));
  TTR_GCHECK(rank_update(abar, dt, m, g.n, y0b, s, om, g.S, core, r, cbar, c.st));
  return TTR_OK;
}

static int backward_saturated(const GradCtx& c, const ModeGeom& g, const ModeTape& tp, const double* core,
                              const void* A, int dt, const void* cbar, void* abar) {
  const GradLayout& G = c.pl->glay;
  const int64_t m = g.m;
  const int r = g.r, q = c.pl->pub.q;
  double* gb = c.d(G.gb);
  double* mb = c.d(G.mb);
  double* vv = c.d(G.vv);
  double* ktil = c.d(G.ktil);
  double* sk = c.d(G.splitk);
  const int* nv = tp.ints + q + 1;
  int rc;
  if (m <= g.n) {
    // G = leading eigenvectors of K = A A^T: Kbar from the eigenvector adjoint.
    rc = a_cbar_t(c, A, dt, m, g.n, cbar, r, gb);
    if (rc) return rc;
    TTR_GCHECK(eig_adjoint(tp.U, tp.lam, (int)m, r, gb, nv, vv, mb, c.st));
    TTR_GCHECK(sym_sum(mb, m, ktil, c.st));
    rc = apply_sym(c, A, dt, m, g.n, ktil, abar);
    if (rc) return rc;
    TTR_GCHECK(rank_update(abar, dt, m, g.n, nullptr, 0, nullptr, 16, core, r, cbar, c.st));
    return TTR_OK;
  }
  // n < m: G = A W, W = V_r Lambda_r^{-1/2}, (V, Lambda) = eig(N), N = A^T A; n is small.
  const int n = (int)g.n;
  double* wmat = c.d(G.qmb);    // n x n, first r columns = W
  double* wb = c.d(G.wb);       // n x r
  double* lb = c.d(G.lb);       // r
  double* vb = c.d(G.ub);       // n x r
  double* nbs = c.d(G.symnb);   // n x n
  double* a64 = c.d(G.abtmp);   // m x n float64 copy of A
  double* c64 = c.d(G.cbar64);  // r x n float64 copy of Cbar
  double* acc = ktil;           // m x n float64 accumulator of Abar
  TTR_GCHECK(svqb_transform(tp.U, tp.lam, n, nullptr, 0.0, wmat, c.at<int>(G.ints), c.st));
  TTR_GCHECK(convert_pad(cbar, dt, r, n, n, c64, TTR_F64, r, n, n, c.st));
  TTR_GCHECK(convert_pad(A, dt, m, n, n, a64, TTR_F64, m, n, n, c.st));
  TTR_GCHECK(gemm_nt(m, r, n, a64, n, c64, n, 1.0, 0.0, gb, r, c.st));
  TTR_GCHECK(gemm_tn(m, n, r, a64, TTR_F64, n, gb, TTR_F64, r, 1.0, 0.0, wb, TTR_F64, r, sk, c.st));
  TTR_GCHECK(scale_adjoint(tp.U, n, r, tp.lam, wb, vb, lb, c.st));
  TTR_GCHECK(eig_adjoint(tp.U, tp.lam, n, r, vb, nv, vv, mb, c.st));
  TTR_GCHECK(add_eigval_adjoint(tp.U, n, r, lb, mb, c.st));
  TTR_GCHECK(sym_sum(mb, n, nbs, c.st));
  // Abar = Gbar W^T + G Cbar + A (Nbar + Nbar^T)
  TTR_GCHECK(gemm_nt(m, n, r, gb, r, wmat, n, 1.0, 0.0, acc, n, c.st));
  TTR_GCHECK(gemm_nn(m, r, n, core, TTR_F64, r, c64, n, 1.0, 1.0, acc, n, c.st));
  TTR_GCHECK(gemm_nn(m, n, n, a64, TTR_F64, n, nbs, n, 1.0, 1.0, acc, n, c.st));
  TTR_GCHECK(convert_pad(acc, TTR_F64, m, n, n, abar, dt, m, n, n, c.st));
  return TTR_OK;
}

// A_k of mode k (1-based): the carry of the closest earlier non-identity mode, else X.
static const void* mode_input(const Plan& pl, const ModeTape* tapes, const void* x, int k, int* dt) {
  for (int j = k - 1; j >= 1; --j)
    if (pl.modes[j - 1].kind != TTR_MODE_IDENTITY) { *dt = pl.pub.carry_dtype; return tapes[j - 1].carry; }
  *dt = pl.pub.x_dtype;
  return x;
}

static int grad_run(const void* x, const Plan& pl, uint64_t seed, void* dx, double* loss, char* ws, hipStream_t st) {
  const ttr_plan_t& P = pl.pub;
  const GradLayout& G = pl.glay;
  const int d = P.d;
  GradCtx c{&pl, ws, st, seed};
  ModeTape tapes[TTR_MAX_D];
  double* cores[TTR_MAX_D];
  for (int k = 1; k < d; ++k) {
    ModeTape& t = tapes[k - 1];
    t.Q = c.d(G.tQ[k - 1]);
    t.Yall = c.d(G.tY[k - 1]);
    t.T = c.d(G.tT[k - 1]);
    t.U = c.d(G.tU[k - 1]);
    t.lam = c.d(G.tL[k - 1]);
    t.ints = c.at<int>(G.tI[k - 1]);
    t.carry = ws + G.tC[k - 1];
  }
  for (int k = 1; k <= d; ++k) cores[k - 1] = c.d(G.cores[k - 1]);
  int rc = sweep(x, pl, seed, cores, ws, st, tapes);
  if (rc) return rc;

  int last_dt = 0;
  const void* last = mode_input(pl, tapes, x, d, &last_dt);
  const int64_t nlast = P.ranks[d - 1] * P.dims[d - 1];
  int64_t numel = 1;
  for (int k = 0; k < d; ++k) numel *= P.dims[k];
  // f = ||X - Xhat||^2 streamed in float64 from the forward cores (the form ||X||^2 -
  // ||C_{d-1}||^2 that the reverse sweep differentiates is equal in exact arithmetic, but
  // cancels when f << ||X||^2)
  double* err3 = c.d(G.err3);
  TTR_GCHECK(tt_error_run(x, P.x_dtype, d, P.dims, P.ranks, cores, err3, ws + G.errws, st));
  TTR_GCHECK(axpby(1, 1, 1.0, err3, 1, 0.0, loss, 1, nullptr, st));
  TTR_GCHECK(flag_nonfinite(loss, 1, reinterpret_cast<int*>(ws + kStatusOffset), st));

  // Cbar_{d-1} = -2 C_{d-1}; identity modes pass the adjoint through unchanged.
  int ping = 0;
  void* cb = ws + G.cbar[ping];
  TTR_GCHECK(scale_copy(last, cb, last_dt, nlast, -2.0, st));
  bool reached_x = false;
  for (int k = d - 1; k >= 1 && !reached_x; --k) {
    const ModeGeom& g = pl.modes[k - 1];
    if (g.kind == TTR_MODE_IDENTITY) continue;
    int adt = 0;
    const void* A = mode_input(pl, tapes, x, k, &adt);
    reached_x = A == x;
    void* ab = reached_x ? dx : (void*)(ws + G.cbar[ping ^ 1]);
    if (g.kind == TTR_MODE_REGULAR) rc = backward_regular(c, g, tapes[k - 1], cores[k - 1], A, adt, cb, ab);
    else rc = backward_saturated(c, g, tapes[k - 1], cores[k - 1], A, adt, cb, ab);
    if (rc) return rc;
    cb = ab;
    ping ^= 1;
  }
  // Every mode an identity: the adjoint so far is -2 X itself.
  if (!reached_x) TTR_GCHECK(scale_copy(cb, dx, P.x_dtype, numel, 1.0, st));
  TTR_GCHECK(two_x_plus(x, dx, P.x_dtype, numel, st));
  return TTR_OK;
}

}  // namespace ttr

using namespace ttr;

extern "C" int ttr_rbki_loss_grad(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims,
                                  const int64_t* target_ranks, int32_t q, int32_t p, uint64_t seed,
                                  const ttr_options* opt, void* dx, double* loss, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(d, dims, target_ranks, q, p, x_dtype, opt, &pl);
  if (rc) return rc;
  if (!x || !dx || !loss) { set_error("null tensor, gradient or loss pointer"); return TTR_EINVAL; }
  if (!pl.grad_ok) {
    set_error("the gradient entry needs float64 or float32 input and regular modes with m <= 4096");
    return TTR_EUNSUPPORTED;
  }
  if (!workspace || workspace_bytes < pl.glay.total) {
    set_error("workspace needs " + std::to_string(pl.glay.total) + " bytes");
    return TTR_EWORKSPACE;
  }
  for (const void* ptr : {x, (const void*)dx, (const void*)workspace})
    if ((reinterpret_cast<uintptr_t>(ptr) & 255) != 0) {
      set_error("x, dx and workspace must be 256-byte aligned");
      return TTR_EINVAL;
    }
  return grad_run(x, pl, seed, dx, loss, static_cast<char*>(workspace), static_cast<hipStream_t>(stream));
}
