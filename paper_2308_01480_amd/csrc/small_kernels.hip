// Small dense float64 kernels of the sweep: the m x w and w x w side of every mode
// (projections between Krylov blocks, Gram matrices, SVQB orthonormalisation,
// Rayleigh-Ritz, completion) and the streaming TT reconstruction error.
#include <hip/hip_runtime.h>

#include "common.h"
#include "convert.h"
#include "kernels.h"
#include "qr_tail.h"
#include "wave_ops.h"

namespace ttr {

template <typename T> __device__ inline double ld_as_double(const T* p, int64_t i) { return (double)p[i]; }

// ----------------------------------------------------------------------------------
// C = alpha X^T Y + beta C (or split-K partials), 16 x 16 output tile per work-group.
// ----------------------------------------------------------------------------------
// Split-K: at most kTnMaxChunks row chunks of at least kTnRowsPerChunk rows each (one
// 64-row LDS block per work-group at the sweep's m = 960, so a work-group waits for one
// round of loads).
constexpr int kTnRowsPerChunk = 64;
constexpr int kTnMaxChunks = 15;

template <typename TX, typename TY, typename TC>
__global__ __launch_bounds__(256) void k_gemm_tn(int64_t m, int ka, int kb, const TX* __restrict__ X, int64_t ldx,
                                                 const TY* __restrict__ Y, int64_t ldy, double alpha, double beta,
                                                 TC* __restrict__ C, int64_t ldc, double* __restrict__ part,
                                                 int64_t rows_per_chunk) {
  __shared__ double Xs[64][17];
  __shared__ double Ys[64][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int64_t r0 = (int64_t)blockIdx.z * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < m ? r0 + rows_per_chunk : m;
  // four interleaved partial sums (rows rr = 4i + q go to q), added in a fixed order
  double acc4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t rb = r0; rb < r1; rb += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int rr = e >> 4, cc = e & 15;
      const int64_t row = rb + rr;
      Xs[rr][cc] = (row < r1 && a0 + cc < ka) ? (double)X[row * ldx + a0 + cc] : 0.0;
      Ys[rr][cc] = (row < r1 && b0 + cc < kb) ? (double)Y[row * ldy + b0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 64; rr += 4)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc4[q] = fma(Xs[rr + q][ty], Ys[rr + q][tx], acc4[q]);
    __syncthreads();
  }
  const double acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
  const int a = a0 + ty, b = b0 + tx;
  if (a < ka && b < kb) {
    if (part) {
      part[(int64_t)blockIdx.z * ka * kb + (int64_t)a * kb + b] = acc;
    } else {
      const double old = beta != 0.0 ? (double)C[(int64_t)a * ldc + b] : 0.0;
      C[(int64_t)a * ldc + b] = (TC)(alpha * acc + beta * old);
    }
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void k_gemm_tn_finish(const double* __restrict__ part, int chunks, int ka, int kb,
                                                        double alpha, double beta, TC* __restrict__ C, int64_t ldc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ka * kb) return;
  const int a = idx / kb, b = idx % kb;
  double acc = 0.0;
  for (int z = 0; z < chunks; ++z) acc += part[(int64_t)z * ka * kb + idx];
  const double old = beta != 0.0 ? (double)C[(int64_t)a * ldc + b] : 0.0;
  C[(int64_t)a * ldc + b] = (TC)(alpha * acc + beta * old);
}

template <typename TX, typename TY>
static hipError_t gemm_tn_t(int64_t m, int ka, int kb, const TX* X, int64_t ldx, const TY* Y, int64_t ldy,
                            double alpha, double beta, void* C, int cdt, int64_t ldc, double* scratch,
                            hipStream_t st) {
  int64_t chunks = (m + kTnRowsPerChunk - 1) / kTnRowsPerChunk;
  if (chunks > kTnMaxChunks) chunks = kTnMaxChunks;
  if (chunks < 1 || scratch == nullptr) chunks = 1;
  const int64_t rpc = (m + chunks - 1) / chunks;
  const dim3 grid((ka + 15) / 16, (kb + 15) / 16, (unsigned)chunks);
  const bool split = chunks > 1;
  if (cdt == TTR_F64) {
    hipLaunchKernelGGL((k_gemm_tn<TX, TY, double>), grid, dim3(256), 0, st, m, ka, kb, X, ldx, Y, ldy, alpha, beta,
                       (double*)C, ldc, split ? scratch : nullptr, rpc);
    if (split)
      hipLaunchKernelGGL((k_gemm_tn_finish<double>), dim3((ka * kb + 255) / 256), dim3(256), 0, st, scratch,
                         (int)chunks, ka, kb, alpha, beta, (double*)C, ldc);
  } else {
    hipLaunchKernelGGL((k_gemm_tn<TX, TY, float>), grid, dim3(256), 0, st, m, ka, kb, X, ldx, Y, ldy, alpha, beta,
                       (float*)C, ldc, split ? scratch : nullptr, rpc);
    if (split)
      hipLaunchKernelGGL((k_gemm_tn_finish<float>), dim3((ka * kb + 255) / 256), dim3(256), 0, st, scratch,
                         (int)chunks, ka, kb, alpha, beta, (float*)C, ldc);
  }
  return hipGetLastError();
}

template <typename TX>
static hipError_t gemm_tn_x(int64_t m, int ka, int kb, const TX* X, int64_t ldx, const void* Y, int ydt,
                            int64_t ldy, double alpha, double beta, void* C, int cdt, int64_t ldc, double* scratch,
                            hipStream_t st) {
  if (ydt == TTR_F64) return gemm_tn_t(m, ka, kb, X, ldx, (const double*)Y, ldy, alpha, beta, C, cdt, ldc, scratch, st);
  if (ydt == TTR_F32) return gemm_tn_t(m, ka, kb, X, ldx, (const float*)Y, ldy, alpha, beta, C, cdt, ldc, scratch, st);
  return gemm_tn_t(m, ka, kb, X, ldx, (const __bf16*)Y, ldy, alpha, beta, C, cdt, ldc, scratch, st);
}

hipError_t gemm_tn(int64_t m, int ka, int kb, const void* X, int xdt, int64_t ldx, const void* Y, int ydt,
                   int64_t ldy, double alpha, double beta, void* C, int cdt, int64_t ldc, double* scratch,
                   hipStream_t st) {
  if (ka <= 0 || kb <= 0) return hipSuccess;
  if (xdt == TTR_F64) return gemm_tn_x(m, ka, kb, (const double*)X, ldx, Y, ydt, ldy, alpha, beta, C, cdt, ldc, scratch, st);
  if (xdt == TTR_F32) return gemm_tn_x(m, ka, kb, (const float*)X, ldx, Y, ydt, ldy, alpha, beta, C, cdt, ldc, scratch, st);
  return gemm_tn_x(m, ka, kb, (const __bf16*)X, ldx, Y, ydt, ldy, alpha, beta, C, cdt, ldc, scratch, st);
}

// Symmetric part of the summed split-K partials, C (k x k) = (S + S^T) / 2: work-group
// (bx, by) sums the 16 x 16 tile (bx, by) and its mirror tile (by, bx), both along rows,
// and meets the mirror's transpose through LDS.
__global__ __launch_bounds__(256) void k_gemm_tn_finish_sym(const double* __restrict__ part, int chunks, int k,
                                                            double* __restrict__ C, int64_t ldc) {
  __shared__ double mir[16][17];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int a0 = blockIdx.y * 16, b0 = blockIdx.x * 16;
  const int64_t kk = (int64_t)k * k;
  double s1 = 0.0, s2 = 0.0;
  if (a0 + ty < k && b0 + tx < k)
    for (int z = 0; z < chunks; ++z) s1 += part[z * kk + (int64_t)(a0 + ty) * k + b0 + tx];
  if (b0 + ty < k && a0 + tx < k)
    for (int z = 0; z < chunks; ++z) s2 += part[z * kk + (int64_t)(b0 + ty) * k + a0 + tx];
  mir[ty][tx] = s2;  // S[b0 + ty][a0 + tx]
  __syncthreads();
  if (a0 + ty < k && b0 + tx < k) C[(int64_t)(a0 + ty) * ldc + b0 + tx] = 0.5 * (s1 + mir[tx][ty]);
}

hipError_t gemm_tn_sym(int64_t m, int k, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* C,
                       int64_t ldc, double* scratch, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  if (ldc != k) return hipErrorInvalidValue;
  int64_t chunks = (m + kTnRowsPerChunk - 1) / kTnRowsPerChunk;
  if (chunks > kTnMaxChunks) chunks = kTnMaxChunks;
  if (chunks < 2 || scratch == nullptr) {
    // one chunk: the product, then the symmetric part in place
    const hipError_t e = gemm_tn_t(m, k, k, X, ldx, Y, ldy, 1.0, 0.0, C, TTR_F64, ldc, nullptr, st);
    if (e != hipSuccess) return e;
    return symmetrize(C, k, st);
  }
  const int64_t rpc = (m + chunks - 1) / chunks;
  const dim3 grid((k + 15) / 16, (k + 15) / 16, (unsigned)chunks);
  const dim3 grid2((k + 15) / 16, (k + 15) / 16);
  hipLaunchKernelGGL((k_gemm_tn<double, double, double>), grid, dim3(256), 0, st, m, k, k, X, ldx, Y, ldy, 1.0, 0.0,
                     C, ldc, scratch, rpc);
  hipLaunchKernelGGL(k_gemm_tn_finish_sym, grid2, dim3(256), 0, st, scratch, (int)chunks, k, C, ldc);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// C = alpha X W + beta C, 16 rows x 16 columns per work-group, one output per thread; the
// inner dimension in chunks of 128 whose X rows and W block are loaded in one round.
// ----------------------------------------------------------------------------------
constexpr int kNnRows = 16, kNnK = 128;

// colvals (optional): only the leading columns c with colvals[c] > 0 of W are used, the
// rest read as zero, and their count goes to *ncols.
template <typename TX>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t m, int ka, int kb, const TX* __restrict__ X, int64_t ldx,
                                                 const double* __restrict__ W, int64_t ldw, double alpha,
                                                 double beta, double* __restrict__ C, int64_t ldc,
                                                 const double* __restrict__ colvals, int* __restrict__ ncols) {
  __shared__ double Xs[kNnRows][kNnK + 1];
  __shared__ double Ws[kNnK][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)blockIdx.y * kNnRows;
  const int c0 = blockIdx.x * 16;
  int kc = kb;
  if (colvals) {
    kc = 0;
    while (kc < kb && colvals[kc] > 0.0) ++kc;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *ncols = kc;
  }
  // four interleaved partial sums (k = 4i + q go to q), added in a fixed order
  double acc4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < ka; k0 += kNnK) {
#pragma unroll
    for (int u = 0; u < kNnRows * kNnK / 256; ++u) {
      const int e = (int)threadIdx.x + 256 * u;
      const int rr = e / kNnK, kk = e % kNnK;
      Xs[rr][kk] = (r0 + rr < m && k0 + kk < ka) ? (double)X[(r0 + rr) * ldx + k0 + kk] : 0.0;
      const int wk = e >> 4, wc = e & 15;
      Ws[wk][wc] = (k0 + wk < ka && c0 + wc < kc) ? W[(int64_t)(k0 + wk) * ldw + c0 + wc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kNnK; kk += 4)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc4[q] = fma(Xs[ty][kk + q], Ws[kk + q][tx], acc4[q]);
    __syncthreads();
  }
  const int c = c0 + tx;
  const int64_t row = r0 + ty;
  if (c < kb && row < m) {
    const double acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    const double old = beta != 0.0 ? C[row * ldc + c] : 0.0;
    C[row * ldc + c] = alpha * acc + beta * old;
  }
}

hipError_t gemm_nn(int64_t m, int ka, int kb, const void* X, int xdt, int64_t ldx, const double* W, int64_t ldw,
                   double alpha, double beta, double* C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || kb <= 0) return hipSuccess;
  const dim3 grid((unsigned)((kb + 15) / 16), (unsigned)((m + kNnRows - 1) / kNnRows));
  if (xdt == TTR_F64)
    hipLaunchKernelGGL(k_gemm_nn<double>, grid, dim3(256), 0, st, m, ka, kb, (const double*)X, ldx, W, ldw, alpha,
                       beta, C, ldc, nullptr, nullptr);
  else if (xdt == TTR_F32)
    hipLaunchKernelGGL(k_gemm_nn<float>, grid, dim3(256), 0, st, m, ka, kb, (const float*)X, ldx, W, ldw, alpha,
                       beta, C, ldc, nullptr, nullptr);
  else
    hipLaunchKernelGGL(k_gemm_nn<__bf16>, grid, dim3(256), 0, st, m, ka, kb, (const __bf16*)X, ldx, W, ldw, alpha,
                       beta, C, ldc, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t gemm_nn_ritz(int64_t m, int w, int r, const double* X, int64_t ldx, const double* vecs,
                        const double* vals, double* C, int64_t ldc, int* nv, hipStream_t st) {
  if (m <= 0 || r <= 0 || r > w) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((r + 15) / 16), (unsigned)((m + kNnRows - 1) / kNnRows));
  hipLaunchKernelGGL(k_gemm_nn<double>, grid, dim3(256), 0, st, m, w, r, X, ldx, vecs, (int64_t)w, 1.0, 0.0, C, ldc,
                     vals, nv);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// C (m1 x m2, ldc) = alpha X (m1 x a, ldx) Y^T (Y: m2 x a, ldy) + beta C, float64.
// 16 x 16 output tile per work-group, contraction in chunks of 16.
// ----------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_nt(int64_t m1, int64_t m2, int a, const double* __restrict__ X,
                                                 int64_t ldx, const double* __restrict__ Y, int64_t ldy,
                                                 double alpha, double beta, double* __restrict__ C, int64_t ldc) {
  __shared__ double Xs[16][17];
  __shared__ double Ys[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i0 = (int64_t)blockIdx.y * 16, j0 = (int64_t)blockIdx.x * 16;
  double acc = 0.0;
  for (int k0 = 0; k0 < a; k0 += 16) {
    Xs[ty][tx] = (i0 + ty < m1 && k0 + tx < a) ? X[(i0 + ty) * ldx + k0 + tx] : 0.0;
    Ys[ty][tx] = (j0 + ty < m2 && k0 + tx < a) ? Y[(j0 + ty) * ldy + k0 + tx] : 0.0;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += Xs[ty][kk] * Ys[tx][kk];
    __syncthreads();
  }
  const int64_t i = i0 + ty, j = j0 + tx;
  if (i < m1 && j < m2) {
    const double old = beta != 0.0 ? C[i * ldc + j] : 0.0;
    C[i * ldc + j] = alpha * acc + beta * old;
  }
}

hipError_t gemm_nt(int64_t m1, int64_t m2, int a, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                   double alpha, double beta, double* C, int64_t ldc, hipStream_t st) {
  if (m1 <= 0 || m2 <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m2 + 15) / 16), (unsigned)((m1 + 15) / 16));
  hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, m1, m2, a, X, ldx, Y, ldy, alpha, beta, C, ldc);
  return hipGetLastError();
}

// Y (rows x cols, ldy) = alpha X (ldx) + beta Y; columns >= *ncols_keep (if given) of the
// result are zeroed.
__global__ __launch_bounds__(256) void k_axpby(int64_t rows, int cols, double alpha, const double* __restrict__ X,
                                               int64_t ldx, double beta, double* __restrict__ Y, int64_t ldy,
                                               const int* __restrict__ keep) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx / cols;
  const int j = (int)(idx % cols);
  double v = (X ? alpha * X[i * ldx + j] : 0.0) + (beta != 0.0 ? beta * Y[i * ldy + j] : 0.0);
  if (keep && j >= *keep) v = 0.0;
  Y[i * ldy + j] = v;
}

hipError_t axpby(int64_t rows, int cols, double alpha, const double* X, int64_t ldx, double beta, double* Y,
                 int64_t ldy, const int* keep, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t total = rows * cols;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, rows, cols, alpha, X, ldx,
                     beta, Y, ldy, keep);
  return hipGetLastError();
}

// Out (s x s) = copyltu(alpha M) = tril(alpha M) + tril(alpha M, -1)^T (out of place).
__global__ __launch_bounds__(256) void k_copyltu(const double* __restrict__ M, int s, double alpha,
                                                 double* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= s * s) return;
  const int i = idx / s, j = idx % s;
  out[idx] = alpha * (i >= j ? M[i * s + j] : M[j * s + i]);
}

hipError_t copyltu(const double* M, int s, double alpha, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copyltu, dim3((s * s + 255) / 256), dim3(256), 0, st, M, s, alpha, out);
  return hipGetLastError();
}

// S (n x n) <- K + K^T (out of place).
__global__ __launch_bounds__(256) void k_sym_sum(const double* __restrict__ K, int64_t n, double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  S[idx] = K[i * n + j] + K[j * n + i];
}

hipError_t sym_sum(const double* K, int64_t n, double* S, hipStream_t st) {
  const int64_t total = n * n;
  hipLaunchKernelGGL(k_sym_sum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, K, n, S);
  return hipGetLastError();
}

// Adjoint of the top-r eigenvectors of a symmetric w x w matrix (gauge-invariant use:
// only kept x discarded pairs).  Inputs: U (w x w, column j = eigenvector j of the
// resolved part, zero columns for unresolved directions), lam (w, decreasing, zero for
// unresolved), Ub (w x r, adjoint of U[:, :r]), nvalid (*nv <= r kept columns).
// Out: Mb (w x w) = sym( sum_i v_i u_i^T ), with
//   v_i = sum_{j >= r resolved} u_j (u_j . ub_i) / (lam_i - lam_j)
//       + (ub_i - U_res U_res^T ub_i) / lam_i                    (unresolved: lam_j = 0).
// One work-group; work (w x r) holds the v_i.
__global__ __launch_bounds__(256) void k_eig_adjoint(const double* __restrict__ U, const double* __restrict__ lam,
                                                     int w, int r, const double* __restrict__ Ub,
                                                     const int* __restrict__ nv, double* __restrict__ V,
                                                     double* __restrict__ Mb) {
  __shared__ double proj[256];
  const int tid = threadIdx.x;
  const int kept = *nv < r ? *nv : r;
  int nres = 0;
  while (nres < w && lam[nres] > 0.0) ++nres;
  for (int i = 0; i < kept; ++i) {
    const double li = lam[i];
    // coefficients c_j = u_j . ub_i for every resolved j
    for (int j = tid; j < nres; j += blockDim.x) {
      double acc = 0.0;
      for (int l = 0; l < w; ++l) acc += U[l * w + j] * Ub[l * r + i];
      proj[j] = acc;
    }
    __syncthreads();
    for (int l = tid; l < w; l += blockDim.x) {
      double res = Ub[l * r + i];
      double v = 0.0;
      for (int j = 0; j < nres; ++j) {
        const double uj = U[l * w + j];
        res -= uj * proj[j];
        if (j >= r) v += uj * proj[j] / (li - lam[j]);
      }
      V[l * r + i] = v + res / li;
    }
    __syncthreads();
  }
  // Mb = sym(V U_kept^T)
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int a = e / w, b = e % w;
    double x = 0.0, y = 0.0;
    for (int i = 0; i < kept; ++i) {
      x += V[a * r + i] * U[b * w + i];
      y += V[b * r + i] * U[a * w + i];
    }
    Mb[e] = 0.5 * (x + y);
  }
}

hipError_t eig_adjoint(const double* U, const double* lam, int w, int r, const double* Ub, const int* nv, double* V,
                       double* Mb, hipStream_t st) {
  if (w > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eig_adjoint, dim3(1), dim3(256), 0, st, U, lam, w, r, Ub, nv, V, Mb);
  return hipGetLastError();
}

// lb[i] = -1/2 lam_i^{-3/2} (Vr^T Wb)_{ii} and Vb = Wb diag(lam^{-1/2}) for the
// n < m saturated mode (W = V_r diag(lam^{-1/2})).  One work-group.
__global__ __launch_bounds__(256) void k_scale_adjoint(const double* __restrict__ Vr, int n, int r,
                                                       const double* __restrict__ lam, const double* __restrict__ Wb,
                                                       double* __restrict__ Vb, double* __restrict__ lb) {
  const int tid = threadIdx.x;
  for (int i = tid; i < r; i += blockDim.x) {
    double acc = 0.0;
    for (int l = 0; l < n; ++l) acc += Vr[l * n + i] * Wb[l * r + i];
    lb[i] = lam[i] > 0.0 ? -0.5 * acc / (lam[i] * sqrt(lam[i])) : 0.0;
  }
  for (int e = tid; e < n * r; e += blockDim.x) {
    const int i = e % r;
    Vb[e] = lam[i] > 0.0 ? Wb[e] / sqrt(lam[i]) : 0.0;
  }
}

hipError_t scale_adjoint(const double* Vr, int n, int r, const double* lam, const double* Wb, double* Vb, double* lb,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_scale_adjoint, dim3(1), dim3(256), 0, st, Vr, n, r, lam, Wb, Vb, lb);
  return hipGetLastError();
}

// Mb (n x n) += sum_{i < r} lb_i u_i u_i^T  (eigenvalue part of an eigen adjoint).
__global__ __launch_bounds__(256) void k_add_eigval_adjoint(const double* __restrict__ U, int n, int r,
                                                            const double* __restrict__ lb, double* __restrict__ Mb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int a = e / n, b = e % n;
  double acc = 0.0;
  for (int i = 0; i < r; ++i) acc += lb[i] * U[a * n + i] * U[b * n + i];
  Mb[e] += acc;
}

hipError_t add_eigval_adjoint(const double* U, int n, int r, const double* lb, double* Mb, hipStream_t st) {
  hipLaunchKernelGGL(k_add_eigval_adjoint, dim3((n * n + 255) / 256), dim3(256), 0, st, U, n, r, lb, Mb);
  return hipGetLastError();
}

// Sum of squares of a large array in float64: per-block partials then a fixed-order finish.
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq_big(const T* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = (double)x[i];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_finish(const double* __restrict__ part, int nb, double sign_a,
                                                    const double* __restrict__ other, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sign_a * red[0] + (other ? *other : 0.0);
}

// *out = sign * sum(x^2) + (*other if given); `part` holds 1024 doubles.
hipError_t sumsq_big(const void* x, int dt, int64_t n, double sign, const double* other, double* part, double* out,
                     hipStream_t st) {
  const int nb = 1024;
  if (dt == TTR_F64)
    hipLaunchKernelGGL(k_sumsq_big<double>, dim3(nb), dim3(256), 0, st, (const double*)x, n, part);
  else if (dt == TTR_F32)
    hipLaunchKernelGGL(k_sumsq_big<float>, dim3(nb), dim3(256), 0, st, (const float*)x, n, part);
  else
    hipLaunchKernelGGL(k_sumsq_big<__bf16>, dim3(nb), dim3(256), 0, st, (const __bf16*)x, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(256), 0, st, part, nb, sign, other, out);
  return hipGetLastError();
}

// dX = 2 X + dX (element-wise, X and dX of the same dtype: float64 or float32).
template <typename T>
__global__ __launch_bounds__(256) void k_two_x_plus(const T* __restrict__ x, T* __restrict__ dx, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dx[i] = (T)(2.0 * (double)x[i] + (double)dx[i]);
}

hipError_t two_x_plus(const void* x, void* dx, int dt, int64_t n, hipStream_t st) {
  if (dt == TTR_F64) hipLaunchKernelGGL(k_two_x_plus<double>, dim3(2048), dim3(256), 0, st, (const double*)x, (double*)dx, n);
  else hipLaunchKernelGGL(k_two_x_plus<float>, dim3(2048), dim3(256), 0, st, (const float*)x, (float*)dx, n);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// Eigen-decomposition of a symmetric positive semi-definite n x n Gram matrix G.
//
// 1. Pivoted Cholesky: P^T G P = R^T R (R upper triangular, k x n), stopping when the
//    largest remaining diagonal falls to n * 2^-52 of the largest initial one (what
//    is left is rounding noise of G).  This is the R factor of a column-pivoted QR of
//    any F with F^T F = G, so
// 2. one-sided (Hestenes) Jacobi on the k rows of R (Drmac and Veselic's preconditioned
//    Jacobi SVD) converges in a few sweeps: rows p, q are rotated until
//    r_p . r_q <= tol ||r_p|| ||r_q|| for every pair.  The converged rows are sigma_j u_j
//    with u_j (in pivoted coordinates) the eigenvectors of G and sigma_j^2 its
//    eigenvalues.
// Pairs follow the round-robin (circle) ordering: in round k of a sweep over npad
// (even) indices, pair 0 is (k, npad-1) and pair i >= 1 is ((k+i) mod (npad-1),
// (k-i) mod (npad-1)); every pair meets once per sweep.  A group of G lanes (G | 16,
// inside one DPP row) handles one pair; lane g owns entries g, g+G, ... of both rows
// (at most RPL each, held in registers during the round).  The three dot products are
// summed across the group with DPP permutes (row mirror, half-row mirror, quad
// butterflies), which pair values symmetrically so every lane of the group obtains the
// bitwise same sums and rotation.  Output: vals[j] = sigma_j^2 decreasing, vecs column j
// the matching unit eigenvector; the n - k unresolved directions get zero columns and
// zero values.
// ----------------------------------------------------------------------------------
constexpr int kEigMaxSweeps = 40;


__device__ inline double group_sum(double v, int G) {
  if (G >= 16) v += dpp_mov<0x140>(v);  // row_mirror: lane i <-> 15 - i
  if (G >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror: lane i <-> 7 - i (within 8)
  if (G >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  if (G >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  return v;
}

template <int NT, int G, int RPL, bool IN_LDS>
__global__ __launch_bounds__(NT) void k_eig_psd(const double* __restrict__ g_in, int n, double* __restrict__ vecs,
                                                double* __restrict__ vals, double* __restrict__ work) {
  // Rows have pitch LDA = G * RPL >= n and are zero beyond column n, so every lane
  // reads and writes its RPL entries of a row without bounds checks.
  constexpr int LDA = G * RPL;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rowid[kMaxSmall];   // row of A holding R row j
  __shared__ int remain[kMaxSmall];  // indices not yet eliminated
  __shared__ int s_piv, s_nrem, rotated;
  __shared__ double s_d0;
  __shared__ double norms[kMaxSmall + 1];
  double* A = IN_LDS ? reinterpret_cast<double*>(smem) : work;  // n rows of pitch LDA
  const int tid = threadIdx.x, lane = tid & 63;
  for (int e = tid; e < n * LDA; e += NT) {
    const int i = e / LDA, l = e % LDA;
    A[e] = l < n ? g_in[i * n + l] : 0.0;
  }
  for (int i = tid; i < n; i += NT) remain[i] = i;
  if (tid == 0) s_nrem = n;
  __syncthreads();

  // ---- pivoted Cholesky of the Schur complements, in place and without row swaps:
  // step j picks the remaining index pv with the largest diagonal, turns row pv into
  // R_j = S[pv, :] / sqrt(S[pv, pv]) (zero on eliminated columns) and updates the
  // remaining block.  Sum_j R_j^T R_j = G on the resolved part. ----
  int k = 0;
  for (int j = 0; j < n; ++j) {
    const int nrem = s_nrem;
    if (tid < 64) {  // wave 0: argmax over the remaining diagonal, ties by smaller index
      double best = -1.0;
      int bi = 1 << 30;
      for (int t = lane; t < nrem; t += 64) {
        const int i = remain[t];
        const double d = A[i * LDA + i];
        if (d > best || (d == best && i < bi)) { best = d; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        if (j == 0) s_d0 = best;
        const bool ok = nrem > 0 && best > 0.0 && best > (double)n * 0x1p-52 * (j == 0 ? best : s_d0);
        s_piv = ok ? bi : -1;
        if (ok) {
          rowid[j] = bi;
          int pos = 0;
          while (remain[pos] != bi) ++pos;
          remain[pos] = remain[nrem - 1];
          s_nrem = nrem - 1;
        }
      }
    }
    __syncthreads();
    const int pv = s_piv;
    if (pv < 0) break;
    k = j + 1;
    const double rinv = 1.0 / sqrt(A[pv * LDA + pv]);
    const int nr = s_nrem;
    __syncthreads();  // everyone has read the pivot before row pv is rewritten
    // R_j: diagonal entry sqrt(d), remaining columns scaled, eliminated columns zero
    for (int l = tid; l < n; l += NT) {
      const double v = A[pv * LDA + l];
      bool rem_l = (l == pv);
      for (int t = 0; t < nr && !rem_l; ++t) rem_l = remain[t] == l;
      A[pv * LDA + l] = rem_l ? v * rinv : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < nr * nr; e += NT) {
      const int i = remain[e / nr], l = remain[e % nr];
      A[i * LDA + l] -= A[pv * LDA + i] * A[pv * LDA + l];
    }
    __syncthreads();
  }
  // rows of unresolved indices hold Schur-complement noise: clear them
  for (int t = 0; t < s_nrem; ++t) {
    const int i = remain[t];
    for (int l = tid; l < LDA; l += NT) A[i * LDA + l] = 0.0;
  }
  __syncthreads();

  // ---- Hestenes on the k rows R_j (rows rowid[j] of A) ----
  const int npad = k + (k & 1);
  const int npairs = npad / 2;
  const int pair = tid / G, gl = tid % G;
  const bool active = pair < npairs && k > 1;
  const double tol = 1e-15 * (double)n;
  for (int sweep = 0; sweep < kEigMaxSweeps && k > 1; ++sweep) {
    int mine = 0;
    if (NT > 64) {
      if (tid == 0) rotated = 0;
      __syncthreads();
    }
    int p = 0, q = 0;
    if (active) { p = pair == 0 ? 0 : pair; q = pair == 0 ? npad - 1 : npad - 1 - pair; }
    for (int r = 0; r < npad - 1; ++r) {
      if (active && p < k && q < k) {
        double* rp = A + rowid[p] * LDA + gl;
        double* rq = A + rowid[q] * LDA + gl;
        double x[RPL], y[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) { x[t] = rp[t * G]; y[t] = rq[t * G]; }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) { al += x[t] * x[t]; be += y[t] * y[t]; ga += x[t] * y[t]; }
        al = group_sum(al, G); be = group_sum(be, G); ga = group_sum(ga, G);
        if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          double t;
          if (fabs(zeta) > 1e150) t = 0.5 / zeta;
          else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
          for (int u = 0; u < RPL; ++u) { rp[u * G] = c * x[u] - s * y[u]; rq[u * G] = s * x[u] + c * y[u]; }
          mine = 1;
        }
      }
      __syncthreads();
      if (active) {  // next round: every index except npad-1 advances by one (mod npad-1)
        p = (p == npad - 1) ? p : (p + 1 == npad - 1 ? 0 : p + 1);
        q = (q == npad - 1) ? q : (q + 1 == npad - 1 ? 0 : q + 1);
      }
    }
    int any;
    if (NT == 64) {
      any = __any(mine);
    } else {
      if (mine) rotated = 1;
      __syncthreads();
      any = rotated;
      __syncthreads();
    }
    if (!any) break;
  }
  // ---- values sigma^2 (decreasing, ties by index), unit vectors; unresolved: zero ----
  for (int j = tid; j < n; j += NT) {
    double s2 = 0.0;
    if (j < k) {
      const double* rj = A + rowid[j] * LDA;
      for (int i = 0; i < n; ++i) s2 += rj[i] * rj[i];
    }
    norms[j] = s2;
  }
  __syncthreads();
  for (int j = tid; j < n; j += NT) {
    const double nj = norms[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double ni = norms[i];
      rank += (ni > nj) || (ni == nj && i < j);
    }
    vals[rank] = nj;
    const double inv = nj > 0.0 ? 1.0 / sqrt(nj) : 0.0;
    const double* rj = A + (j < k ? rowid[j] : 0) * LDA;
    for (int i = 0; i < n; ++i) vecs[(int64_t)i * n + rank] = j < k ? rj[i] * inv : 0.0;
  }
}

template <int NT, int G, int RPL, bool IN_LDS>
static hipError_t launch_eig(const double* a, int n, double* vecs, double* vals, double* work, hipStream_t st) {
  const size_t lds = IN_LDS ? (size_t)n * G * RPL * 8 : 0;
  if (IN_LDS) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig_psd<NT, G, RPL, IN_LDS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) { (void)hipGetLastError(); return e; }
  }
  hipLaunchKernelGGL((k_eig_psd<NT, G, RPL, IN_LDS>), dim3(1), dim3(NT), lds, st, a, n, vecs, vals, work);
  return hipGetLastError();
}

hipError_t sym_eig(const double* a, int n, double* vecs, double* vals, double* work, hipStream_t st) {
  if (n <= 0 || n > kMaxSmall) return hipErrorInvalidValue;
  // (threads, lanes per pair, entries per lane): lanes x entries = row pitch >= n,
  // lanes x pairs <= threads.
  if (n <= 16) return launch_eig<64, 8, 2, true>(a, n, vecs, vals, work, st);
  if (n <= 32) return launch_eig<64, 4, 8, true>(a, n, vecs, vals, work, st);
  if (n <= 64) return launch_eig<256, 8, 8, true>(a, n, vecs, vals, work, st);
  if (n <= 128) return launch_eig<1024, 16, 8, true>(a, n, vecs, vals, work, st);
  return launch_eig<1024, 8, 32, false>(a, n, vecs, vals, work, st);
}

// ----------------------------------------------------------------------------------
// Leading eigenpairs of a symmetric n x n matrix (n <= kTopMaxN, r wanted pairs), for
// the Rayleigh-Ritz and saturated Gram steps that only keep the top r directions.
// 1. Householder reduction T = Q^T A Q to tridiagonal form.  A lives in registers:
//    entry (i, j) belongs to thread (i mod 16, j mod 16) of a 16 x 16 grid, so the
//    product A v is summed across the 16 lanes of one row group inside a wave (DPP).
//    The reflectors are kept in LDS, packed.
// 2. The r largest eigenvalues of T by multisection: gl lanes per eigenvalue count the
//    eigenvalues below gl interior points of the current interval (sign changes of
//    the leading principal minors of T - x I, rescaled by powers of two) and keep the
//    sub-interval that holds the wanted index.
// 3. Eigenvectors of T from twisted factorisations of T - lambda I (one forward and
//    one backward recurrence per vector), then two Cholesky-QR passes over all r
//    vectors (clustered eigenvalues give an orthonormal basis of the cluster).
// 4. Back-transformation z = Q y with the stored reflectors.
// Output: vals[0..r) decreasing, vecs[:, 0..r) (leading dimension n) unit vectors;
// a value at or below n 2^-52 vals[0] counts as unresolved and gets a zero value and a
// zero vector; vals[r..n) = 0.
// ----------------------------------------------------------------------------------
constexpr int kTopMaxN = 128;
constexpr int kTopMaxR = 64;
constexpr int kTopThreads = 256;

template <int W>
__device__ inline double group_total(double v) {
  if constexpr (W == 16) return sum16(v);
  else return sum32(v);
}

// 1/x to full precision from the hardware estimate and two Newton steps (|x| >= DBL_MIN).
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Number of eigenvalues of the tridiagonal (d, e2 = e^2) below x: sign changes of
// p_i = det(T_i - x I), p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}, renormalised by a
// power of two every 4 steps; an exact zero counts as a sign change (tiny pivot).
__device__ inline int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n, double x) {
  double pm = 1.0, p = d[0] - x;
  if (p == 0.0) p = -0x1p-1000;
  int c = p < 0.0;
  int i = 1;
  for (; i + 3 < n; i += 4) {
    const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
#define TTR_STURM_STEP(dv, fv)                         \
    {                                                  \
      double pn = fma(dv - x, p, -(fv)*pm);            \
      if (pn == 0.0) pn = -0x1p-1000 * p;              \
      c += (pn < 0.0) != (p < 0.0);                    \
      pm = p;                                          \
      p = pn;                                          \
    }
    TTR_STURM_STEP(d0, f0)
    TTR_STURM_STEP(d1, f1)
    TTR_STURM_STEP(d2, f2)
    TTR_STURM_STEP(d3, f3)
    const int ex = max(__builtin_amdgcn_frexp_exp(p), __builtin_amdgcn_frexp_exp(pm));
    p = ldexp(p, -ex);
    pm = ldexp(pm, -ex);
  }
  for (; i < n; ++i) TTR_STURM_STEP(d[i], e2[i - 1])
#undef TTR_STURM_STEP
  return c;
}

// Packed reflector storage: v_k (entries k+1..n-1) starts at refl_off(k).
__device__ inline int refl_off(int k, int n) { return k * (n - 1) - (k * (k - 1)) / 2; }

// Pivot used for the LDL^T / UDU^T recurrences: magnitudes below `tiny` become +-tiny.
__device__ inline double guard_pivot(double x, double tiny) { return fabs(x) < tiny ? (x < 0.0 ? -tiny : tiny) : x; }

// One panel of the Householder tridiagonalisation in k_eig_top: steps k = 16 KB + kc,
// kc = 0..15, with the register column KB a compile-time index.  Rows and columns below
// 16 KB are finished: their register blocks (a, b < KB) are neither read nor updated.
template <int NB, int KB>
__device__ inline void tri_panel(double (&A)[NB][NB], int n, double (*colb)[kTopMaxN], double (*pb)[kTopMaxN],
                                 double* __restrict__ Vs, double* __restrict__ dd, double* __restrict__ ee,
                                 double* __restrict__ taus) {
  constexpr int TG = 16;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int tr = tid / TG, tc = tid % TG;
  for (int kc = 0; kc < TG; ++kc) {
    const int k = KB * TG + kc;
    if (k + 2 >= n) break;
    double* col = colb[k & 1];
    double* p = pb[k & 1];
    if (tc == kc) {
#pragma unroll
      for (int a = KB; a < NB; ++a) col[tr + TG * a] = A[a][KB];
    }
    __syncthreads();
    double cr[NB], cc[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      cr[a] = col[tr + TG * a];
      cc[a] = col[tc + TG * a];
    }
    const int i1 = k + 1 + lane, i2 = i1 + 64;
    const double c1 = col[i1 < kTopMaxN ? i1 : 0], c2 = col[i2 < kTopMaxN ? i2 : 0];
    const double x0 = col[k + 1];
    // ||x(2:)||^2 over rows k+2 .. n-1 (c1 of lane 0 is x0 itself)
    double s = (lane > 0 && i1 < n ? c1 * c1 : 0.0) + (i2 < n ? c2 * c2 : 0.0);
    s = sum64(s);
    double tau = 0.0, beta = x0, scale = 0.0;
    if (s > 0.0) {
      const double nrm = sqrt(fma(x0, x0, s));
      beta = x0 >= 0.0 ? -nrm : nrm;
      tau = (beta - x0) * rcp_nr(beta);
      scale = rcp_nr(x0 - beta);
    }
    double vr[NB], vc[NB], w[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = tr + TG * a, j = tc + TG * a;
      vr[a] = i == k + 1 ? 1.0 : ((i > k + 1 && i < n) ? cr[a] * scale : 0.0);
      vc[a] = j == k + 1 ? 1.0 : ((j > k + 1 && j < n) ? cc[a] * scale : 0.0);
    }
#pragma unroll
    for (int a = KB; a < NB; ++a) {
      double t = 0.0;
#pragma unroll
      for (int b = KB; b < NB; ++b) t = fma(A[a][b], vc[b], t);
      w[a] = sum16(t);
    }
    if (tc == 0) {
#pragma unroll
      for (int a = KB; a < NB; ++a) p[tr + TG * a] = tau * w[a];
    }
    const double v1 = lane == 0 ? 1.0 : c1 * scale, v2 = c2 * scale;
    if (wid == 0) {
      const int o = refl_off(k, n) - (k + 1);
      if (i1 < n) Vs[o + i1] = v1;
      if (i2 < n) Vs[o + i2] = v2;
      if (lane == 0) { taus[k] = tau; ee[k] = beta; dd[k] = col[k]; }
    }
    __syncthreads();
    double pr[NB], pc[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      pr[a] = p[tr + TG * a];
      pc[a] = p[tc + TG * a];
    }
    const double q1 = p[i1 < kTopMaxN ? i1 : 0], q2 = p[i2 < kTopMaxN ? i2 : 0];
    const double sk = (i1 < n ? v1 * q1 : 0.0) + (i2 < n ? v2 * q2 : 0.0);
    const double K = 0.5 * tau * sum64(sk);
    double wc[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = tr + TG * a, j = tc + TG * a;
      w[a] = (i > k && i < n) ? fma(-K, vr[a], pr[a]) : 0.0;
      wc[a] = (j > k && j < n) ? fma(-K, vc[a], pc[a]) : 0.0;
    }
#pragma unroll
    for (int a = KB; a < NB; ++a)
#pragma unroll
      for (int b = KB; b < NB; ++b) A[a][b] -= vr[a] * wc[b] + w[a] * vc[b];
  }
}

template <int NB, int KB>
struct TriPanels {
  __device__ static void run(double (&A)[NB][NB], int n, double (*colb)[kTopMaxN], double (*pb)[kTopMaxN],
                             double* Vs, double* dd, double* ee, double* taus) {
    if (16 * KB + 2 >= n) return;
    tri_panel<NB, KB>(A, n, colb, pb, Vs, dd, ee, taus);
    TriPanels<NB, KB + 1>::run(A, n, colb, pb, Vs, dd, ee, taus);
  }
};
template <int NB>
struct TriPanels<NB, NB> {
  __device__ static void run(double (&)[NB][NB], int, double (*)[kTopMaxN], double (*)[kTopMaxN], double*, double*,
                             double*, double*) {}
};

// Back-transformation panel KB of k_eig_top: y <- H_k y for k = 16 KB + 15 down to 16 KB
// (k <= n - 3).  Rows below 16 KB are untouched by these reflectors, so only register
// blocks a >= KB take part, and only block KB (rows on both sides of k) and the last block
// (rows beyond n) need a mask.  Two reflectors at a time:
// H_{k-1} H_k y = y - f1 v_k - f2 v_{k-1}, f1 = tau_k v_k^T y,
// f2 = tau_{k-1} (v_{k-1}^T y - (v_{k-1}^T v_k) f1); the three dot products of a pair are
// summed over the 16 lanes of a column group together.
// Reflector v_k (entries k+1..n-1, v_k[k+1] = 1) read by the back-transformation:
// packed in LDS behind each other (n <= kTopMaxN), or one row of pitch kBigPitch each in
// global memory (larger n).  kMaskAll: every register block may hold rows >= n.
struct ReflPacked {
  const double* Vs;
  int n;
  static constexpr bool kMaskAll = false;
  __device__ double operator()(int k, int i) const { return Vs[refl_off(k, n) - (k + 1) + i]; }
};
constexpr int kBigPitch = 256;
struct ReflPitched {
  const double* W;
  static constexpr bool kMaskAll = true;
  __device__ double operator()(int k, int i) const { return W[(int64_t)k * kBigPitch + i]; }
};

template <int NB, int CB2, int KB, class Refl>
__device__ inline void back_panel(double (&yv)[NB][CB2], const Refl& refl, const double* __restrict__ taus, int n,
                                  int rg) {
  constexpr int TG = 16;
  auto load_v = [&](int k, double (&v)[NB]) {
#pragma unroll
    for (int a = KB; a < NB; ++a) {
      const int i = rg + TG * a;
      if (a == KB || a == NB - 1 || Refl::kMaskAll) {
        const int ic = i <= k ? k + 1 : (i < n ? i : n - 1);
        const double x = refl(k, ic);
        v[a] = (i > k && i < n) ? x : 0.0;
      } else {
        v[a] = refl(k, i);
      }
    }
  };
  int k = min(TG * KB + TG - 1, n - 3);
  if (k < TG * KB) return;
  if (((k - TG * KB) & 1) == 0) {  // odd count: one reflector first
    double va[NB];
    load_v(k, va);
    const double t0 = taus[k];
#pragma unroll
    for (int b = 0; b < CB2; ++b) {
      double x1 = 0.0;
#pragma unroll
      for (int a = KB; a < NB; ++a) x1 = fma(va[a], yv[a][b], x1);
      const double f = t0 * sum16(x1);
#pragma unroll
      for (int a = KB; a < NB; ++a) yv[a][b] = fma(-f, va[a], yv[a][b]);
    }
    --k;
  }
  // the next pair's reflectors are loaded while the current pair is applied
  double va[NB], vb[NB];
  if (k > TG * KB) {
    load_v(k, va);
    load_v(k - 1, vb);
  }
  for (; k > TG * KB; k -= 2) {
    const bool more = k - 2 > TG * KB;
    double na[NB], nb[NB];
    if (more) {
      load_v(k - 2, na);
      load_v(k - 3, nb);
    }
    const double ta = taus[k], tb = taus[k - 1];
    double cp = 0.0;
#pragma unroll
    for (int a = KB; a < NB; ++a) cp = fma(vb[a], va[a], cp);
    double d1[CB2], d2[CB2];
#pragma unroll
    for (int b = 0; b < CB2; ++b) {
      double x1 = 0.0, x2 = 0.0;
#pragma unroll
      for (int a = KB; a < NB; ++a) {
        x1 = fma(va[a], yv[a][b], x1);
        x2 = fma(vb[a], yv[a][b], x2);
      }
      d1[b] = sum16(x1);
      d2[b] = sum16(x2);
    }
    const double cab = sum16(cp);
#pragma unroll
    for (int b = 0; b < CB2; ++b) {
      const double f1 = ta * d1[b];
      const double f2 = tb * fma(-cab, f1, d2[b]);
#pragma unroll
      for (int a = KB; a < NB; ++a) yv[a][b] = fma(-f2, vb[a], fma(-f1, va[a], yv[a][b]));
    }
    if (more) {
#pragma unroll
      for (int a = KB; a < NB; ++a) {
        va[a] = na[a];
        vb[a] = nb[a];
      }
    }
  }
}

template <int NB, int CB2, int KB, class Refl>
struct BackPanels {
  __device__ static void run(double (&yv)[NB][CB2], const Refl& refl, const double* taus, int n, int rg) {
    back_panel<NB, CB2, KB>(yv, refl, taus, n, rg);
    BackPanels<NB, CB2, KB - 1, Refl>::run(yv, refl, taus, n, rg);
  }
};
template <int NB, int CB2, class Refl>
struct BackPanels<NB, CB2, -1, Refl> {
  __device__ static void run(double (&)[NB][CB2], const Refl&, const double*, int, int) {}
};

// Parts 2-4 of the leading-eigenpair solver, on the tridiagonal T = (dd, ee) of step 1
// with its Householder reflectors (taus, refl): multisection for the r largest
// eigenvalues, eigenvectors of T (twisted factorisations or inverse iteration inside
// clusters) with Cholesky-QR, back-transformation into vecs / vals (without BACK, vecs
// receives the eigenvectors of T and a separate launch applies the reflectors).  Runs on
// kTopThreads threads; every array is shared memory except vecs, vals (and refl's storage).
template <int NB, int RMAX, bool BACK = true, class Refl>
__device__ inline void eig_top_tail(int n, int r, int bv, int gl, const double* __restrict__ dd,
                                    const double* __restrict__ ee, double* __restrict__ e2,
                                    const double* __restrict__ taus, const Refl& refl, double* __restrict__ lam,
                                    double* __restrict__ rdiag, double (*colx)[64], int* __restrict__ twist,
                                    double* __restrict__ Ys, double* __restrict__ Gm, double* __restrict__ Xi,
                                    double* __restrict__ SD, double* __restrict__ SL, double* __restrict__ SU,
                                    double* __restrict__ vecs, double* __restrict__ vals) {
  constexpr int TG = 16, NT = kTopThreads;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rp = r + 1;
  for (int i = tid; i + 1 < n; i += NT) e2[i] = ee[i] * ee[i];

  // ---- 2. the r largest eigenvalues of T: gl lanes per eigenvalue, gl + 1 subintervals ----
  double glo = 1e308, ghi = -1e308;
  for (int i = lane; i < n; i += 64) {
    const double el = i > 0 ? fabs(ee[i - 1]) : 0.0, er = i + 1 < n ? fabs(ee[i]) : 0.0;
    glo = fmin(glo, dd[i] - el - er);
    ghi = fmax(ghi, dd[i] + el + er);
  }
  glo = min64(glo);
  ghi = max64(ghi);
  const double tnrm = fmax(fmax(fabs(glo), fabs(ghi)), 0x1p-1000);
  const double fudge = 4.0 * (double)n * 0x1p-52 * tnrm;
  glo -= fudge;
  ghi += fudge;
  const double tol = 4.0 * 0x1p-52 * tnrm;
  __syncthreads();
  // groups of gl lanes (2 <= gl <= 32) never straddle a wave: GPW = 64 / gl per wave, the
  // last 64 - GPW gl lanes of a wave idle
  const double frac = 1.0 / (double)(gl + 1);
  const unsigned gmask = (gl >= 32) ? 0xFFFFFFFFu : ((1u << gl) - 1u);
  const int gpw = 64 / gl, gi = lane / gl, g = lane % gl;
  for (int j0 = 0; j0 < r; j0 += (NT / 64) * gpw) {
    const int j = j0 + wid * gpw + gi;
    if (gi < gpw && j < r) {
      const int idx = n - 1 - j;  // ascending index of the j-th largest eigenvalue
      double lo = glo, hi = ghi;
      for (int it = 0; it < 96 && hi - lo > tol; ++it) {
        const double h = (hi - lo) * frac;
        const int c = sturm_count(dd, e2, n, lo + h * (double)(g + 1));
        const uint64_t ball = __ballot(c <= idx);
        const unsigned bits = (unsigned)(ball >> (gi * gl)) & gmask;
        const int top = bits ? 31 - __clz(bits) : -1;  // last point with <= idx values below it
        const double nlo = top >= 0 ? lo + h * (double)(top + 1) : lo;
        const double nhi = top < gl - 1 ? lo + h * (double)(top + 2) : hi;
        lo = nlo;
        hi = nhi;
      }
      if (g == 0) lam[j] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();

  // ---- 3. eigenvectors of T.  Lane pair (2t, 2t+1) factors T - lambda I = L D L^T (forward)
  //         and = U R U^T (backward).  An isolated value takes the twisted vector: at the
  //         index k with the smallest |gamma_k| = |D_k + R_k - (d_k - lambda)|, z_k = 1,
  //         z_i = -L_i z_{i+1} (i < k), z_{i+1} = -U_i z_i (i >= k).  A value within
  //         1e-3 ||T|| of a neighbour instead takes two solves with L D L^T from a hashed
  //         right-hand side, so that the vectors of a cluster span its eigenspace.  Column j
  //         of Ys holds R (then the vector) of eigenvalue j. ----
  const double tiny = 0x1p-52 * tnrm;
  const double cthr = 1e-3 * tnrm;
  bool any_clust = false;
  for (int j = 0; j < r; ++j)
    any_clust |= (j > 0 && lam[j - 1] - lam[j] < cthr) || (j + 1 < r && lam[j] - lam[j + 1] < cthr);
  for (int jb = 0; jb < r; jb += bv) {
    const int t = tid >> 1, side = tid & 1, j = jb + t;
    const bool act = t < bv && j < r;
    const double lj = act ? lam[j] : 0.0;
    const bool clust = act && ((j > 0 && lam[j - 1] - lj < cthr) || (j + 1 < r && lj - lam[j + 1] < cthr));
    if (act && (side == 0 || !clust)) {
      // both lanes of a pair run the same instructions: side 0 forward (L, D: p = D),
      // side 1 backward (U, R: p = R, R kept in column j of Ys)
      double* Xo = side ? SU : SL;
      double* Po = side ? Ys : SD;
      const int ps = side ? rp : bv, pc = side ? j : t;
      double P = guard_pivot(dd[side ? n - 1 : 0] - lj, tiny);
      Po[(side ? n - 1 : 0) * ps + pc] = P;
      for (int st = 0; st + 1 < n; ++st) {
        const int ie = side ? n - 2 - st : st;      // off-diagonal entry of this step
        const int id = side ? n - 2 - st : st + 1;  // diagonal entry it updates
        const double x = ee[ie] * rcp_nr(P);
        Xo[ie * bv + t] = x;
        P = guard_pivot(fma(-x, ee[ie], dd[id] - lj), tiny);
        Po[id * ps + pc] = P;
      }
    }
    __syncthreads();
    if (act && side == 0 && !clust) {
      int kbest = 0;
      double gbest = 1e308;
      for (int k = 0; k < n; ++k) {
        const double gk = fabs(SD[k * bv + t] + Ys[k * rp + j] - (dd[k] - lj));
        if (gk < gbest) { gbest = gk; kbest = k; }
      }
      twist[t] = kbest;
    }
    __syncthreads();
    if (act && !clust) {
      // side 0: z_i = -L_i z_{i+1} for i = kt-1 .. 0; side 1: z_{i+1} = -U_i z_i for
      // i = kt .. n-2 (a zero z takes the three-term relation instead)
      const int kt = twist[t];
      const double* X = side ? SU : SL;
      const int cnt = side ? n - 1 - kt : kt;
      if (side == 0) Ys[kt * rp + j] = 1.0;
      double nn = side ? 0.0 : 1.0;
      double zp = 1.0, zpp = 0.0;
      for (int st = 0; st < cnt; ++st) {
        const int i = side ? kt + st : kt - 1 - st;
        double z = -X[i * bv + t] * zp;
        const bool nb = side ? i > 0 : i + 1 < n - 1;
        const int inb = side ? (i > 0 ? i - 1 : 0) : i + 1;
        if (zp == 0.0 && ee[i] != 0.0 && nb) z = -(ee[inb] / ee[i]) * zpp;
        Ys[(side ? i + 1 : i) * rp + j] = z;
        nn = fma(z, z, nn);
        zpp = zp;
        zp = z;
      }
      const double inv = 1.0 / sqrt(nn + __shfl_xor(nn, 1, 64));
      for (int i = side ? kt + 1 : 0; i < (side ? n : kt + 1); ++i) Ys[i * rp + j] *= inv;
    }
    if (act && clust && side == 0) {
      // x = (L D L^T)^{-1} b twice, in column j of Ys; b_i in [0.5, 1.5) from a hash of (i, j)
      for (int it = 0; it < 2; ++it) {
        double yv = 0.0;
        for (int i = 0; i < n; ++i) {
          const uint32_t hsh = (uint32_t)(i * 2654435761u) ^ (uint32_t)((j + 1) * 40503u);
          const double b = it == 0 ? 0.5 + (double)((hsh >> 8) & 0xFFFF) * (1.0 / 65536.0) : Ys[i * rp + j];
          yv = i == 0 ? b : fma(-SL[(i - 1) * bv + t], yv, b);
          Ys[i * rp + j] = yv;
        }
        double xv = 0.0, nn = 0.0;
        for (int i = n - 1; i >= 0; --i) {
          const double yi = Ys[i * rp + j] * rcp_nr(SD[i * bv + t]);
          xv = i == n - 1 ? yi : fma(-SL[i * bv + t], xv, yi);
          Ys[i * rp + j] = xv;
          nn = fma(xv, xv, nn);
        }
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int i = 0; i < n; ++i) Ys[i * rp + j] *= inv;
      }
    }
    __syncthreads();
  }

  // ---- Cholesky-QR of Y (a second pass when a cluster took inverse iteration): Gram (one
  //      thread per entry), Cholesky on the four waves (lane l holds row l, each wave a
  //      quarter of the columns), then every row of Y solved against R in registers ----
  for (int pass = 0; pass < (any_clust ? 2 : 1); ++pass) {
    for (int e = tid; e < r * r; e += NT) {
      const int c1 = e / r, c2 = e % r;
      if (c1 <= c2) {
        double sacc = 0.0;
#pragma unroll 8
        for (int i = 0; i < n; ++i) sacc = fma(Ys[i * rp + c1], Ys[i * rp + c2], sacc);
        Gm[c1 * rp + c2] = sacc;
      }
    }
    __syncthreads();
    {  // R (upper, rows in Gm), 1 / R_jj in Xi[j]: lane l holds row l, wave w the columns
       // [w CW, (w+1) CW); the pivot row comes from lane k of each wave, the pivot column
       // (= row, by symmetry) through LDS from the wave that owns it
      constexpr int CW = RMAX / 4;
      const int c0 = wid * CW;
      double row[CW];
#pragma unroll
      for (int t = 0; t < CW; ++t) {
        const int c = c0 + t;
        row[t] = (lane < r && c < r) ? (c >= lane ? Gm[lane * rp + c] : Gm[c * rp + lane]) : 0.0;
      }
      for (int k = 0; k < r; ++k) {
        double* cb = colx[k & 1];
        if (k >= c0 && k < c0 + CW) {
          double cv = 0.0;
#pragma unroll
          for (int t = 0; t < CW; ++t) cv = (c0 + t == k) ? row[t] : cv;
          cb[lane] = cv;
        }
        __syncthreads();
        const double d = cb[k];
        const bool ok = d > 1e-20;
        const double rinv = ok ? rsqrt_nr(d) : 0.0;
        const double rl = (ok && lane > k && lane < r) ? cb[lane] * rinv : 0.0;
        if (wid == 0 && lane > k && lane < r) Gm[k * rp + lane] = rl;
        if (tid == 0) { Xi[k] = rinv; rdiag[k] = ok ? d * rinv : 0.0; }
        const double f = -rl * rinv;
#pragma unroll
        for (int t = 0; t < CW; ++t) row[t] = fma(f, lane_value(row[t], k), row[t]);
      }
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) {  // y R = y_old, row by row (dependent columns give zeros)
      double y[RMAX];
#pragma unroll
      for (int jj = 0; jj < RMAX; ++jj) y[jj] = jj < r ? Ys[i * rp + jj] : 0.0;
#pragma unroll
      for (int jj = 0; jj < RMAX; ++jj) {
        double acc = y[jj];
#pragma unroll
        for (int c = 0; c < jj; ++c) acc = fma(-y[c], Gm[c * rp + jj], acc);
        y[jj] = jj < r ? acc * Xi[jj] : 0.0;
      }
#pragma unroll
      for (int jj = 0; jj < RMAX; ++jj)
        if (jj < r) Ys[i * rp + jj] = y[jj];
    }
    __syncthreads();
  }

  if constexpr (!BACK) {
    const double res0 = (double)n * 0x1p-52 * fmax(lam[0], 0.0);
    for (int e = tid; e < n * r; e += NT) {
      const int i = e / r, c = e % r;
      vecs[i * n + c] = (rdiag[c] > 0.0 && lam[c] > res0) ? Ys[i * rp + c] : 0.0;
    }
    for (int c = tid; c < n; c += NT) vals[c] = (c < r && rdiag[c] > 0.0 && lam[c] > res0) ? lam[c] : 0.0;
    return;
  }
  // ---- 4. back-transformation z = Q y with the stored reflectors, last first.  Thread
  //      (row group rg = lane % 16, column group cg = tid / 16) keeps rows rg + 16 a and
  //      columns cg + 16 b of y in registers; the dot products of a reflector with a column
  //      are summed over the 16 lanes of the column group (DPP), so no barrier is needed. ----
  constexpr int CB2 = RMAX / 16;
  const int rg = lane & 15, cg = tid >> 4;
  const double res = (double)n * 0x1p-52 * fmax(lam[0], 0.0);
  double yv[NB][CB2];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < CB2; ++b) {
      const int i = rg + TG * a, c = cg + 16 * b;
      yv[a][b] = (c < r && i < n) ? Ys[i * rp + c] : 0.0;
    }
  // Reflectors are applied two at a time, panel by panel (k = 16 KB + 15 .. 16 KB): see
  // back_panel.
  BackPanels<NB, CB2, NB - 1, Refl>::run(yv, refl, taus, n, rg);
#pragma unroll
  for (int b = 0; b < CB2; ++b) {
    const int c = cg + 16 * b;
    if (c < r) {
      const bool keep = rdiag[c] > 0.0 && lam[c] > res;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int i = rg + TG * a;
        if (i < n) vecs[i * n + c] = keep ? yv[a][b] : 0.0;
      }
      if (rg == 0) vals[c] = keep ? lam[c] : 0.0;
    }
  }
  for (int j = r + tid; j < n; j += NT) vals[j] = 0.0;
}

template <int NB, int RMAX>
__global__ __launch_bounds__(kTopThreads) void k_eig_top(const double* __restrict__ a_in, int n, int r,
                                                         double* __restrict__ vecs, double* __restrict__ vals, int bv,
                                                         int gl) {
  constexpr int TG = 16;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double colb[2][kTopMaxN], pb[2][kTopMaxN];
  __shared__ double dd[kTopMaxN], ee[kTopMaxN], e2[kTopMaxN], taus[kTopMaxN];
  __shared__ double lam[kTopMaxR], rdiag[kTopMaxR], colx[2][64];
  __shared__ int twist[kTopMaxR];
  const int tid = threadIdx.x;
  const int tr = tid / TG, tc = tid % TG;
  const int rp = r + 1;
  double* Vs = reinterpret_cast<double*>(smem);            // packed reflectors
  double* Ys = Vs + ((n * (n - 1) / 2 + 1) & ~1);          // n x rp eigenvectors of T, then of A
  double* Gm = Ys + n * rp;                                // r x rp Gram / R factor
  double* Xi = Gm + r * rp;                                // 1 / R_jj
  double* SD = Xi + r * rp;                                // twisted factorisations, [i * bv + t]
  double* SL = SD + n * bv;
  double* SU = SL + n * bv;

  // ---- 1. tridiagonalisation: every LDS operand of a step is read in one batch ----
  double A[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = tr + TG * a, j = tc + TG * b;
      A[a][b] = (i < n && j < n) ? a_in[i * n + j] : 0.0;
    }
  TriPanels<NB, 0>::run(A, n, colb, pb, Vs, dd, ee, taus);
  {
    const int k0 = n >= 2 ? n - 2 : 0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = tr + TG * a, j = tc + TG * b;
        if (i == j && i >= k0 && i < n) dd[i] = A[a][b];
        if (n >= 2 && i == n - 1 && j == n - 2) ee[n - 2] = A[a][b];
      }
  }
  __syncthreads();
  eig_top_tail<NB, RMAX>(n, r, bv, gl, dd, ee, e2, taus, ReflPacked{Vs, n}, lam, rdiag, colx, twist, Ys, Gm, Xi, SD, SL,
                         SU, vecs, vals);
}

// Dynamic LDS of k_eig_top: packed reflectors, Y, its Gram / R factor and 1 / R_jj, and bv
// pairs of twisted factorisations (D, L, U: 3 doubles per entry and vector).
static size_t eig_top_lds(int n, int r, int bv) {
  const size_t refl = (size_t)((n * (n - 1) / 2 + 1) & ~1) * 8;
  const size_t gx = 2 * (size_t)r * (r + 1);
  return refl + ((size_t)n * (r + 1) + gx) * 8 + (size_t)bv * n * 24 + 16;
}

template <int NB, int RMAX>
static hipError_t launch_eig_top_r(const double* a, int n, int r, double* vecs, double* vals, hipStream_t st, int bv) {
  const size_t lds = eig_top_lds(n, r, bv);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig_top<NB, RMAX>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) { (void)hipGetLastError(); return e; }
  // lanes per eigenvalue: the most (at most 16) that still bisect all r values in one
  // round, with 64 / gl groups in each of the four waves
  int gl = 16;
  while (gl > 2 && (kTopThreads / 64) * (64 / gl) < r) --gl;
  hipLaunchKernelGGL((k_eig_top<NB, RMAX>), dim3(1), dim3(kTopThreads), lds, st, a, n, r, vecs, vals, bv, gl);
  return hipGetLastError();
}

template <int NB>
static hipError_t launch_eig_top(const double* a, int n, int r, double* vecs, double* vals, hipStream_t st, int bv) {
  if (r <= 16) return launch_eig_top_r<NB, 16>(a, n, r, vecs, vals, st, bv);
  if (r <= 32) return launch_eig_top_r<NB, 32>(a, n, r, vecs, vals, st, bv);
  return launch_eig_top_r<NB, 64>(a, n, r, vecs, vals, st, bv);
}

// ----------------------------------------------------------------------------------
// Leading eigenpairs for kTopMaxN < n <= kMaxSmall (the Rayleigh-Ritz matrix of wide
// Krylov spaces, e.g. w = 200): the matrix no longer fits one work-group's registers or
// LDS, so step 1 runs on a copy in global memory (L2-resident: at most 512 KB) and the
// other steps follow on the tridiagonal form.
//
// k_tridiag_big: Householder tridiagonalisation (lower form, as in step 1 of k_eig_top)
// by 1024 threads.  Step k's rank-2 update A -= v w^T + w v^T is applied lazily, fused
// with step k+1's product p = tau A v: one pass over the trailing block per step.  The
// first k0 steps keep the matrix in global memory (L2-resident, rows of pitch kBigPitch;
// wave w owns rows i = w (mod 16), lane l columns l + 64 c).  From step k0 on the trailing
// block's lower triangle (rows and columns >= k0, packed by rows) fits in LDS and the
// product is split in two passes: rows (the update, and sum_{j <= i} A_ij v_j) then
// columns (sum_{i > j} A_ij v_j).  Eight lanes own the pair of rows (and of columns)
// k + 1 + a and n - 1 - a, whose lengths add up to the same count for every a, and sum
// them in a fixed order.  Row k (the symmetric copy of column k) is formed with the
// pending update, gives d_k, e_k and the reflector, which is stored in W[k][k+1..n) for
// the back-transformation.  W: n rows of pitch kBigPitch, then d, e, tau (kBigPitch each).
// ----------------------------------------------------------------------------------
constexpr int kTriThreads = 1024;

__device__ inline double block_sum_tri(double v, double* red, int tid) {
  v = sum64(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kTriThreads / 64; ++w) t += red[w];  // fixed order: every thread the same sum
  __syncthreads();
  return t;
}

// Offset of (i, j), j <= i, in the packed lower triangle of the block that starts at k0.
__device__ inline int tri_off(int i, int j, int k0) {
  const int a = i - k0;
  return a * (a + 1) / 2 + (j - k0);
}

// Step-k start shared by both storage forms: the reflector from xs (row k with the
// pending update), stored as d_k, e_k, tau_k and W[k][k+1..n); vc <- v.  Returns tau.
__device__ inline double tri_reflector(int n, int k, double* xs, double* red, double* s_sc, double* dg, double* eg,
                                       double* tg, double* W, double* vc) {
  const int tid = threadIdx.x;
  double sq = 0.0;
  for (int i = k + 2 + tid; i < n; i += kTriThreads) sq += xs[i] * xs[i];
  sq = block_sum_tri(sq, red, tid);
  if (tid == 0) {
    const double x0 = xs[k + 1];
    double tau = 0.0, beta = x0, scale = 0.0;
    if (sq > 0.0) {
      const double nrm = sqrt(fma(x0, x0, sq));
      beta = x0 >= 0.0 ? -nrm : nrm;
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    s_sc[0] = tau; s_sc[1] = scale;
    dg[k] = xs[k];
    eg[k] = beta;
    tg[k] = tau;
  }
  __syncthreads();
  const double tau = s_sc[0], scale = s_sc[1];
  for (int i = k + 1 + tid; i < n; i += kTriThreads) {
    const double v = i == k + 1 ? 1.0 : xs[i] * scale;
    vc[i] = v;
    W[(int64_t)k * kBigPitch + i] = v;  // reflector k
  }
  if (tid == 0) vc[k] = 0.0;
  __syncthreads();
  return tau;
}

// w = p - (tau/2 v^T p) v on wc (holding p), then the pending update becomes (vc, wc).
__device__ inline void tri_finish_w(int n, int k, double tau, const double* vc, double* wc, double* red) {
  const int tid = threadIdx.x;
  double kv = 0.0;
  for (int i = k + 1 + tid; i < n; i += kTriThreads) kv += vc[i] * wc[i];
  const double K = 0.5 * tau * block_sum_tri(kv, red, tid);
  for (int i = k + 1 + tid; i < n; i += kTriThreads) wc[i] = fma(-K, vc[i], wc[i]);
  if (tid == 0) wc[k] = 0.0;
  __syncthreads();
}

// Row pass of one LDS step for the pair of rows i1 <= i2 (i1 == i2: one row): the pending
// update A_ij -= v_i w_j + w_i v_j over j = k+1..i, written back, and sum_j A_ij c_j with
// the new reflector c_j = x_j scale (c_{k+1} = 1; x = row k, xs).  Lane q of eight takes
// j = k+1+q (mod 8); the vector entries of a column serve both rows, and every load of a
// round is issued before its stores.
__device__ inline void tri_row_pair(double* T, int k0, int k, int i1, int i2, int q, const double* vp,
                                    const double* wp, const double* xs, double scale, double& p1, double& p2) {
  double* ra = T + (i1 - k0) * (i1 - k0 + 1) / 2 - k0;  // element (i1, j) at ra[j]
  double* rb = T + (i2 - k0) * (i2 - k0 + 1) / 2 - k0;
  const bool two = i2 != i1;
  const double va = vp[i1], wa = wp[i1], vb = vp[i2], wb = wp[i2];
  auto cof = [&](int j) { return j == k + 1 ? 1.0 : xs[j] * scale; };
  double pa = 0.0, pb = 0.0;
  int j = k + 1 + q;
  // columns of both rows, two per round
  for (; j + 8 <= i1; j += 16) {
    const double w0 = wp[j], w1 = wp[j + 8], v0 = vp[j], v1 = vp[j + 8];
    const double c0 = cof(j), c1 = cof(j + 8);
    double a0 = ra[j], a1 = ra[j + 8];
    double b0 = two ? rb[j] : 0.0, b1 = two ? rb[j + 8] : 0.0;
    a0 = a0 - va * w0 - wa * v0;
    a1 = a1 - va * w1 - wa * v1;
    ra[j] = a0; ra[j + 8] = a1;
    pa = fma(a0, c0, pa);
    pa = fma(a1, c1, pa);
    if (two) {
      b0 = b0 - vb * w0 - wb * v0;
      b1 = b1 - vb * w1 - wb * v1;
      rb[j] = b0; rb[j + 8] = b1;
      pb = fma(b0, c0, pb);
      pb = fma(b1, c1, pb);
    }
  }
  for (; j <= i1; j += 8) {
    const double w0 = wp[j], v0 = vp[j], c0 = cof(j);
    const double a0 = ra[j] - va * w0 - wa * v0;
    ra[j] = a0;
    pa = fma(a0, c0, pa);
    if (two) {
      const double b0 = rb[j] - vb * w0 - wb * v0;
      rb[j] = b0;
      pb = fma(b0, c0, pb);
    }
  }
  // the rest of row i2, four columns per round
  if (two) {
    for (; j + 24 <= i2; j += 32) {
      double r0 = rb[j], r1 = rb[j + 8], r2 = rb[j + 16], r3 = rb[j + 24];
      const double w0 = wp[j], w1 = wp[j + 8], w2 = wp[j + 16], w3 = wp[j + 24];
      const double v0 = vp[j], v1 = vp[j + 8], v2 = vp[j + 16], v3 = vp[j + 24];
      const double c0 = cof(j), c1 = cof(j + 8), c2 = cof(j + 16), c3 = cof(j + 24);
      r0 = r0 - vb * w0 - wb * v0;
      r1 = r1 - vb * w1 - wb * v1;
      r2 = r2 - vb * w2 - wb * v2;
      r3 = r3 - vb * w3 - wb * v3;
      rb[j] = r0; rb[j + 8] = r1; rb[j + 16] = r2; rb[j + 24] = r3;
      pb = fma(r0, c0, pb);
      pb = fma(r1, c1, pb);
      pb = fma(r2, c2, pb);
      pb = fma(r3, c3, pb);
    }
    for (; j <= i2; j += 8) {
      const double r0 = rb[j] - vb * wp[j] - wb * vp[j];
      rb[j] = r0;
      pb = fma(r0, cof(j), pb);
    }
  }
  p1 = pa;
  p2 = pb;
}

// Column pass for column j: sum_{r > j} A_rj vc_r, lane q of eight taking r = j+1+q (mod 8).
__device__ inline double tri_col_pass(const double* T, int k0, int n, int j, int q, const double* vc) {
  double part = 0.0;
  int r = j + 1 + q;
  int off = tri_off(r, j, k0);  // off(r + 8) = off(r) + 8 (r - k0) + 36
  for (; r + 24 < n; r += 32) {
    const int o1 = off + 8 * (r - k0) + 36;
    const int o2 = o1 + 8 * (r + 8 - k0) + 36;
    const int o3 = o2 + 8 * (r + 16 - k0) + 36;
    const double t0 = T[off], t1 = T[o1], t2 = T[o2], t3 = T[o3];
    const double c0 = vc[r], c1 = vc[r + 8], c2 = vc[r + 16], c3 = vc[r + 24];
    part = fma(t0, c0, part);
    part = fma(t1, c1, part);
    part = fma(t2, c2, part);
    part = fma(t3, c3, part);
    off = o3 + 8 * (r + 24 - k0) + 36;
  }
  for (; r < n; r += 8) {
    part = fma(T[off], vc[r], part);
    off += 8 * (r - k0) + 36;
  }
  return part;
}

__global__ __launch_bounds__(kTriThreads) void k_tridiag_big(const double* __restrict__ a_in, int n,
                                                            double* __restrict__ W, int k0) {
  extern __shared__ double T[];  // packed lower triangle of rows / columns >= k0
  __shared__ double vbuf[2][kBigPitch], wbuf[2][kBigPitch], xs[kBigPitch];
  __shared__ double red[kTriThreads / 64], redK[kTriThreads / 64];
  __shared__ double s_sc[2], s_x0[1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double* dg = W + (int64_t)n * kBigPitch;
  double* eg = dg + kBigPitch;
  double* tg = eg + kBigPitch;
  for (int e = tid; e < n * kBigPitch; e += kTriThreads) {
    const int i = e / kBigPitch, j = e % kBigPitch;
    W[e] = j < n ? a_in[(int64_t)i * n + j] : 0.0;
  }
  for (int i = tid; i < kBigPitch; i += kTriThreads) { vbuf[0][i] = 0.0; wbuf[0][i] = 0.0; }
  if (tid < kTriThreads / 64) redK[tid] = 0.0;
  __syncthreads();
  int cur = 0;  // vbuf/wbuf[cur]: the update pending from the previous step
  int k = 0;
  for (; k + 2 < n && k < k0; ++k) {
    const double* vp = vbuf[cur];
    const double* wp = wbuf[cur];
    for (int i = k + tid; i < n; i += kTriThreads)
      xs[i] = W[(int64_t)k * kBigPitch + i] - vp[k] * wp[i] - wp[k] * vp[i];
    __syncthreads();
    double* vc = vbuf[cur ^ 1];
    double* wc = wbuf[cur ^ 1];
    const double tau = tri_reflector(n, k, xs, red, s_sc, dg, eg, tg, W, vc);
    // fused: pending update of the trailing block, then p_i = tau sum_j A_ij v_j
    for (int i = k + 1 + wid; i < n; i += kTriThreads / 64) {
      double* row = W + (int64_t)i * kBigPitch;
      const double vpi = vp[i], wpi = wp[i];
      double part = 0.0;
#pragma unroll
      for (int c = 0; c < kBigPitch / 64; ++c) {
        const int j = lane + 64 * c;
        if (j > k && j < n) {
          const double a = row[j] - vpi * wp[j] - wpi * vp[j];
          row[j] = a;
          part = fma(a, vc[j], part);
        }
      }
      part = sum64(part);
      if (lane == 0) wc[i] = tau * part;  // p, turned into w below
    }
    __syncthreads();
    tri_finish_w(n, k, tau, vc, wc, red);
    cur ^= 1;
  }
  if (k + 2 < n) {
    // the trailing block (rows and columns >= k = k0) moves to LDS, without the pending update
    for (int i = k + wid; i < n; i += kTriThreads / 64)
      for (int j = k + lane; j <= i; j += 64) T[tri_off(i, j, k0)] = W[(int64_t)i * kBigPitch + j];
    __syncthreads();
  }
  // LDS steps.  At the start of step k, vbuf[cur] holds v of step k - 1 and wbuf[cur] its
  // p = tau A v; its w = p - K v, K = kscale * (sum of redK), is completed by the owner of
  // each entry in phase X (K = 0 on entry: wbuf then holds w itself).
  double kscale = 0.0;
  for (; k + 2 < n; ++k) {
    const double* vp = vbuf[cur];
    double* wp = wbuf[cur];
    double* vc = vbuf[cur ^ 1];
    double* pc = wbuf[cur ^ 1];
    double ks = 0.0;
#pragma unroll
    for (int w = 0; w < kTriThreads / 64; ++w) ks += redK[w];  // fixed order
    const double K = kscale * ks;
    // phase X: thread i - k forms w_i and row k's entry x_i with the pending update
    const int i = k + tid;
    const double vk = vp[k], wk = fma(-K, vk, wp[k]);
    double x = 0.0, sq = 0.0;
    if (i < n) {
      const double vi = vp[i];
      const double wi = fma(-K, vi, wp[i]);
      if (i > k) wp[i] = wi;  // w_k stays p_k in LDS: every thread reads it above
      x = T[tri_off(i, k, k0)] - vk * wi - wk * vi;
      if (i >= k + 2) sq = x * x;
      if (i == k + 1) s_x0[0] = x;
      if (i == k) dg[k] = x;
      xs[i] = x;
    }
    sq = sum64(sq);
    if (lane == 0) red[wid] = sq;
    __syncthreads();
    // the reflector, by every thread from the same sums
    double sqs = 0.0;
#pragma unroll
    for (int w = 0; w < kTriThreads / 64; ++w) sqs += red[w];
    const double x0 = s_x0[0];
    double tau = 0.0, beta = x0, scale = 0.0;
    if (sqs > 0.0) {
      const double nrm = sqrt(fma(x0, x0, sqs));
      beta = x0 >= 0.0 ? -nrm : nrm;
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    if (tid == 0) { eg[k] = beta; tg[k] = tau; }
    // v_i = x_i scale (v_{k+1} = 1): kept by its owner for the column pass and the next
    // step (visible after the row pass's barrier); the row pass forms it from xs itself
    if (i < n) {
      const double v = i == k ? 0.0 : (i == k + 1 ? 1.0 : x * scale);
      vc[i] = v;
      if (i > k) W[(int64_t)k * kBigPitch + i] = v;  // reflector k
    }
    const int N = n - k - 1;  // rows and columns k + 1 .. n - 1
    const int a = tid >> 3, q = tid & 7;
    const int i1 = k + 1 + a, i2 = n - 1 - a;  // i1 == i2: the middle row of an odd N
    const bool act = a < (N + 1) / 2, two = i2 != i1;
    double p1 = 0.0, p2 = 0.0;
    if (act) tri_row_pair(T, k0, k, i1, i2, q, vp, wp, xs, scale, p1, p2);
    p1 = sum8(p1);
    p2 = sum8(p2);
    if (act && q == 0) {
      pc[i1] = p1;
      if (two) pc[i2] = p2;
    }
    __syncthreads();
    double c1 = 0.0, c2 = 0.0;
    if (act) {
      c1 = tri_col_pass(T, k0, n, i1, q, vc);
      if (two) c2 = tri_col_pass(T, k0, n, i2, q, vc);
    }
    c1 = sum8(c1);
    c2 = sum8(c2);
    double kv = 0.0;
    if (act && q == 0) {
      const double pa = tau * (pc[i1] + c1);
      pc[i1] = pa;
      kv = vc[i1] * pa;
      if (two) {
        const double pb = tau * (pc[i2] + c2);
        pc[i2] = pb;
        kv = fma(vc[i2], pb, kv);
      }
    }
    kv = sum64(kv);
    if (lane == 0) redK[wid] = kv;
    kscale = 0.5 * tau;
    __syncthreads();
    cur ^= 1;
  }
  // the last 2 x 2 block with the update of the last step
  if (tid == 0) {
    const double* vp = vbuf[cur];
    const double* wp = wbuf[cur];
    double ks = 0.0;
    for (int w = 0; w < kTriThreads / 64; ++w) ks += redK[w];
    const double K = kscale * ks;
    const int a = n - 2, b = n - 1;
    const double wa = fma(-K, vp[a], wp[a]), wb = fma(-K, vp[b], wp[b]);
    const bool lds = k0 <= a;
    const double aa = lds ? T[tri_off(a, a, k0)] : W[(int64_t)a * kBigPitch + a];
    const double bb = lds ? T[tri_off(b, b, k0)] : W[(int64_t)b * kBigPitch + b];
    const double ba = lds ? T[tri_off(b, a, k0)] : W[(int64_t)b * kBigPitch + a];
    dg[a] = aa - 2.0 * vp[a] * wa;
    dg[b] = bb - 2.0 * vp[b] * wb;
    eg[a] = ba - vp[b] * wa - wb * vp[a];
    tg[a] = 0.0;
    tg[b] = 0.0;
  }
}

// Static LDS of k_tridiag_big (vectors, sums, scalars) and its first LDS step: the smallest
// k0 whose trailing lower triangle (n - k0 rows) fits in the rest of the LDS.
constexpr size_t kTriStaticBytes = (5 * kBigPitch + 2 * (kTriThreads / 64) + 3) * sizeof(double);
static void tri_lds_plan(int n, int* k0, size_t* bytes) {
  const size_t budget = (kLdsBytes - kTriStaticBytes - 256) / sizeof(double);
  int m0 = n;
  while (m0 > 0 && (size_t)m0 * (m0 + 1) / 2 > budget) --m0;
  *k0 = n - m0;
  *bytes = (size_t)m0 * (m0 + 1) / 2 * sizeof(double);
}

// Steps 2-3 on the tridiagonal form of k_tridiag_big (one work-group of kTopThreads): the
// eigenvectors of T go to vecs, k_back_wy applies the reflectors.
template <int RMAX>
__global__ __launch_bounds__(kTopThreads) void k_eig_top_big(const double* __restrict__ W, int n, int r,
                                                             double* __restrict__ vecs, double* __restrict__ vals,
                                                             int bv, int gl) {
  constexpr int NB = kBigPitch / 16;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double dd[kBigPitch], ee[kBigPitch], e2[kBigPitch], taus[kBigPitch];
  __shared__ double lam[kTopMaxR], rdiag[kTopMaxR], colx[2][64];
  __shared__ int twist[kTopMaxR];
  const int tid = threadIdx.x;
  const int rp = r + 1;
  double* Ys = reinterpret_cast<double*>(smem);  // n x rp eigenvectors of T, then of A
  double* Gm = Ys + n * rp;                      // r x rp Gram / R factor
  double* Xi = Gm + r * rp;                      // 1 / R_jj
  double* SD = Xi + r * rp;                      // twisted factorisations, [i * bv + t]
  double* SL = SD + n * bv;
  double* SU = SL + n * bv;
  const double* dg = W + (int64_t)n * kBigPitch;
  for (int i = tid; i < kBigPitch; i += kTopThreads) {
    dd[i] = i < n ? dg[i] : 0.0;
    ee[i] = i + 1 < n ? dg[kBigPitch + i] : 0.0;
    taus[i] = i < n ? dg[2 * kBigPitch + i] : 0.0;
  }
  __syncthreads();
  eig_top_tail<NB, RMAX, false>(n, r, bv, gl, dd, ee, e2, taus, ReflPitched{W}, lam, rdiag, colx, twist, Ys, Gm, Xi,
                                SD, SL, SU, vecs, vals);
}

// ----------------------------------------------------------------------------------
// Step 4 for k_tridiag_big's reflectors: vecs (n x r, row pitch n) <- Q vecs with
// Q = H_0 H_1 ... H_{n-3}, in compact-WY panels of kWyPanel reflectors applied last panel
// first.  Panel p (reflectors k0 = 16 p ...) is P = I - V T V^T with T upper triangular:
// T_jj = tau_j and column j above the diagonal -tau_j T (V_{<j}^T v_j).  The T factors of
// all panels are formed first (one wave each, row a of T in lane a), then each panel is
// three small products over Y held in LDS: X = V^T Y, X <- T X, Y <- Y - V X.  One
// work-group of 1024 threads.
// ----------------------------------------------------------------------------------
constexpr int kWyPanel = 16;
constexpr int kWyThreads = 1024;
constexpr int kWyPairs = kWyPanel * (kWyPanel - 1) / 2;

template <int RMAX>
__global__ __launch_bounds__(kWyThreads) void k_back_wy(const double* __restrict__ W, int n, int r,
                                                        double* __restrict__ vecs) {
  constexpr int P = kWyPanel;
  extern __shared__ __align__(16) unsigned char smem[];
  const int rp = r + 1;
  const int npan = (n - 3) / P + 1;  // reflectors 0 .. n - 3
  double* Ys = reinterpret_cast<double*>(smem);  // n x rp
  double* Vp = Ys + n * rp;                      // n x (P + 1): the current panel, zero where v is
  double* Ts = Vp + n * (P + 1);                 // npan x P x P
  double* Gs = Ts + npan * P * P;                // npan x kWyPairs: v_a . v_b, a < b
  double* Xs = Gs + npan * kWyPairs;             // P x rp
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double* taus = W + (int64_t)(n + 2) * kBigPitch;
  for (int e = tid; e < n * r; e += kWyThreads) Ys[(e / r) * rp + e % r] = vecs[(e / r) * n + e % r];
  // Gram entries of every panel: v_{k0+a} . v_{k0+b} over rows i > k0 + b
  for (int e = tid; e < npan * kWyPairs; e += kWyThreads) {
    const int pn = e / kWyPairs;
    int q = e - pn * kWyPairs, b = 1;
    while (q >= b) { q -= b; ++b; }  // pair (a = q, b), a < b
    const int ka = pn * P + q, kb = pn * P + b;
    double g = 0.0;
    if (kb <= n - 3)
      for (int i = kb + 1; i < n; ++i) g = fma(W[(int64_t)ka * kBigPitch + i], W[(int64_t)kb * kBigPitch + i], g);
    Gs[e] = g;
  }
  __syncthreads();
  if (wid < npan && lane < P) {
    // row a = lane of T for panel wid: T_aj = -tau_j sum_{b=a}^{j-1} T_ab G_bj (j > a)
    const int k0 = wid * P, a = lane;
    const double* G = Gs + wid * kWyPairs;
    double trow[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double tj = k0 + j <= n - 3 ? taus[k0 + j] : 0.0;
      double v = 0.0;
      if (j == a) {
        v = tj;
      } else if (j > a) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < j; ++b)
          if (b >= a) acc = fma(trow[b], G[j * (j - 1) / 2 + b], acc);
        v = -tj * acc;
      }
      trow[j] = v;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) Ts[(wid * P + a) * P + j] = trow[j];
  }
  for (int pn = npan - 1; pn >= 0; --pn) {
    const int k0 = pn * P;
    const int kc = min(P, n - 2 - k0);  // reflectors of this panel
    __syncthreads();
    for (int e = tid; e < n * P; e += kWyThreads) {
      const int i = e / P, j = e % P;
      const int k = k0 + j;
      Vp[i * (P + 1) + j] = (j < kc && i > k) ? W[(int64_t)k * kBigPitch + i] : 0.0;
    }
    __syncthreads();
    {  // X = V^T Y: two lanes per entry (alternate rows), summed by one lane exchange
      const int ent = tid >> 1, h = tid & 1;
      const int j = ent / RMAX, c = ent % RMAX;
      double acc = 0.0;
      if (j < kc && c < r)
        for (int i = k0 + 1 + j + h; i < n; i += 2) acc = fma(Vp[i * (P + 1) + j], Ys[i * rp + c], acc);
      acc += dpp_mov<0xB1>(acc);
      if (h == 0 && j < P && c < r) Xs[j * rp + c] = acc;
    }
    __syncthreads();
    double x2 = 0.0;
    const int j2 = tid / RMAX, c2 = tid % RMAX;
    if (j2 < kc && c2 < r) {
      const double* T = Ts + (pn * P + j2) * P;
      for (int b = j2; b < kc; ++b) x2 = fma(T[b], Xs[b * rp + c2], x2);
    }
    __syncthreads();
    if (j2 < P && c2 < r) Xs[j2 * rp + c2] = x2;
    __syncthreads();
    for (int e = tid; e < (n - k0 - 1) * r; e += kWyThreads) {
      const int i = k0 + 1 + e / r, c = e % r;
      double acc = Ys[i * rp + c];
#pragma unroll
      for (int j = 0; j < P; ++j) acc = fma(-Vp[i * (P + 1) + j], Xs[j * rp + c], acc);
      Ys[i * rp + c] = acc;
    }
  }
  __syncthreads();
  for (int e = tid; e < n * r; e += kWyThreads) vecs[(e / r) * n + e % r] = Ys[(e / r) * rp + e % r];
}

static size_t back_wy_lds(int n, int r) {
  const int npan = (n - 3) / kWyPanel + 1;
  return ((size_t)n * (r + 1) + (size_t)n * (kWyPanel + 1) + (size_t)npan * kWyPanel * kWyPanel +
          (size_t)npan * kWyPairs + (size_t)kWyPanel * (r + 1)) * sizeof(double);
}

// Dynamic LDS of k_eig_top_big: Y, its Gram / R factor and 1 / R_jj, bv twisted factorisations.
static size_t eig_top_big_lds(int n, int r, int bv) {
  return ((size_t)n * (r + 1) + 2 * (size_t)r * (r + 1)) * 8 + (size_t)bv * n * 24 + 16;
}

template <int RMAX>
static hipError_t launch_eig_top_big(const double* a, int n, int r, double* vecs, double* vals, double* work,
                                     hipStream_t st, int bv) {
  int k0 = 0;
  size_t tri_bytes = 0;
  tri_lds_plan(n, &k0, &tri_bytes);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_tridiag_big),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)tri_bytes);
  if (e != hipSuccess) { (void)hipGetLastError(); return e; }
  hipLaunchKernelGGL(k_tridiag_big, dim3(1), dim3(kTriThreads), tri_bytes, st, a, n, work, k0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = eig_top_big_lds(n, r, bv);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig_top_big<RMAX>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) { (void)hipGetLastError(); return e; }
  int gl = 16;
  while (gl > 2 && (kTopThreads / 64) * (64 / gl) < r) --gl;
  hipLaunchKernelGGL((k_eig_top_big<RMAX>), dim3(1), dim3(kTopThreads), lds, st, work, n, r, vecs, vals, bv, gl);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t wy = back_wy_lds(n, r);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_back_wy<RMAX>), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)wy);
  if (e != hipSuccess) { (void)hipGetLastError(); return e; }
  hipLaunchKernelGGL((k_back_wy<RMAX>), dim3(1), dim3(kWyThreads), wy, st, work, n, r, vecs);
  return hipGetLastError();
}

hipError_t sym_eig_top(const double* a, int n, int r, double* vecs, double* vals, double* work, hipStream_t st) {
  if (n <= 0 || r <= 0) return hipErrorInvalidValue;
  if (r > n) r = n;
  // largest batch of twisted factorisations that fits next to the static arrays (~12 KB)
  const size_t budget = kLdsBytes - 14 * 1024;
  int bv = r < kTopThreads / 2 ? r : kTopThreads / 2;
  while (bv > 1 && eig_top_lds(n, r, bv) > budget) --bv;
  if (n > kTopMaxN && n <= kBigPitch && r <= 32 && work) {
    // static arrays of k_eig_top_big: about 11 KB
    const size_t big_budget = kLdsBytes - 14 * 1024;
    int bvb = r < kTopThreads / 2 ? r : kTopThreads / 2;
    while (bvb > 1 && eig_top_big_lds(n, r, bvb) > big_budget) --bvb;
    if (eig_top_big_lds(n, r, bvb) <= big_budget) {
      if (r <= 16) return launch_eig_top_big<16>(a, n, r, vecs, vals, work, st, bvb);
      return launch_eig_top_big<32>(a, n, r, vecs, vals, work, st, bvb);
    }
  }
  if (n > kTopMaxN || r > kTopMaxR || eig_top_lds(n, r, bv) > budget) {
    const hipError_t e = sym_eig(a, n, vecs, vals, work, st);
    if (e != hipSuccess || r == n) return e;
    return axpby(1, n - r, 0.0, nullptr, 0, 0.0, vals + r, n, nullptr, st);  // vals[r..n) = 0
  }
  switch ((n + 15) / 16) {
    case 1: return launch_eig_top<1>(a, n, r, vecs, vals, st, bv);
    case 2: return launch_eig_top<2>(a, n, r, vecs, vals, st, bv);
    case 3: return launch_eig_top<3>(a, n, r, vecs, vals, st, bv);
    case 4: return launch_eig_top<4>(a, n, r, vecs, vals, st, bv);
    case 5: return launch_eig_top<5>(a, n, r, vecs, vals, st, bv);
    case 6: return launch_eig_top<6>(a, n, r, vecs, vals, st, bv);
    case 7: return launch_eig_top<7>(a, n, r, vecs, vals, st, bv);
    default: return launch_eig_top<8>(a, n, r, vecs, vals, st, bv);
  }
}

// ----------------------------------------------------------------------------------
// SVQB transform, Ritz / saturated selection.
// ----------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_svqb(const double* __restrict__ vecs, const double* __restrict__ vals, int n,
                                              const double* __restrict__ ref, double coef, double* __restrict__ T,
                                              int* __restrict__ kept) {
  const double thr = coef * (ref ? *ref : vals[0]);
  int k = 0;
  while (k < n && vals[k] > thr) ++k;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int j = e % n;
    T[e] = j < k ? vecs[e] / sqrt(vals[j]) : 0.0;
  }
  if (threadIdx.x == 0) *kept = k;
}

hipError_t svqb_transform(const double* vecs, const double* vals, int n, const double* ref, double coef, double* T,
                          int* kept, hipStream_t st) {
  hipLaunchKernelGGL(k_svqb, dim3(1), dim3(256), 0, st, vecs, vals, n, ref, coef, T, kept);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// Rank-revealing block orthonormalisation (the economy QR of Algorithm 3, step 5, with
// column pivoting): the pivoted Cholesky of the block Gram Gm = P^T P produces, in exact
// arithmetic, the R factor of P's column-pivoted QR; a Cholesky-QR pass follows.
// ----------------------------------------------------------------------------------
template <int SMAX>
__global__ __launch_bounds__(256) void k_qrcp(const double* __restrict__ Gm, int s, const double* __restrict__ ref,
                                              double coef, double* __restrict__ T, int* __restrict__ kept) {
  __shared__ QrTailSmem<SMAX> sm;
  qrcp_block<SMAX>(Gm, s, s, coef * (*ref), T, kept, sm);
}

hipError_t qrcp_transform(const double* Gm, int s, const double* ref, double coef, double* T, int* kept,
                          hipStream_t st) {
  if (s <= 0 || s > 64) return hipErrorInvalidValue;
  if (s <= 16) hipLaunchKernelGGL(k_qrcp<16>, dim3(1), dim3(256), 0, st, Gm, s, ref, coef, T, kept);
  else if (s <= 32) hipLaunchKernelGGL(k_qrcp<32>, dim3(1), dim3(256), 0, st, Gm, s, ref, coef, T, kept);
  else if (s <= 48) hipLaunchKernelGGL(k_qrcp<48>, dim3(1), dim3(256), 0, st, Gm, s, ref, coef, T, kept);
  else hipLaunchKernelGGL(k_qrcp<64>, dim3(1), dim3(256), 0, st, Gm, s, ref, coef, T, kept);
  return hipGetLastError();
}

template <int SMAX>
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ Gm, int s, const int* __restrict__ kept_in,
                                                  double thresh, double* __restrict__ T, int* __restrict__ kept_out) {
  __shared__ QrTailSmem<SMAX> sm;
  chol_inv_block<SMAX>(Gm, s, s, *kept_in, thresh, T, kept_out, sm);
}

hipError_t chol_inv_transform(const double* Gm, int s, const int* kept_in, double thresh, double* T, int* kept_out,
                              hipStream_t st) {
  if (s <= 0 || s > 64) return hipErrorInvalidValue;
  if (s <= 16) hipLaunchKernelGGL(k_chol_inv<16>, dim3(1), dim3(256), 0, st, Gm, s, kept_in, thresh, T, kept_out);
  else if (s <= 32) hipLaunchKernelGGL(k_chol_inv<32>, dim3(1), dim3(256), 0, st, Gm, s, kept_in, thresh, T, kept_out);
  else if (s <= 48) hipLaunchKernelGGL(k_chol_inv<48>, dim3(1), dim3(256), 0, st, Gm, s, kept_in, thresh, T, kept_out);
  else hipLaunchKernelGGL(k_chol_inv<64>, dim3(1), dim3(256), 0, st, Gm, s, kept_in, thresh, T, kept_out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sat(const double* __restrict__ vecs, const double* __restrict__ vals, int m,
                                             int r, double tau, double* __restrict__ G, int* __restrict__ nv) {
  double tot = 0.0;
  for (int j = 0; j < r && j < m; ++j) tot += vals[j];
  const double thr = tau * tau * tot;
  int k = 0;
  while (k < r && k < m && vals[k] > thr) ++k;
  for (int e = threadIdx.x; e < m * r; e += blockDim.x) {
    const int i = e / r, j = e % r;
    G[e] = j < k ? vecs[(int64_t)i * m + j] : 0.0;
  }
  if (threadIdx.x == 0) *nv = k;
}

hipError_t sat_select(const double* vecs, const double* vals, int m, int r, double tau, double* G, int* nv,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_sat, dim3(1), dim3(256), 0, st, vecs, vals, m, r, tau, G, nv);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// Completion: for i = 0, 1, ... v = e_i - G_c (G_c^T e_i); v -= G_c (G_c^T v); accept
// v / ||v|| when ||v||^2 > 1/(4m), until r columns.  One work-group; v in `work`.
// ----------------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

__global__ __launch_bounds__(256) void k_complete(double* __restrict__ G, int64_t m, int r, const int* __restrict__ nv,
                                                  double* __restrict__ v) {
  __shared__ double red[256];
  __shared__ double coef[64];
  int col = *nv;
  if (col >= r) return;
  const double thresh = 1.0 / (4.0 * (double)m);
  for (int64_t cand = 0; cand < m && col < r; ++cand) {
    // v = e_cand - G_c G_c^T e_cand  (G_c^T e_cand = row cand of G)
    if (threadIdx.x < 64) coef[threadIdx.x] = (int)threadIdx.x < col ? G[cand * r + threadIdx.x] : 0.0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
      double acc = (i == cand) ? 1.0 : 0.0;
      for (int c = 0; c < col; ++c) acc -= G[i * r + c] * coef[c];
      v[i] = acc;
    }
    __syncthreads();
    // second pass: v -= G_c (G_c^T v)
    for (int c = 0; c < col; ++c) {
      double part = 0.0;
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x) part += G[i * r + c] * v[i];
      const double sum = block_sum(part, red);
      if (threadIdx.x == 0) coef[c] = sum;
    }
    __syncthreads();
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
      double acc = v[i];
      for (int c = 0; c < col; ++c) acc -= G[i * r + c] * coef[c];
      v[i] = acc;
      part += acc * acc;
    }
    const double nv2 = block_sum(part, red);
    if (nv2 > thresh) {
      const double inv = 1.0 / sqrt(nv2);
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x) G[i * r + col] = v[i] * inv;
      ++col;
    }
    __syncthreads();
  }
}

hipError_t complete_columns(double* G, int64_t m, int r, const int* nv, double* work, hipStream_t st) {
  if (r > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_complete, dim3(1), dim3(256), 0, st, G, m, r, nv, work);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// Conversions, symmetrisation, identity.
// ----------------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert(const TI* __restrict__ in, int64_t rows, int cols, int64_t ldi,
                                                 TO* __restrict__ out, int64_t rows_pad, int cols_pad, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows_pad * cols_pad) return;
  const int64_t i = idx / cols_pad;
  const int j = (int)(idx % cols_pad);
  out[i * ldo + j] = round_from_f64<TO>((i < rows && j < cols) ? (double)in[i * ldi + j] : 0.0);
}

template <typename TI>
static hipError_t convert_from(const TI* in, int64_t rows, int cols, int64_t ldi, void* out, int odt,
                               int64_t rows_pad, int cols_pad, int64_t ldo, hipStream_t st) {
  const int64_t total = rows_pad * cols_pad;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (odt == TTR_F64)
    hipLaunchKernelGGL((k_convert<TI, double>), grid, dim3(256), 0, st, in, rows, cols, ldi, (double*)out, rows_pad,
                       cols_pad, ldo);
  else if (odt == TTR_F32)
    hipLaunchKernelGGL((k_convert<TI, float>), grid, dim3(256), 0, st, in, rows, cols, ldi, (float*)out, rows_pad,
                       cols_pad, ldo);
  else
    hipLaunchKernelGGL((k_convert<TI, __bf16>), grid, dim3(256), 0, st, in, rows, cols, ldi, (__bf16*)out, rows_pad,
                       cols_pad, ldo);
  return hipGetLastError();
}

hipError_t convert_pad(const void* in, int idt, int64_t rows, int cols, int64_t ldi, void* out, int odt,
                       int64_t rows_pad, int cols_pad, int64_t ldo, hipStream_t st) {
  if (rows_pad <= 0 || cols_pad <= 0) return hipSuccess;
  if (idt == TTR_F64) return convert_from((const double*)in, rows, cols, ldi, out, odt, rows_pad, cols_pad, ldo, st);
  if (idt == TTR_F32) return convert_from((const float*)in, rows, cols, ldi, out, odt, rows_pad, cols_pad, ldo, st);
  return convert_from((const __bf16*)in, rows, cols, ldi, out, odt, rows_pad, cols_pad, ldo, st);
}

__global__ __launch_bounds__(256) void k_symmetrize(double* __restrict__ a, int n) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx / n, j = idx % n;
  if (i < j) {
    const double v = 0.5 * (a[i * n + j] + a[j * n + i]);
    a[i * n + j] = v;
    a[j * n + i] = v;
  }
}

// status |= 1 when any of the n float64 values is NaN or infinite (every writer stores the
// same value, so the race between them is benign).
__global__ __launch_bounds__(256) void k_flag_nonfinite(const double* __restrict__ v, int64_t n,
                                                        int* __restrict__ status) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(v[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) *status = 1;
}

hipError_t flag_nonfinite(const double* v, int64_t n, int* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256);
  hipLaunchKernelGGL(k_flag_nonfinite, dim3((unsigned)blocks), dim3(256), 0, st, v, n, status);
  return hipGetLastError();
}

__global__ void k_set_scalar(double* __restrict__ p, double v) { *p = v; }

hipError_t set_scalar(double* p, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t symmetrize(double* a, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3((n * n + 255) / 256), dim3(256), 0, st, a, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_identity(double* __restrict__ a, int64_t m) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  a[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
}

hipError_t identity(double* a, int64_t m, hipStream_t st) {
  hipLaunchKernelGGL(k_identity, dim3((unsigned)((m * m + 255) / 256)), dim3(256), 0, st, a, m);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// TT reconstruction error.  The modes are split at s: the right part
// R (r_s x inner) = contraction of cores s+1..d is formed once (by the caller);
// work-group o (one outer index tuple of modes 1..s) forms its left interface row
// L = G_1[i_1] ... G_s[i_s] (1 x r_s) and the inner slab Xhat = L R, and
// accumulates ||X - Xhat||^2, ||X||^2 and max |Xhat| in float64.
// ----------------------------------------------------------------------------------
struct TTErrArgs {
  int s;
  int64_t dims[TTR_MAX_D];
  int64_t ranks[TTR_MAX_D + 1];
  const double* cores[TTR_MAX_D];
};

template <typename TX>
__global__ __launch_bounds__(256) void k_tt_error(const TX* __restrict__ x, int64_t outer, int64_t inner,
                                                  TTErrArgs args, const double* __restrict__ R,
                                                  double* __restrict__ part) {
  __shared__ double L[2][64];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t o = blockIdx.x;
  // digits of o in the mixed radix dims[0..s-1] (first index slowest)
  int64_t idx[TTR_MAX_D];
  int64_t rem = o;
  for (int k = args.s - 1; k >= 0; --k) { idx[k] = rem % args.dims[k]; rem /= args.dims[k]; }
  if (tid < 64) L[0][tid] = tid == 0 ? 1.0 : 0.0;
  __syncthreads();
  int cur = 0;
  for (int k = 0; k < args.s; ++k) {
    const int64_t ra = args.ranks[k], rb = args.ranks[k + 1], I = args.dims[k];
    const double* Gk = args.cores[k];
    if (tid < rb) {
      double acc = 0.0;
      for (int a = 0; a < ra; ++a) acc += L[cur][a] * Gk[((int64_t)a * I + idx[k]) * rb + tid];
      L[cur ^ 1][tid] = acc;
    }
    __syncthreads();
    cur ^= 1;
  }
  const int rs = (int)args.ranks[args.s];
  double e2 = 0.0, x2 = 0.0, xinf = 0.0;
  const TX* xo = x + o * inner;
  for (int64_t e = tid; e < inner; e += 256) {
    double xh = 0.0;
    for (int a = 0; a < rs; ++a) xh += L[cur][a] * R[(int64_t)a * inner + e];
    const double xv = (double)xo[e];
    const double df = xv - xh;
    e2 += df * df;
    x2 += xv * xv;
    xinf = fmax(xinf, fabs(xh));
  }
  const double se2 = block_sum(e2, red);
  const double sx2 = block_sum(x2, red);
  red[tid] = xinf;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (tid == 0) {
    part[o * 3 + 0] = se2;
    part[o * 3 + 1] = sx2;
    part[o * 3 + 2] = red[0];
  }
}

__global__ __launch_bounds__(256) void k_tt_error_finish(const double* __restrict__ part, int64_t outer,
                                                         double* __restrict__ out3) {
  __shared__ double r0[256], r1[256], r2[256];
  const int tid = threadIdx.x;
  // fixed assignment of outer blocks to threads, then a fixed tree
  const int64_t per = (outer + 255) / 256;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t o = tid * per; o < (tid + 1) * per && o < outer; ++o) {
    a += part[o * 3]; b += part[o * 3 + 1]; c = fmax(c, part[o * 3 + 2]);
  }
  r0[tid] = a; r1[tid] = b; r2[tid] = c;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) { r0[tid] += r0[tid + off]; r1[tid] += r1[tid + off]; r2[tid] = fmax(r2[tid], r2[tid + off]); }
    __syncthreads();
  }
  if (tid == 0) { out3[0] = r0[0]; out3[1] = r1[0]; out3[2] = r2[0]; }
}

hipError_t tt_error_blocks(const void* x, int xdt, int64_t outer, int64_t inner, int s_split, const int64_t* dims,
                           const int64_t* ranks, const double* const* cores, const double* R, double* part,
                           double* out3, hipStream_t st) {
  TTErrArgs args;
  args.s = s_split;
  for (int k = 0; k < TTR_MAX_D; ++k) {
    args.dims[k] = k < s_split ? dims[k] : 1;
    args.cores[k] = k < s_split ? cores[k] : nullptr;
  }
  for (int k = 0; k <= TTR_MAX_D; ++k) args.ranks[k] = k <= s_split ? ranks[k] : 1;
  const dim3 grid((unsigned)outer);
  if (xdt == TTR_F64)
    hipLaunchKernelGGL(k_tt_error<double>, grid, dim3(256), 0, st, (const double*)x, outer, inner, args, R, part);
  else if (xdt == TTR_F32)
    hipLaunchKernelGGL(k_tt_error<float>, grid, dim3(256), 0, st, (const float*)x, outer, inner, args, R, part);
  else
    hipLaunchKernelGGL(k_tt_error<__bf16>, grid, dim3(256), 0, st, (const __bf16*)x, outer, inner, args, R, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tt_error_finish, dim3(1), dim3(256), 0, st, part, outer, out3);
  return hipGetLastError();
}

}  // namespace ttr
