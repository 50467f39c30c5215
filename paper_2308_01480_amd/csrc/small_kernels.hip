// Small dense float64 kernels of the sweep: the m x w and w x w side of every mode
// (projections between Krylov blocks, Gram matrices, SVQB orthonormalisation,
// Rayleigh-Ritz, completion) and the streaming TT reconstruction error.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace ttr {

template <typename T> __device__ inline double ld_as_double(const T* p, int64_t i) { return (double)p[i]; }

// ----------------------------------------------------------------------------------
// C = alpha X^T Y + beta C (or split-K partials), 16 x 16 output tile per work-group.
// ----------------------------------------------------------------------------------
// Split-K: at most kTnMaxChunks row chunks of about kTnRowsPerChunk rows each.
constexpr int kTnRowsPerChunk = 1024;
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
  double acc = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int rr = e >> 4, cc = e & 15;
      const int64_t row = rb + rr;
      Xs[rr][cc] = (row < r1 && a0 + cc < ka) ? (double)X[row * ldx + a0 + cc] : 0.0;
      Ys[rr][cc] = (row < r1 && b0 + cc < kb) ? (double)Y[row * ldy + b0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 16
    for (int rr = 0; rr < 64; ++rr) acc += Xs[rr][ty] * Ys[rr][tx];
    __syncthreads();
  }
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
  double acc = 0.0;
  for (int z = 0; z < chunks; ++z) acc += part[(int64_t)z * ka * kb + idx];
  const int a = idx / kb, b = idx % kb;
  const double old = beta != 0.0 ? (double)C[(int64_t)a * ldc + b] : 0.0;
  C[(int64_t)a * ldc + b] = (TC)(alpha * acc + beta * old);
}

template <typename TX, typename TY>
static hipError_t gemm_tn_t(int64_t m, int ka, int kb, const TX* X, int64_t ldx, const TY* Y, int64_t ldy,
                            double alpha, double beta, void* C, int cdt, int64_t ldc, double* scratch,
                            hipStream_t st) {
  int64_t chunks = (m + kTnRowsPerChunk - 1) / kTnRowsPerChunk;
  if (chunks > kTnMaxChunks) chunks = kTnMaxChunks;
  if (chunks < 1) chunks = 1;
  const int64_t rpc = (m + chunks - 1) / chunks;
  const dim3 grid((ka + 15) / 16, (kb + 15) / 16, (unsigned)chunks);
  const bool split = chunks > 1;
  if (cdt == TTR_F64) {
    hipLaunchKernelGGL((k_gemm_tn<TX, TY, double>), grid, dim3(256), 0, st, m, ka, kb, X, ldx, Y, ldy, alpha, beta,
                       (double*)C, ldc, split ? scratch : nullptr, rpc);
    if (split)
      hipLaunchKernelGGL(k_gemm_tn_finish<double>, dim3((ka * kb + 255) / 256), dim3(256), 0, st, scratch,
                         (int)chunks, ka, kb, alpha, beta, (double*)C, ldc);
  } else {
    hipLaunchKernelGGL((k_gemm_tn<TX, TY, float>), grid, dim3(256), 0, st, m, ka, kb, X, ldx, Y, ldy, alpha, beta,
                       (float*)C, ldc, split ? scratch : nullptr, rpc);
    if (split)
      hipLaunchKernelGGL(k_gemm_tn_finish<float>, dim3((ka * kb + 255) / 256), dim3(256), 0, st, scratch,
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

// ----------------------------------------------------------------------------------
// C = alpha X W + beta C, 64 rows x 16 columns per work-group.
// ----------------------------------------------------------------------------------
template <typename TX>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t m, int ka, int kb, const TX* __restrict__ X, int64_t ldx,
                                                 const double* __restrict__ W, int64_t ldw, double alpha,
                                                 double beta, double* __restrict__ C, int64_t ldc) {
  __shared__ double Xs[64][17];
  __shared__ double Ws[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int c0 = blockIdx.x * 16;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < ka; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int rr = e >> 4, kk = e & 15;
      Xs[rr][kk] = (r0 + rr < m && k0 + kk < ka) ? (double)X[(r0 + rr) * ldx + k0 + kk] : 0.0;
    }
    {
      const int kk = threadIdx.x >> 4, cc = threadIdx.x & 15;
      Ws[kk][cc] = (k0 + kk < ka && c0 + cc < kb) ? W[(int64_t)(k0 + kk) * ldw + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double w = Ws[kk][tx];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += Xs[ty * 4 + i][kk] * w;
    }
    __syncthreads();
  }
  const int c = c0 + tx;
  if (c < kb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = r0 + ty * 4 + i;
      if (row < m) {
        const double old = beta != 0.0 ? C[row * ldc + c] : 0.0;
        C[row * ldc + c] = alpha * acc[i] + beta * old;
      }
    }
  }
}

hipError_t gemm_nn(int64_t m, int ka, int kb, const void* X, int xdt, int64_t ldx, const double* W, int64_t ldw,
                   double alpha, double beta, double* C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || kb <= 0) return hipSuccess;
  const dim3 grid((unsigned)((kb + 15) / 16), (unsigned)((m + 63) / 64));
  if (xdt == TTR_F64)
    hipLaunchKernelGGL(k_gemm_nn<double>, grid, dim3(256), 0, st, m, ka, kb, (const double*)X, ldx, W, ldw, alpha,
                       beta, C, ldc);
  else if (xdt == TTR_F32)
    hipLaunchKernelGGL(k_gemm_nn<float>, grid, dim3(256), 0, st, m, ka, kb, (const float*)X, ldx, W, ldw, alpha,
                       beta, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_nn<__bf16>, grid, dim3(256), 0, st, m, ka, kb, (const __bf16*)X, ldx, W, ldw, alpha,
                       beta, C, ldc);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi on a symmetric n x n matrix held column by column.
// Columns p, q are rotated until a_p^T a_q <= tol ||a_p|| ||a_q|| for every pair; the
// columns then equal lambda_j v_j, so the eigenvectors are the normalised columns and
// the eigenvalues their norms (the matrices here are positive semi-definite).
// Pairs follow the round-robin (circle) ordering: in round k of a sweep over npad
// (even) indices, pair 0 is (k, npad-1) and pair i >= 1 is ((k+i) mod (npad-1),
// (k-i) mod (npad-1)); every pair of columns meets once per sweep.  A group of G lanes
// (a power of two inside one wave) handles one pair; the groups of a round are
// independent, rounds are separated by barriers.
// ----------------------------------------------------------------------------------
constexpr int kEigThreads = 1024;
constexpr int kEigMaxSweeps = 60;

__device__ inline double group_sum(double v, int G) {
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <bool IN_LDS>
__global__ __launch_bounds__(kEigThreads) void k_jacobi(const double* __restrict__ a_in, int n,
                                                       double* __restrict__ vecs, double* __restrict__ vals,
                                                       double* __restrict__ work) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rotated;
  __shared__ double norms[kMaxSmall + 1];
  double* Mc = IN_LDS ? reinterpret_cast<double*>(smem) : work;  // column-major, column j at Mc + j * n
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kEigThreads) {
    const int i = e / n, j = e % n;
    Mc[(int64_t)j * n + i] = a_in[(int64_t)i * n + j];  // symmetric input: either order
  }
  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  int G = 64;
  while (G > 1 && G * npairs > kEigThreads) G >>= 1;
  const int pair = tid / G, gl = tid % G;
  const double tol = 1e-15 * (double)n;
  __syncthreads();
  for (int sweep = 0; sweep < kEigMaxSweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int k = 0; k < npad - 1; ++k) {
      if (pair < npairs) {
        int p, q;
        if (pair == 0) { p = k; q = npad - 1; }
        else { p = (k + pair) % (npad - 1); q = (k - pair + (npad - 1)) % (npad - 1); }
        if (p < n && q < n) {
          double* cp = Mc + (int64_t)p * n;
          double* cq = Mc + (int64_t)q * n;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = gl; i < n; i += G) {
            const double x = cp[i], y = cq[i];
            al += x * x; be += y * y; ga += x * y;
          }
          al = group_sum(al, G); be = group_sum(be, G); ga = group_sum(ga, G);
          if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
            const double zeta = (be - al) / (2.0 * ga);
            double t;
            if (fabs(zeta) > 1e150) t = 0.5 / zeta;
            else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int i = gl; i < n; i += G) {
              const double x = cp[i], y = cq[i];
              cp[i] = c * x - s * y;
              cq[i] = s * x + c * y;
            }
            if (gl == 0) rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  // norms, ranks (decreasing norm, ties by index), normalised vectors
  for (int j = tid; j < n; j += kEigThreads) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) { const double x = Mc[(int64_t)j * n + i]; s2 += x * x; }
    norms[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < n; j += kEigThreads) {
    const double nj = norms[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double ni = norms[i];
      rank += (ni > nj) || (ni == nj && i < j);
    }
    vals[rank] = nj;
    const double inv = nj > 0.0 ? 1.0 / nj : 0.0;
    for (int i = 0; i < n; ++i) vecs[(int64_t)i * n + rank] = Mc[(int64_t)j * n + i] * inv;
  }
}

hipError_t sym_eig(const double* a, int n, double* vecs, double* vals, double* work, hipStream_t st) {
  if (n <= 0 || n > kMaxSmall) return hipErrorInvalidValue;
  const size_t lds = (size_t)n * n * 8;
  if (n <= 128) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_jacobi<true>, dim3(1), dim3(kEigThreads), lds, st, a, n, vecs, vals, work);
  } else {
    hipLaunchKernelGGL(k_jacobi<false>, dim3(1), dim3(kEigThreads), 0, st, a, n, vecs, vals, work);
  }
  return hipGetLastError();
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

__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ X, int64_t m, int s, int64_t ldx,
                                               double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < m * s; e += 256) {
    const double v = X[(e / s) * ldx + e % s];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t sumsq(const double* X, int64_t m, int s, int64_t ldx, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, st, X, m, s, ldx, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ritz(const double* __restrict__ vecs, const double* __restrict__ vals, int w,
                                              int r, double* __restrict__ U, int* __restrict__ nv) {
  int k = 0;
  while (k < r && k < w && vals[k] > 0.0) ++k;
  for (int e = threadIdx.x; e < w * r; e += blockDim.x) {
    const int i = e / r, j = e % r;
    U[e] = j < k ? vecs[(int64_t)i * w + j] : 0.0;
  }
  if (threadIdx.x == 0) *nv = k;
}

hipError_t ritz_select(const double* vecs, const double* vals, int w, int r, double* U, int* nv, hipStream_t st) {
  hipLaunchKernelGGL(k_ritz, dim3(1), dim3(256), 0, st, vecs, vals, w, r, U, nv);
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
  out[i * ldo + j] = (i < rows && j < cols) ? (TO)(double)in[i * ldi + j] : (TO)0.0;
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
