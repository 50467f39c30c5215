// Launchers of the library's kernels (internal).  Every launcher enqueues on the given
// stream and returns the HIP error of the launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ttr {

// Operands of a streaming launch over the wide unfolding A (m x n, row-major).
struct StreamArgs {
  const void* A = nullptr;
  int dtype = 0;           // storage of A (TTR_F64 / TTR_F32 / TTR_BF16)
  int64_t m = 0, n = 0, m_pad = 0;
  const void* Z = nullptr; // m_pad x S, dtype of A, zero padded (fused, A^T Z)
  const void* W = nullptr; // n x S, dtype of A (A W)
  void* part = nullptr;    // per-group partial sums
  size_t part_bytes = 0;   // capacity of `part`; a launch that would exceed it is refused
  int S = 16, s = 0;       // padded / used width
  double* y = nullptr;     // m x s float64 result, leading dimension ldy
  int ldy = 0;
  hipStream_t stream = nullptr;
  // Optional timing events (fused product only): recorded on `stream` immediately before
  // and after the streaming kernel, so that their interval excludes the partial reduction.
  // The kernel is launched `reps` times between them (each launch rewrites the same partials).
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  int reps = 1;
  // Gram of float32 input with float64 matrix-core products and sums (launch_gram)
  bool gram_f64 = false;
  // Omega_k of the sketch formed inside a streaming pass (launch_gram_sketch): seed and mode
  uint64_t seed = 0;
  int kmode = 0;
  // float32 A W and A^T Z / carry on the bf16 matrix cores with split operands
  // (launch_aw_split / launch_atz_split) instead of the float32 ones.  With it, the W
  // written by A^T Z (outmode 0) and read by A W is three transposed bf16 planes, plane p
  // row c at W + (p S + c) n (bf16 elements), unless w_f32 marks a float32 n x S W (the
  // materialised Omega of a sketch).
  bool split_f32 = false;
  bool w_f32 = false;
};

inline hipError_t mark_event(hipEvent_t ev, hipStream_t st) { return ev ? hipEventRecord(ev, st) : hipSuccess; }

// True when `groups` partial blocks of `per_group` elements of `elem` bytes fit in a.part.
inline bool part_fits(const StreamArgs& a, int64_t groups, int64_t per_group, size_t elem) {
  return a.part && (size_t)groups * (size_t)per_group * elem <= a.part_bytes;
}

// Streaming kernels (stream_kernels.hip, bf16_kernels.hip).
hipError_t launch_fused(const StreamArgs& a);                 // y = A (A^T Z)
hipError_t launch_aw(const StreamArgs& a);                    // y = A W
hipError_t launch_atz(const StreamArgs& a, void* out, int out_dtype, int64_t ldo, int s_out, int outmode);
hipError_t launch_gram(const StreamArgs& a, double* gm);      // gm = A A^T (m x m)
// gm = A A^T (m x m) and y (m x s, ldy) = A Omega_k in one pass, Omega_k drawn inside the
// kernel from (seed, kmode); float32 input takes float64 Gram products.  The partials
// region holds the Gram partials, then (at gram_part_bytes) the sketch partials.
hipError_t launch_gram_sketch(const StreamArgs& a, double* gm);
hipError_t launch_gram_sketch_bf16(const StreamArgs& a, double* gm);
// y = A Omega_k with Omega_k drawn inside the streaming kernel (m_pad <= 256)
hipError_t launch_aw_omega(const StreamArgs& a);
hipError_t launch_aw_omega_bf16(const StreamArgs& a);
hipError_t launch_omega(uint64_t seed, int k, int64_t beta0, int64_t nrows, int s, int ldo, void* out,
                        int out_dtype, hipStream_t st);
hipError_t launch_fused_bf16(const StreamArgs& a);
// Omega_k transposed (S x nrows float32, pitch ldt; rows c >= s zero).
hipError_t launch_omega_t(uint64_t seed, int k, int64_t nrows, int s, int S, int64_t ldt, float* out, hipStream_t st);
// bfloat16 A (m_pad <= 256): the float32 carry out = Z^T A (rows < s_out, pitch ldo) and,
// in the same pass, the next mode's sketch y = C' Omega (float64, (s_out n / nc) x s2,
// pitch ldy) of the carry read as the (s_out n / nc) x nc unfolding, with the transposed
// Omega omt (S2 x nc float32).  a.part holds carry_sketch_part_bytes of partials.
bool carry_sketch_fits(int dtype, int64_t m_pad, int S, int64_t n, int64_t nc, int S2);
size_t carry_sketch_part_bytes(int64_t n, int64_t nc, int S, int S2);
hipError_t launch_carry_sketch_bf16(const StreamArgs& a, float* out, int64_t ldo, int s_out, const float* omt, int64_t nc,
                                    int S2, int s2, double* y, int64_t ldy);
hipError_t launch_aw_bf16(const StreamArgs& a);
hipError_t launch_atz_bf16(const StreamArgs& a, void* out, int out_dtype, int64_t ldo, int s_out, int outmode);
hipError_t launch_gram_bf16(const StreamArgs& a, double* gm);
// Float32 A W and A^T Z / carry on the bf16 matrix cores with three-way split operands
// (float32 accuracy); out of A^T Z is float32.  With `omega` W is Omega_k drawn inside the
// kernel (m_pad <= 256).
hipError_t launch_aw_split(const StreamArgs& a, bool omega = false);
hipError_t launch_atz_split(const StreamArgs& a, void* out, int64_t ldo, int s_out, int outmode);

// Block orthonormalisation in row-parallel launches (block_orth.hip).  G <= kOrthMaxGroups
// work-groups write partials (G x len doubles in `part`, G doubles in `norm_part`); the
// last one, found through `counter` (zero between launches), reduces them.
struct OrthArgs {
  int64_t m = 0;
  int s = 0, js = 0;                               // block width, previous basis width
  const double* Q = nullptr; int64_t ldq = 0;      // previous basis (m x js)
  double* P = nullptr; int64_t ldp = 0;            // projected block (m x s)
  double* U = nullptr; int64_t ldu = 0;            // P T1 (m x s)
  double* h = nullptr; double* h2 = nullptr;       // js x s projection coefficients
  double* T1 = nullptr; double* T2 = nullptr;      // s x s transforms of the two passes
  double* Tprod = nullptr;                         // T1 T2 (optional)
  int* kept1 = nullptr; int* kept2 = nullptr;
  double* ref = nullptr;                           // ||Y||_F^2 of the raw block
  bool ref_from_gram = false;                      // ref = trace(P^T P) of the first update
  double coef = 0.0;                               // first-pass drop: pivot <= coef * ref
  double thresh2 = 1e-6;                           // second-pass drop threshold
  double* part = nullptr; size_t part_bytes = 0;
  double* norm_part = nullptr;
  int* counter = nullptr;
  double* Qout = nullptr; int64_t ldqo = 0;        // Q_j (m x s)
  void* zs = nullptr; int zdt = 0; int64_t m_pad = 0; int Sz = 0;  // stream copy of Q_j
  hipStream_t st = nullptr;
  // Tall blocks: up to kOrthBigGroups row-parallel work-groups write partials (part,
  // norm_part sized for them), and a separate reduction launch sums them in group order;
  // its last work-group runs the s x s step on the sum, kept in gsum (s x s).
  bool big = false;
  double* gsum = nullptr;
};

hipError_t orth_reset_counter(int* counter, hipStream_t st);  // *counter = 0 (device)
// *status = 1 when any of v[0..n) is not finite (status otherwise left unchanged)
hipError_t flag_nonfinite(const double* v, int64_t n, int* status, hipStream_t st);
hipError_t orth_project(const OrthArgs& a, const double* Y, int64_t ldy);     // h = Q^T Y (+ ref)
hipError_t orth_update(const OrthArgs& a, const double* S, int64_t lds, const double* W, bool next_proj);
hipError_t orth_tgram(const OrthArgs& a);                                     // U = P T1, T2
hipError_t orth_out(const OrthArgs& a);                                       // Q_j = U T2

// Small dense float64 kernels (small_kernels.hip).
// C (ka x kb, ldc) = alpha * X^T Y + beta * C, X: m x ka (ldx, dtype xdt), Y: m x kb (ldy, ydt).
// `scratch` holds split-K partials (up to 15 * ka * kb doubles when m > 64; NULL: no split).
hipError_t gemm_tn(int64_t m, int ka, int kb, const void* X, int xdt, int64_t ldx, const void* Y, int ydt,
                   int64_t ldy, double alpha, double beta, void* C, int cdt, int64_t ldc, double* scratch,
                   hipStream_t st);
// C (k x k, ldc) = the symmetric part (X^T Y + Y^T X) / 2 of X^T Y, X and Y: m x k float64.
hipError_t gemm_tn_sym(int64_t m, int k, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* C,
                       int64_t ldc, double* scratch, hipStream_t st);
// C (m x kb, ldc) = alpha * X (m x ka, ldx, dtype xdt) W (ka x kb, ldw) + beta * C.
hipError_t gemm_nn(int64_t m, int ka, int kb, const void* X, int xdt, int64_t ldx, const double* W, int64_t ldw,
                   double alpha, double beta, double* C, int64_t ldc, hipStream_t st);
// Rayleigh-Ritz basis: C (m x r, ldc) = X (m x w, ldx) U with U = the leading columns j < nv
// of vecs (w x w) whose vals[j] > 0 (the rest zero); *nv = their count.
hipError_t gemm_nn_ritz(int64_t m, int w, int r, const double* X, int64_t ldx, const double* vecs,
                        const double* vals, double* C, int64_t ldc, int* nv, hipStream_t st);
// One-sided Jacobi eigen-decomposition of symmetric a (n x n): vecs (n x n, column j =
// vector j) and vals (n), by decreasing value.  `work` holds n*n doubles when n > 128.
hipError_t sym_eig(const double* a, int n, double* vecs, double* vals, double* work, hipStream_t st);
// The r leading eigenpairs only: vals[0..r) decreasing, vecs[:, 0..r) (leading dimension n),
// vals[r..n) zero; unresolved values (<= n 2^-52 vals[0]) get zero values and vectors.
// Falls back to sym_eig (which uses `work` for n > 128) beyond n = 128 or r = 64.
hipError_t sym_eig_top(const double* a, int n, int r, double* vecs, double* vals, double* work, hipStream_t st);
// SVQB transform T (n x n): columns j < kept are vecs[:, j] / sqrt(vals[j]) for the
// vals[j] > thresh, the rest zero.  thresh = coef * (*ref) (ref on device; NULL: vals[0]).
hipError_t svqb_transform(const double* vecs, const double* vals, int n, const double* ref, double coef,
                          double* T, int* kept, hipStream_t st);
// Rank-revealing first pass: T (s x s) from the pivoted Cholesky of Gm = P^T P (the R of
// P's column-pivoted QR), pivots d > coef * (*ref) kept; P T = leading columns of Q.
hipError_t qrcp_transform(const double* Gm, int s, const double* ref, double coef, double* T, int* kept,
                          hipStream_t st);
// Second-pass transform T = R^{-1} of the Cholesky factor of Gm (s x s, s <= 64) restricted to
// the first *kept_in columns, dropping pivots <= thresh; surviving columns packed first.
hipError_t chol_inv_transform(const double* Gm, int s, const int* kept_in, double thresh, double* T, int* kept_out,
                              hipStream_t st);
// Saturated selection: G (m x r) = eigenvectors j < r with vals[j] > tau^2 * sum_{i<r} vals[i]; nv = count.
hipError_t sat_select(const double* vecs, const double* vals, int m, int r, double tau, double* G, int* nv,
                      hipStream_t st);
// Completion of G (m x r, first *nv columns valid) by e_1, e_2, ... (classical Gram-Schmidt twice).
hipError_t complete_columns(double* G, int64_t m, int r, const int* nv, double* work, hipStream_t st);
// Dtype conversion with zero padding: out (rows_pad x cols_pad, ldo) <- in (rows x cols, ldi).
hipError_t convert_pad(const void* in, int idt, int64_t rows, int cols, int64_t ldi, void* out, int odt,
                       int64_t rows_pad, int cols_pad, int64_t ldo, hipStream_t st);
hipError_t symmetrize(double* a, int n, hipStream_t st);
hipError_t set_scalar(double* p, double v, hipStream_t st);  // *p = v (device)
hipError_t identity(double* a, int64_t m, hipStream_t st);
// Streaming TT reconstruction error: partial sums per outer prefix, then out3.
hipError_t tt_error_blocks(const void* x, int xdt, int64_t outer, int64_t inner, int s_split,
                           const int64_t* dims, const int64_t* ranks, const double* const* cores_dev,
                           const double* R, double* part, double* out3, hipStream_t st);

// ---- backward-pass helpers (float64 small matrices) ----
// C (m1 x m2) = alpha X (m1 x a) Y^T (Y: m2 x a) + beta C.
hipError_t gemm_nt(int64_t m1, int64_t m2, int a, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                   double alpha, double beta, double* C, int64_t ldc, hipStream_t st);
// Y = alpha X + beta Y (X may be null), columns >= *keep zeroed when keep is given.
hipError_t axpby(int64_t rows, int cols, double alpha, const double* X, int64_t ldx, double beta, double* Y,
                 int64_t ldy, const int* keep, hipStream_t st);
// out = copyltu(alpha M) = tril(alpha M) + tril(alpha M, -1)^T, s x s.
hipError_t copyltu(const double* M, int s, double alpha, double* out, hipStream_t st);
// S = K + K^T (n x n).
hipError_t sym_sum(const double* K, int64_t n, double* S, hipStream_t st);
// Adjoint of the leading eigenvectors (kept x discarded pairs), see small_kernels.hip.
hipError_t eig_adjoint(const double* U, const double* lam, int w, int r, const double* Ub, const int* nv, double* V,
                       double* Mb, hipStream_t st);
hipError_t scale_adjoint(const double* Vr, int n, int r, const double* lam, const double* Wb, double* Vb, double* lb,
                         hipStream_t st);
hipError_t add_eigval_adjoint(const double* U, int n, int r, const double* lb, double* Mb, hipStream_t st);
// *out = sign * sum(x^2) + (*other if given); part holds 1024 doubles.
hipError_t sumsq_big(const void* x, int dt, int64_t n, double sign, const double* other, double* part, double* out,
                     hipStream_t st);
// dx = 2 x + dx (float64 or float32).
hipError_t two_x_plus(const void* x, void* dx, int dt, int64_t n, hipStream_t st);

}  // namespace ttr
