/*
 * ttrbki.h -- C ABI of the MI355X (gfx950) library for randomized block-Krylov
 * tensor-train approximation (TT-RBKI, arXiv:2308.01480).
 *
 * The library computes, on one GPU, the left-to-right sweep of Algorithm 3:
 * for every mode k it views the current carry as the unfolding A_k
 * (Definition 1), builds the block Krylov space
 *     K = [A Omega, (A A^T) A Omega, ..., (A A^T)^q A Omega]
 * (Algorithm 3, steps 3-5, in column-space form), orthonormalises it,
 * truncates by Rayleigh-Ritz on B = Q^T A (steps 6-9) to the TT core G_k and
 * carries G_k^T A_k forward as the next unfolding (step 10).  The last core
 * is the final carry (step 12).  Tensors are dense, row-major (C order, first
 * index slowest); unfoldings are reshapes of the same memory, never copies.
 *
 * Conventions shared by every entry point
 *   - Pointers named "device" are GPU memory owned by the caller; the library
 *     never allocates, frees or retains memory after returning.
 *   - `stream` is a hipStream_t passed as void*.  All device work is enqueued
 *     on it and the call returns without synchronising.
 *   - Return value 0 = success, negative = error (TTR_E*).  On any argument
 *     error nothing is enqueued.  ttr_strerror() names the code and
 *     ttr_last_error_detail() gives a thread-local message for the last error.
 *   - Index arithmetic is 64-bit: tensors of 2^32 entries and more are valid.
 */
#ifndef TTRBKI_H
#define TTRBKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTR_MAX_D 64

/* Storage type of the input tensor X. */
typedef enum { TTR_F64 = 0, TTR_F32 = 1, TTR_BF16 = 2 } ttr_dtype;

/* Error codes. */
enum {
  TTR_OK = 0,
  TTR_EINVAL = -1,       /* bad argument: d < 2 or > TTR_MAX_D, dims <= 0, ranks <= 0,
                            q < 0, p < 0, null pointer, unknown dtype, size overflow   */
  TTR_EWORKSPACE = -2,   /* workspace smaller than the planned size                    */
  TTR_EHIP = -3,         /* a HIP runtime call failed (launch or attribute query)      */
  TTR_ENUMERIC = -4,     /* non-finite values detected (returned by ttr_check)         */
  TTR_EUNSUPPORTED = -5  /* a mode shape outside what the kernels implement            */
};

/* Kind of a mode after rank clamping (r_k = min(target_k, m_k, n_k), s_k = r_k + p,
 * w_k = (q+1) s_k):
 *   IDENTITY  r_k == m_k: G_k = I and the carry is A_k itself;
 *   SATURATED w_k >= min(m_k, n_k): exact truncated SVD through the short-side Gram;
 *   REGULAR   otherwise: block Krylov space and Rayleigh-Ritz.                          */
enum { TTR_MODE_IDENTITY = 0, TTR_MODE_SATURATED = 1, TTR_MODE_REGULAR = 2 };

/* Sweep drivers (ttr_options.method).  TTR_METHOD_RBKI is the block Krylov method of
 * Algorithm 3 (the default); TTR_METHOD_RSI the subspace iteration of Algorithm 4;
 * TTR_METHOD_RSVD the single sketch of Algorithm 2 (q is ignored). */
enum { TTR_METHOD_RBKI = 0, TTR_METHOD_RSI = 1, TTR_METHOD_RSVD = 2 };

/* Options; pass NULL for defaults. */
typedef struct {
  /* Drop threshold of the rank-revealing orthonormalisation of each Krylov
   * block: a direction is dropped when its singular value is <= tau*||Y_j||_F.
   * <= 0 selects, per mode, the default for the data that mode streams: 1e-10
   * when it is float64, 1e-5 when it is float32 or bfloat16 (both accumulate in
   * float32).  A value > 0 applies to every mode.  Saturated modes complete
   * (replace) singular directions with sigma_i <= tau * sqrt(sum_{j<=r} sigma_j^2). */
  double tau;
  /* TTR_METHOD_*.  With literal = 0 every method truncates by Rayleigh-Ritz: the r_k
   * leading Ritz directions of its final basis (TT-RBKI: the column-space block Krylov
   * space [A Omega, ..., (A A^T)^q A Omega]; TT-rSI: (A A^T)^q A Omega, renormalised each
   * step; TT-rSVD: A Omega), and a mode whose basis width reaches min(m_k, n_k) takes the
   * exact truncated SVD.  With literal = 1 the algorithms run as printed: the first r_k
   * columns of an unpivoted economy QR, for TT-RBKI of Y = A U with U = qr of the
   * row-space K = [A^T A Omega, ..., (A^T A)^q Omega] (needs q >= 1).  Those columns span
   * (A A^T)^j A Omega_r (Omega_r: the first r_k columns of Omega; j = 0 for Algorithm 2,
   * 1 for Algorithm 3, q for Algorithm 4), which the library computes as j renormalised
   * products of an r_k-column block; the gradient entry supports method 0, literal 0. */
  int32_t method;
  int32_t literal;
  /* TTR_KRYLOV_*: how the regular modes of TT-RBKI (method 0, literal 0) form their block
   * products A (A^T Z) and the Rayleigh-Ritz matrix Q^T A A^T Q.  AUTO (0) takes them
   * through the m x m Gram A A^T (one streaming pass, then float64 m x m products) when
   * m <= 256 and that costs fewer flops than q+1 streamed products (m + 16 <= 4 S (q+1),
   * half that for float32 input, whose Gram uses float64 products; S = s rounded up to
   * 16), and streams A otherwise; STREAMED (1) always streams; GRAM (2) takes the Gram
   * whenever m <= 256.  Both forms compute the same quantities (by associativity) up to
   * rounding; the gradient entry always streams. */
  int32_t krylov_form;
  int32_t reserved[5];
} ttr_options;
enum { TTR_KRYLOV_AUTO = 0, TTR_KRYLOV_STREAMED = 1, TTR_KRYLOV_GRAM = 2 };

/* Per-call plan: clamped ranks, mode kinds, shapes and workspace size. */
typedef struct {
  int32_t d, q, p;
  int32_t x_dtype;                 /* ttr_dtype of X                                   */
  int32_t carry_dtype;             /* ttr_dtype of the carries: F64 for F64, else F32  */
  double tau;                      /* drop threshold of the first mode (later modes    */
                                   /* streaming the carry use the carry's default)     */
  int64_t dims[TTR_MAX_D];
  int64_t ranks[TTR_MAX_D + 1];    /* r_0 = 1, r_1..r_{d-1} clamped, r_d = 1           */
  int64_t m[TTR_MAX_D];            /* mode k = 1..d-1 stored at index k-1: m_k rows    */
  int64_t n[TTR_MAX_D];            /*   n_k columns                                     */
  int32_t s[TTR_MAX_D];            /*   s_k = r_k + p                                   */
  int32_t w[TTR_MAX_D];            /*   w_k = (q+1) s_k                                 */
  int32_t kind[TTR_MAX_D];         /*   TTR_MODE_*                                      */
  int32_t two_pass[TTR_MAX_D];     /*   1 if Krylov products use the two-pass kernels   */
  int64_t core_elems[TTR_MAX_D];   /* r_{k-1} I_k r_k elements of core k (k = 1..d)    */
  size_t workspace_bytes;          /* bytes of device workspace ttr_rbki needs         */
  size_t grad_workspace_bytes;     /* bytes ttr_rbki_loss_grad needs; 0 if unsupported */
  int32_t method, literal;         /* the driver (ttr_options); w[] is the width of    */
                                   /* its final basis (s_k or r_k for methods 1, 2)    */
  int32_t gram_first[TTR_MAX_D];   /* 1: mode k's Krylov products go through A_k A_k^T */
} ttr_plan_t;

/*
 * ttr_plan -- validate arguments and plan a sweep.  Host only; touches no GPU.
 *   d              order of X, 2 <= d <= TTR_MAX_D
 *   dims[d]        mode sizes I_1..I_d (> 0)
 *   target_ranks   d-1 target TT ranks (> 0); clamped to min(target, m_k, n_k)
 *                  (Algorithm 3 input r with r_0 = 1)
 *   q              Krylov depth (>= 0): the space has q+1 blocks of s_k columns
 *   p              oversampling (>= 0), s_k = r_k + p (Algorithm 3, step 3)
 *   x_dtype        ttr_dtype of X
 *   opt            options or NULL
 *   out            filled on success
 * Returns TTR_OK, TTR_EINVAL or TTR_EUNSUPPORTED.
 */
int ttr_plan(int32_t d, const int64_t* dims, const int64_t* target_ranks, int32_t q, int32_t p,
             int32_t x_dtype, const ttr_options* opt, ttr_plan_t* out);

/*
 * ttr_rbki -- TT-RBKI sweep (Algorithm 3) of the dense tensor X.
 *   x          device, X in row-major order, x_dtype, numel = prod(dims)
 *   seed       64-bit seed of the Gaussian test matrices: entry (beta, c) of Omega_k is
 *              Box-Muller over Philox4x64-10 with key (seed, k) and counter
 *              (beta, c/8, 0, 0): word j = (c%8)/2 gives u = ((lo32 >> 9) + 1/2) 2^-23 and
 *              v = ((hi32 >> 9) + 1/2) 2^-23, and entries 2j, 2j+1 of the group are
 *              sqrt(-2 ln u) (cos, sin)(2 pi v), evaluated in float32 by a fixed sequence
 *              of correctly rounded operations (the values are float32 numbers).
 *   cores      d device pointers, core k is float64 of shape (r_{k-1}, I_k, r_k),
 *              plan.core_elems[k-1] elements (the G_k are left-orthonormal)
 *   workspace  device scratch of at least plan.workspace_bytes, 256-byte aligned; its
 *              first bytes keep the call's non-finite flag for ttr_check
 * Other arguments as in ttr_plan.  Returns TTR_OK, TTR_EINVAL, TTR_EWORKSPACE,
 * TTR_EUNSUPPORTED or TTR_EHIP.
 */
int ttr_rbki(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims,
             const int64_t* target_ranks, int32_t q, int32_t p, uint64_t seed,
             const ttr_options* opt, double* const* cores, void* workspace,
             size_t workspace_bytes, void* stream);

/*
 * ttr_rbki_noalloc -- ttr_rbki without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The sweep runs the same kernels on a scratch array of
 * TTR_NOALLOC_SCRATCH_BYTES that the library holds in device memory (one per GPU it runs
 * on, from the first call there until the process ends); the call itself allocates
 * nothing.  Plans whose workspace_bytes exceed that size are refused with TTR_EWORKSPACE
 * (nothing enqueued).  The caller still provides X and the cores.  Calls that overlap on
 * one GPU (several streams or threads at once) share the array and race: serialise them.
 * ttr_check(NULL, stream) reads this scratch's non-finite flag on the current device.
 * Returns as ttr_rbki.
 */
#define TTR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int ttr_rbki_noalloc(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims,
                     const int64_t* target_ranks, int32_t q, int32_t p, uint64_t seed,
                     const ttr_options* opt, double* const* cores, void* stream);

/*
 * ttr_check -- status of the last ttr_rbki or ttr_rbki_loss_grad call that used
 * `workspace` (device, the same pointer; NULL: the scratch of ttr_rbki_noalloc on the
 * current device).  Those calls flag non-finite values on the
 * device without synchronising: every mode's first product over its unfolding (A Omega,
 * A A^T or A^T A, which every entry of the unfolding reaches), the last core (which every
 * carry reaches) and, for the gradient entry, the loss.  NaN or infinite input, and
 * products that overflow, are therefore reported.  ttr_check copies the flag to the host
 * on `stream` and waits for it.  Returns TTR_OK, TTR_ENUMERIC, TTR_EINVAL or TTR_EHIP.
 */
int ttr_check(const void* workspace, void* stream);

/*
 * ttr_rbki_loss_grad -- loss f(X) = ||X - TT_r(X)||_F^2 of the TT-RBKI sweep (with the
 * Gaussian test matrices fixed by `seed`) and its gradient df/dX.  f is the streamed
 * ||X - Xhat||^2 of the forward cores (float64 accumulation, as ttr_tt_error).  With
 * left-orthonormal cores it equals ||X||^2 - ||C_{d-1}||^2, the form differentiated in
 * reverse mode through every step of the sweep: carries, Rayleigh-Ritz eigenvectors (pairs of
 * kept and discarded directions), the pivoted QR of each Krylov block (pivots and kept
 * counts held fixed), the projections between blocks and the Krylov products
 * (the Krylov space is recomputed by a forward sweep inside the call, the m x w
 * state is kept).  The function is piecewise smooth; it is not differentiable where a
 * pivot choice, a kept count or the order of the r-th and (r+1)-th eigenvalue changes.
 *   x, x_dtype  device tensor, float64 or float32 (bfloat16: TTR_EUNSUPPORTED)
 *   dx          device output, same shape and dtype as x
 *   loss        device output, one float64
 *   workspace   at least plan.grad_workspace_bytes (0 there means unsupported: regular
 *               modes need m <= 4096); x, dx and workspace 256-byte aligned.  The
 *               workspace holds the forward state and the reverse-sweep scratch.
 * Other arguments as in ttr_rbki.  Returns TTR_OK, TTR_EINVAL, TTR_EWORKSPACE,
 * TTR_EUNSUPPORTED or TTR_EHIP.
 */
int ttr_rbki_loss_grad(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims,
                       const int64_t* target_ranks, int32_t q, int32_t p, uint64_t seed,
                       const ttr_options* opt, void* dx, double* loss, void* workspace,
                       size_t workspace_bytes, void* stream);

/*
 * ttr_tt_error_workspace -- bytes of workspace ttr_tt_error needs.
 * ttr_tt_error -- streaming reconstruction error of a TT (Section 4 metrics):
 *   out3 (device, 3 doubles) <- ( ||X - Xhat||_F^2, ||X||_F^2, ||Xhat||_inf )
 *   where Xhat is the contraction of the float64 cores (Definition 2) with bond
 *   ranks ranks[0..d] (ranks[0] = ranks[d] = 1).  Accumulation is float64 in a
 *   fixed order (bitwise reproducible).
 */
size_t ttr_tt_error_workspace(int32_t d, const int64_t* dims, const int64_t* ranks);
int ttr_tt_error(const void* x, int32_t x_dtype, int32_t d, const int64_t* dims,
                 const int64_t* ranks, const double* const* cores, double* out3,
                 void* workspace, size_t workspace_bytes, void* stream);

/*
 * Building blocks of one mode, exposed for testing and reuse.  A is an m x n
 * row-major matrix (leading dimension n) of dtype a_dtype; small operands and
 * results are float64 row-major device arrays.  ttr_block_workspace gives the
 * scratch size for an (m, n, cols) block call.
 *
 * ttr_omega         out (nrows x s, float64, leading dim s) <- rows beta0..beta0+nrows-1
 *                   of Omega_k drawn from (seed, k) as in ttr_rbki (Algorithm 3, step 3).
 * ttr_sketch        Y (m x s) <- A Omega_k                   (Algorithm 2 step 4 / Alg. 3)
 * ttr_krylov        Y (m x s) <- A (A^T Z), Z (m x s)         (one Krylov block, Alg. 3 step 4)
 * ttr_carry         C (s x n, dtype c_dtype) <- G^T A, G (m x s)  (Alg. 3 step 10)
 * ttr_gram          Gm (m x m) <- A A^T                       (saturated modes)
 * The streamed operand Z or G is rounded to a_dtype before use; accumulation is
 * float32 (f32, bf16) or float64 (f64) inside a work-group, float64 across them.
 */
size_t ttr_block_workspace(int64_t m, int64_t n, int32_t cols, int32_t a_dtype);
int ttr_omega(uint64_t seed, int32_t k, int64_t beta0, int64_t nrows, int32_t s, double* out,
              void* stream);
int ttr_sketch(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k,
               int32_t s, double* y, void* workspace, size_t workspace_bytes, void* stream);
int ttr_krylov(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* z, int32_t s,
               double* y, int32_t force_two_pass, void* workspace, size_t workspace_bytes,
               void* stream);
/* ttr_krylov_timed: ttr_krylov on the one-pass fused path with the streaming kernel
 * launched `reps` times (1..1000) back to back between two caller-created timing events
 * (hipEvent_t, created with timing enabled), recorded on `stream`.  Their elapsed time
 * divided by reps is that kernel's average launch duration: the conversion of Z and the
 * reduction of the per-group partials fall outside it.  Every launch rewrites the same
 * partials, so Y is that of one product.  Returns TTR_EINVAL when an event is null, reps
 * is out of range or the shape takes the two-pass path (see ttr_plan_t.two_pass). */
int ttr_krylov_timed(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* z, int32_t s,
                     double* y, int32_t reps, void* workspace, size_t workspace_bytes, void* ev_begin,
                     void* ev_end, void* stream);
int ttr_carry(const void* a, int32_t a_dtype, int64_t m, int64_t n, const double* g, int32_t s,
              void* c, int32_t c_dtype, void* workspace, size_t workspace_bytes, void* stream);
int ttr_gram(const void* a, int32_t a_dtype, int64_t m, int64_t n, double* gm, void* workspace,
             size_t workspace_bytes, void* stream);

/* ttr_gram_sketch: Gm (m x m) <- A A^T and Y (m x s) <- A Omega_k for m <= 256 (the
 * Gram-first form of Algorithm 3, steps 3-4: the Krylov products of a short unfolding
 * become (A A^T) Q_{j-1}).  Omega_k is drawn inside the streaming kernel, entry by entry as
 * in ttr_rbki (the same values as ttr_omega), and never stored.  bf16: one pass over A
 * forms both (bf16 products, float32 sums per work-group); f32 and f64: the Gram pass
 * (float64 products) and a second pass for the sketch (products in A's dtype).  Workspace:
 * ttr_block_workspace(m, n, s, a_dtype) bytes.
 * ttr_gram_sketch_timed (bf16 only): the same with the one-pass kernel launched `reps`
 * times (1..1000) between two caller-created timing events recorded on `stream` (the
 * reductions of its partials fall outside them); the results are those of one pass.
 * Returns TTR_OK, TTR_EINVAL, TTR_EWORKSPACE, TTR_EUNSUPPORTED (m > 256, or a timed call
 * on f32 / f64) or TTR_EHIP. */
int ttr_gram_sketch(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k, int32_t s,
                    double* gm, double* y, void* workspace, size_t workspace_bytes, void* stream);
int ttr_gram_sketch_timed(const void* a, int32_t a_dtype, int64_t m, int64_t n, uint64_t seed, int32_t k, int32_t s,
                          double* gm, double* y, int32_t reps, void* workspace, size_t workspace_bytes, void* ev_begin,
                          void* ev_end, void* stream);

/* Rank-revealing orthonormal basis of one Krylov block, the economy QR of step 5 of
 * Algorithm 3 read as a QR with column pivoting.  P (m x s, float64, row-major, device)
 * is left unchanged.  Pivots follow the largest remaining column norm; the first k
 * pivots with |R_jj| > tau * ref_norm are kept, then a Cholesky-QR pass restores
 * orthogonality.  Q (m x s, leading dimension s, device): the k kept orthonormal
 * columns first, zeros after; *kept (device int32) = k.  1 <= s <= 64; workspace
 * (device, 256-byte aligned) of ttr_orth_workspace(m, s) bytes.  Returns TTR_OK,
 * TTR_EINVAL, TTR_EWORKSPACE or TTR_EHIP. */
size_t ttr_orth_workspace(int64_t m, int32_t s);
int ttr_orth(const double* p, int64_t m, int32_t s, double ref_norm, double tau, double* q, int32_t* kept,
             void* workspace, size_t workspace_bytes, void* stream);

/* Scratch of the two eigen entries below: ttr_sym_eig_workspace(n) bytes of device
 * memory (256-byte aligned), 0 for n outside [1, 256].  Matrices with n > 128 no longer
 * fit one work-group's LDS and keep their working rows there. */
size_t ttr_sym_eig_workspace(int32_t n);

/* Full eigen-decomposition of a small symmetric positive semi-definite float64 matrix
 * (1 <= n <= 256) on one work-group: pivoted Cholesky, then one-sided Jacobi on the
 * rows of the Cholesky factor.  vecs (n x n, column i = eigenvector i) and vals (n),
 * decreasing; directions whose Cholesky pivot falls below n 2^-52 of the largest
 * diagonal entry are unresolved and get a zero vector and value.  The gradient entry
 * records this decomposition (its adjoint pairs kept with discarded directions).
 * Returns TTR_OK, TTR_EINVAL, TTR_EWORKSPACE or TTR_EHIP. */
int ttr_sym_eig(const double* a, int32_t n, double* vecs, double* vals, void* workspace, size_t workspace_bytes,
                void* stream);

/* Leading r eigenpairs of a small symmetric positive semi-definite float64 matrix
 * (1 <= n <= 256, 1 <= r <= min(n, 64)), the truncation of step 8 of Algorithm 3 read
 * as the r leading Rayleigh-Ritz directions, and the exact truncated SVD of saturated
 * modes.  One work-group: Householder tridiagonalisation, multisection on Sturm counts,
 * inverse iteration and two Cholesky-QR passes, back-transformation (sizes whose
 * working set exceeds the LDS take the full decomposition of ttr_sym_eig).
 *   vals (n): vals[0..r) decreasing, vals[r..n) = 0
 *   vecs (n x n, leading dimension n): columns 0..r-1 unit eigenvectors (for clustered
 *        values an orthonormal basis of the cluster's eigenspace); columns r.. are not
 *        written.  Values at or below n 2^-52 vals[0] are reported as 0 with a zero vector.
 * All pointers are device memory; returns TTR_OK, TTR_EINVAL, TTR_EWORKSPACE or TTR_EHIP. */
int ttr_sym_eig_top(const double* a, int32_t n, int32_t r, double* vecs, double* vals, void* workspace,
                    size_t workspace_bytes, void* stream);

const char* ttr_strerror(int code);
const char* ttr_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* TTRBKI_H */
