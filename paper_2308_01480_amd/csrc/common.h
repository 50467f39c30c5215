// Internal declarations of the TT-RBKI library: mode geometry, workspace layout and
// error reporting shared by the planner (host only) and the HIP driver.
#pragma once

#include <cstddef>
#include <algorithm>
#include <cstdint>
#include <string>

#include "../../include/ttrbki.h"

namespace ttr {

// ---------------------------------------------------------------------------------
// Tile geometry of the streaming kernels.  Every streaming kernel runs NW = 4
// wavefronts of 64 lanes and walks the wide unfolding in column tiles of TT(dtype)
// columns; Krylov blocks are padded to S = 16 * ceil(s / 16) columns (MFMA width).
// ---------------------------------------------------------------------------------
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxGroups = 1024;          // column groups of one streaming launch
constexpr int kGramMaxM = 128;            // Gram kernel on 256 threads keeps all rows on chip
constexpr int kGramBigM = 256;            // ... and on kGramBigThreads threads
constexpr int kGramBigThreads = 1024;
constexpr int kGramGroups = 256;          // column groups of the Gram kernel (m_pad^2 partials each)
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU on gfx950
constexpr int kMaxSmall = 256;            // largest Gram / Rayleigh-Ritz eigenproblem
constexpr int kRowChunk = 256;            // row chunk of the A^T Z kernel
constexpr int kSplitTCols = 128;         // tile columns of the split-operand float32 A^T Z kernel
// Block orthonormalisation: at most kOrthMaxGroups row work-groups whose last one sums
// the partials, or, for tall blocks (more 64-row chunks than that), up to kOrthBigGroups
// row work-groups followed by a separate reduction launch.
constexpr int kOrthMaxGroups = 15;
constexpr int kOrthBigGroups = 256;
inline bool orth_big_rows(int64_t m) { return (m + 63) / 64 > kOrthMaxGroups; }

// float64 scratch of the small eigen-solvers: n rows of pitch 256 (plus the tridiagonal
// form and the reflector scalars, 3 x 256) when the matrix no longer fits one work-group's
// LDS (n > 128), nothing otherwise.
inline size_t eig_work_doubles(int n) { return n <= 128 ? 0 : (size_t)(n + 3) * kMaxSmall; }

constexpr int dtype_bytes(int dt) { return dt == TTR_F64 ? 8 : (dt == TTR_F32 ? 4 : 2); }
constexpr int tile_cols(int dt) { return dt == TTR_F64 ? 16 : (dt == TTR_F32 ? 32 : 64); }
inline int pad16(int v) { return (v + 15) / 16 * 16; }
inline int64_t pad_rows(int64_t m, int dt) { return dt == TTR_BF16 ? (m + 31) / 32 * 32 : (m + 15) / 16 * 16; }
inline int acc_bytes(int dt) { return dt == TTR_F64 ? 8 : 4; }

// Rows of one work-group of the row-blocked A W kernel.
constexpr int kAwRows = 256;
// Float32 streams of tall, wide unfoldings (more than one row block of the A W kernel: the
// two-pass Krylov products; at least kMaxGroups / 4 column tiles of the A^T Z kernel, which
// has no row split) multiply on the bf16 matrix cores with three-way split operands.  Their
// W = A^T Z travels between the two passes as three transposed bf16 planes (n x S x 6 bytes).
inline bool split_f32_mode(int dt, int64_t m_pad, int64_t n) {
  return dt == TTR_F32 && m_pad > kAwRows && n >= (int64_t)kSplitTCols * (kMaxGroups / 4);
}
inline int64_t split_w_ld(int64_t n) { return (n + 7) / 8 * 8; }  // row pitch of the W planes

// LDS footprints (bytes) of the streaming kernels.  The kernels carve their
// dynamic shared memory with exactly these pitches:
//   float32/float64: A tile pitch TT+1 elements, Z pitch S, W partials fp32/fp64;
//   bfloat16: row-major A tile pitch TT+8 (the only copy of the tile), transposed Z
//             and W pitch rows+8 and TT+8; no cross-wave partials (each wave forms W
//             for its own 16 tile columns).
inline size_t fused_lds_bytes(int64_t m_pad, int S, int dt) {
  const int tt = tile_cols(dt);
  if (dt == TTR_BF16) return (size_t)m_pad * (tt + 8) * 2 + (size_t)S * (m_pad + 8) * 2 + (size_t)S * (tt + 8) * 2;
  const int b = dtype_bytes(dt);
  return (size_t)m_pad * (tt + 1) * b + (size_t)m_pad * S * b + (size_t)kWaves * tt * S * b;
}
inline size_t aw_lds_bytes(int S, int dt) {
  const int tt = tile_cols(dt);
  if (dt == TTR_BF16) return (size_t)kAwRows * (tt + 8) * 2 + (size_t)S * (tt + 8) * 2;
  const int b = dtype_bytes(dt);
  return (size_t)kAwRows * (tt + 1) * b + (size_t)tt * S * b;
}
constexpr size_t atz_lds_bytes_rc(int S, int dt, int rc) {
  return dt == TTR_BF16
             ? (size_t)rc * (tile_cols(dt) + 8) * 2 + (size_t)S * (rc + 8) * 2
             : (size_t)rc * (tile_cols(dt) + 1) * dtype_bytes(dt) + (size_t)rc * S * dtype_bytes(dt) +
                   (size_t)kWaves * tile_cols(dt) * S * dtype_bytes(dt);
}
// Rows per chunk of the A^T Z kernel: kRowChunk unless the chunk would overflow LDS; for
// float64, half of it when that lets two work-groups share a CU.
constexpr int atz_row_chunk(int S, int dt) {
  if (dt == TTR_F64 && atz_lds_bytes_rc(S, dt, kRowChunk / 2) <= kLdsBytes / 2) return kRowChunk / 2;
  return atz_lds_bytes_rc(S, dt, kRowChunk) <= kLdsBytes ? kRowChunk : kRowChunk / 2;
}
inline size_t atz_lds_bytes(int S, int dt) { return atz_lds_bytes_rc(S, dt, atz_row_chunk(S, dt)); }
inline size_t gram_lds_bytes(int64_t m_pad, int dt) {
  const int tt = tile_cols(dt);
  if (dt == TTR_BF16) return (size_t)m_pad * (tt + 8) * 2;
  return (size_t)m_pad * (tt + 1) * dtype_bytes(dt);
}
// The two Omega tiles of the Gram kernels that also form the sketch (Gram-first modes):
// TT x (S + 1) row-major (float32 / float64), S x (TT + 8) transposed (bfloat16).
inline size_t gram_sketch_lds_bytes(int S, int dt) {
  const int tt = tile_cols(dt);
  if (dt == TTR_BF16) return (size_t)2 * S * (tt + 8) * 2;
  return (size_t)2 * tt * (S + 1) * dtype_bytes(dt);
}
// Gram partials of `groups` work-groups (m_pad x m_pad float64 each), 256-byte aligned so
// that the sketch partials can follow them.
inline size_t gram_part_bytes(int64_t groups, int64_t m_pad) {
  return ((size_t)groups * m_pad * m_pad * 8 + 255) / 256 * 256;
}
// The fused kernel keeps ceil(m_pad/16/4) accumulator blocks per wave, at most 8.
constexpr int kFusedMaxRows = 16 * kWaves * 8;
// float32 unfoldings with kFusedMaxRows < m_pad <= 1024 and S <= 32 use the variant that
// keeps Z in registers; its row count is rounded up to a multiple of 64 (MPK, a multiple
// of 4 rows x 8 waves x 2) and it runs one 512-thread work-group per CU.
constexpr int kFusedZrGroups = 256;
constexpr int kFusedZrTileCols = 16;
inline int64_t fused_zr_rows(int64_t m_pad) { return (m_pad + 63) / 64 * 64; }
inline size_t fused_zr_lds_bytes(int64_t mpk, int S) {
  // A tile of 16 columns (pitch 17), eight partial-W slots and the summed W
  return (size_t)mpk * 17 * 4 + (size_t)9 * 16 * S * 4;
}
inline bool fused_zr_fits(int64_t m_pad, int S, int dt) {
  // S = 16 stops at 896 rows: beyond that its register allocation spills
  const int64_t rows = fused_zr_rows(m_pad);
  return dt == TTR_F32 && m_pad > kFusedMaxRows && S <= 32 && rows <= (S == 16 ? 896 : 1024) &&
         fused_zr_lds_bytes(rows, S) <= kLdsBytes;
}
// Short unfoldings: per-wave carry and Gram kernels (no LDS tiles) for m_pad <= 64.
constexpr int kSmallGroups = 2048;      // work-groups of the short carry kernel
constexpr int kGramSmallGroups = 512;   // work-groups (float64 partials) of the short Gram kernel
inline bool carry_small_fits(int64_t m_pad, int S) { return m_pad <= 64 && S <= 64; }
inline bool fused_fits(int64_t m_pad, int S, int dt) {
  if (fused_zr_fits(m_pad, S, dt)) return true;
  return m_pad <= kFusedMaxRows && S <= 64 && fused_lds_bytes(m_pad, S, dt) <= kLdsBytes;
}
// Bytes of per-group partial results that the streaming launches over an m x n
// unfolding (padded rows m_pad, padded width S) may write: the row-blocked A W, the
// fused product (either variant, when the shape takes it) and, with `gram`, the
// m_pad x m_pad float64 Gram partials.  Every launcher takes its group count from the
// same caps used here.
inline size_t stream_partial_bytes(int64_t n, int64_t m_pad, int S, int dt, bool gram) {
  auto groups = [](int64_t ntiles, int64_t cap) { return ntiles < 1 ? (int64_t)1 : (ntiles < cap ? ntiles : cap); };
  const int64_t ntiles = (n + tile_cols(dt) - 1) / tile_cols(dt);
  const int64_t rb = (m_pad + kAwRows - 1) / kAwRows;
  const size_t ab = acc_bytes(dt);
  const size_t row = (size_t)m_pad * S * ab;
  size_t part = (size_t)groups(ntiles, kMaxGroups / rb > 1 ? kMaxGroups / rb : 1) * row;
  if (fused_zr_fits(m_pad, S, dt))
    part = std::max(part, (size_t)groups((n + kFusedZrTileCols - 1) / kFusedZrTileCols, kFusedZrGroups) * row);
  else if (fused_fits(m_pad, S, dt))
    part = std::max(part, (size_t)groups(ntiles, kMaxGroups) * row);
  if (gram) part = std::max(part, (size_t)groups(ntiles, kMaxGroups) * m_pad * m_pad * 8);
  return part;
}

// Partials of the Gram-and-sketch pass over an m x n unfolding: the Gram partials, then
// m_pad x S sketch partials per work-group (accumulation type of the dtype).
inline size_t gram_sketch_partial_bytes(int64_t n, int64_t m_pad, int S, int dt) {
  const int64_t ntiles = (n + tile_cols(dt) - 1) / tile_cols(dt);
  const int64_t groups = ntiles < 1 ? 1 : (ntiles < kGramGroups ? ntiles : kGramGroups);
  return gram_part_bytes(groups, m_pad) + (size_t)groups * m_pad * S * acc_bytes(dt);
}

struct ModeGeom {
  int k;           // mode index, 1-based
  int64_t m, n;    // unfolding is m x n
  int r, s, S, w;  // rank, sketch width, padded width, Krylov width (q+1)*s
  int kind;        // TTR_MODE_*
  int two_pass;    // Krylov products by A^T Z then A W (rows too many for one pass)
  int method;      // TTR_METHOD_* (regular modes of the Rayleigh-Ritz TT-RBKI: run_regular;
                   // every other regular mode: the power-block driver)
  int literal;     // 1: first-r-columns truncation as printed
  int gram_first;  // regular TT-RBKI mode whose products go through the m x m Gram A A^T
  int b;           // block width of the power-block driver: r (literal) or s
  int iters;       // its renormalised products after the sketch
  int a_dtype;     // storage of A_k (X's dtype for k = 1 and after identity modes)
  double tau;      // drop threshold of this mode (from a_dtype unless the caller set one)
  int64_t m_pad;
};

// Byte offsets of every workspace region (all 256-aligned).  The first 256 bytes hold the
// status word (non-finite flag) that ttr_check reads, at the same offset in the forward and
// the gradient workspace.
constexpr size_t kStatusOffset = 0;
struct Layout {
  size_t carry[2];     // carry ping-pong, carry dtype
  size_t wbuf;         // n x S stream buffer (Omega or A^T Z)
  size_t partials;     // per-work-group partial results
  size_t partials_bytes;
  size_t zs;           // m_pad x S stream copy of the current block
  size_t ybuf;         // m x s float64 raw block
  size_t yall;         // m x (q+1) s float64: A A^T Q_j for j = 0..q
  size_t qbuf;         // m x w float64 orthonormal Krylov basis (zero = dropped)
  size_t gram;         // m x m float64 Gram A A^T of the Gram-first modes
  size_t pbuf;         // m x s float64 projected block
  size_t small;        // small float64 matrices (Gram, eigenvectors, transforms)
  size_t small_bytes;
  size_t orth_big;     // partials of the tall-block orthonormalisation (0 bytes if unused):
  size_t orth_big_bytes;  // kOrthBigGroups x w s, then kOrthBigGroups norms, then 64 x 64 (gsum)
  int small_ne;         // side of the square float64 matrices carved from `small`
  size_t total;
};

// Workspace of the gradient entry: the forward layout, a tape per mode and the
// reverse-sweep scratch (byte offsets, 256-aligned).
struct GradLayout {
  size_t base;                     // forward Layout occupies [0, base)
  size_t tQ[TTR_MAX_D], tY[TTR_MAX_D], tT[TTR_MAX_D], tU[TTR_MAX_D], tL[TTR_MAX_D], tI[TTR_MAX_D];
  size_t tC[TTR_MAX_D];            // carries C_k
  size_t cores[TTR_MAX_D];         // float64 cores G_1 .. G_d of the forward sweep
  size_t cbar[2];                  // adjoints of the carries (carry dtype)
  size_t wt;                       // n x R transposed carry adjoint (dtype of A_k)
  size_t gpart;                    // partial sums of the A W launch with R columns
  size_t gpart_bytes;
  size_t splitk;                   // split-K partials of the small X^T Y products
  size_t gb, ub, qb, mb, vv, qmb, kbar, ktil, ktildt, zb, cl, mq, pb, hh, qtpb, yb, ktmp;
  size_t parts, scal, ints, lb, wb, abtmp, cbar64, symnb;
  size_t err3, errws;              // streamed ||X - Xhat||^2 (the loss) and its scratch
  size_t total;
};
struct Plan {
  ttr_plan_t pub;
  ModeGeom modes[TTR_MAX_D];
  Layout lay;
  GradLayout glay;
  bool grad_ok;                    // shapes and dtype supported by the gradient entry
};

// Largest regular-mode row count supported by the gradient entry (m x m adjoint Gram).
constexpr int64_t kGradMaxM = 4096;

// Validates arguments and fills a plan (host only, no HIP calls).
int make_plan(int32_t d, const int64_t* dims, const int64_t* target_ranks, int32_t q, int32_t p,
              int32_t x_dtype, const ttr_options* opt, Plan* out);

// Split of the streaming reconstruction error: the smallest s >= 1 whose trailing block
// prod_{k>s} I_k has at most 2^20 entries (its size in *inner), and the scratch bytes.
int error_split(int32_t d, const int64_t* dims, int64_t* inner);
size_t tt_error_ws_bytes(int32_t d, const int64_t* dims, const int64_t* ranks);

// Workspace needs of a single block call (m x n matrix, cols <= 64 columns).
size_t block_workspace(int64_t m, int64_t n, int cols, int dt);

void set_error(const std::string& msg);

// Number of column groups a streaming launch uses for ntiles column tiles.
inline int64_t groups_for(int64_t ntiles, int64_t cap) {
  int64_t g = ntiles < cap ? ntiles : cap;
  return g < 1 ? 1 : g;
}

}  // namespace ttr
