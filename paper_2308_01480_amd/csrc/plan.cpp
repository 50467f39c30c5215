// Host-only planning of a TT-RBKI sweep: argument validation, rank clamping, mode
// classification and workspace layout.  No HIP calls, so it runs without a GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "common.h"

namespace ttr {

static thread_local std::string g_detail;

void set_error(const std::string& msg) { g_detail = msg; }

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  if (a < 0 || b < 0) return false;
  if (a != 0 && b > INT64_MAX / a) return false;
  *out = a * b;
  return true;
}

// Default drop threshold of a mode, from the arithmetic that forms its Krylov blocks
// (Algorithm 3, step 5, read as a pivoted economy QR): float64 streams accumulate in
// float64; float32 and bfloat16 streams both accumulate in float32 (a bf16 stream rounds
// the streamed operand, but every computed column is still A times a vector).
static double default_tau(int dt) { return dt == TTR_F64 ? 1e-10 : 1e-5; }

// Partial-result bytes of the streaming launches of one regular / saturated mode.
static size_t mode_partials(const ModeGeom& g) {
  if (g.kind == TTR_MODE_REGULAR)
    return std::max({stream_partial_bytes(g.n, g.m_pad, g.S, g.a_dtype, g.gram_first != 0),
                     stream_partial_bytes(g.n, g.m_pad, pad16(g.b), g.a_dtype, false),
                     g.gram_first ? gram_sketch_partial_bytes(g.n, g.m_pad, g.S, g.a_dtype) : (size_t)0});
  if (g.kind == TTR_MODE_SATURATED && g.m <= g.n) {
    const int tt = tile_cols(g.a_dtype);
    return (size_t)groups_for((g.n + tt - 1) / tt, kMaxGroups) * g.m_pad * g.m_pad * 8;
  }
  return 0;
}

// Gradient workspace: forward layout, one tape per mode, reverse scratch.
static void grad_layout(Plan* pl) {
  const ttr_plan_t& P = pl->pub;
  GradLayout& G = pl->glay;
  std::memset(&G, 0, sizeof(G));
  const size_t cb = (size_t)dtype_bytes(P.carry_dtype);
  size_t off = pl->lay.total;
  G.base = off;
  int64_t M1 = 1, E1 = 1, W1 = 64, N1 = 1, MN1 = 1;
  size_t cbar_max = 0, wt_max = 0, gpart_max = 0;
  pl->grad_ok = P.x_dtype != TTR_BF16 && P.method == TTR_METHOD_RBKI && !P.literal;
  for (int k = 1; k < P.d; ++k) {
    const ModeGeom& g = pl->modes[k - 1];
    if (g.kind == TTR_MODE_IDENTITY) continue;
    const int64_t e = g.kind == TTR_MODE_REGULAR ? g.w : std::min(g.m, g.n);
    if (g.kind == TTR_MODE_REGULAR && g.m > kGradMaxM) pl->grad_ok = false;
    const int64_t mw = g.kind == TTR_MODE_REGULAR ? g.m * g.w : 0;
    G.tQ[k - 1] = off; off = align256(off + (size_t)mw * 8);
    G.tY[k - 1] = off; off = align256(off + (size_t)mw * 8);
    G.tT[k - 1] = off; off = align256(off + (size_t)(P.q + 1) * 64 * 64 * 8);
    G.tU[k - 1] = off; off = align256(off + (size_t)e * e * 8);
    G.tL[k - 1] = off; off = align256(off + (size_t)e * 8);
    G.tI[k - 1] = off; off = align256(off + (size_t)(P.q + 2) * 4);
    G.tC[k - 1] = off; off = align256(off + (size_t)g.r * g.n * cb);
    M1 = std::max(M1, g.m);
    E1 = std::max(E1, e);
    if (g.kind == TTR_MODE_REGULAR) W1 = std::max<int64_t>(W1, g.w);
    if (g.kind == TTR_MODE_SATURATED && g.n < g.m) { N1 = std::max(N1, g.n); MN1 = std::max(MN1, g.m * g.n); }
    if (k >= 2) cbar_max = std::max(cbar_max, (size_t)(g.m * g.n));
    const int R = pad16(g.r);
    wt_max = std::max(wt_max, (size_t)g.n * R * dtype_bytes(g.a_dtype));
    const int64_t tt = tile_cols(g.a_dtype), ntiles = (g.n + tt - 1) / tt;
    const int64_t rb = (g.m_pad + kAwRows - 1) / kAwRows;
    gpart_max = std::max(gpart_max, (size_t)groups_for(ntiles, std::max<int64_t>(1, kMaxGroups / rb)) * g.m_pad * R *
                                        acc_bytes(g.a_dtype));
  }
  for (int k = 1; k <= P.d; ++k) { G.cores[k - 1] = off; off = align256(off + (size_t)P.core_elems[k - 1] * 8); }
  cbar_max = std::max(cbar_max, (size_t)(P.ranks[P.d - 1] * P.dims[P.d - 1]));
  G.cbar[0] = off; off = align256(off + cbar_max * cb);
  G.cbar[1] = off; off = align256(off + cbar_max * cb);
  G.wt = off; off = align256(off + wt_max);
  G.gpart = off; off = align256(off + gpart_max);
  G.gpart_bytes = gpart_max;
  G.splitk = off; off = align256(off + (size_t)15 * std::max(W1, E1) * 64 * 8);
  const size_t m64 = (size_t)M1 * 64 * 8, mw = (size_t)M1 * W1 * 8, mm = (size_t)M1 * M1 * 8;
  G.gb = off; off = align256(off + m64);
  G.ub = off; off = align256(off + (size_t)E1 * 64 * 8);
  G.qb = off; off = align256(off + mw);
  G.mb = off; off = align256(off + (size_t)E1 * E1 * 8);
  G.vv = off; off = align256(off + (size_t)E1 * 64 * 8);
  G.qmb = off; off = align256(off + std::max(mw, (size_t)N1 * N1 * 8));
  G.kbar = off; off = align256(off + mm);
  G.ktil = off; off = align256(off + std::max(mm, (size_t)MN1 * 8));
  G.ktildt = off; off = align256(off + (size_t)(M1 + 32) * 64 * 8);
  G.zb = off; off = align256(off + m64);
  G.cl = off; off = align256(off + 64 * 64 * 8);
  G.mq = off; off = align256(off + 64 * 64 * 8);
  G.pb = off; off = align256(off + m64);
  G.hh = off; off = align256(off + (size_t)W1 * 64 * 8);
  G.qtpb = off; off = align256(off + (size_t)W1 * 64 * 8);
  G.yb = off; off = align256(off + m64);
  G.ktmp = off; off = align256(off + m64);
  G.parts = off; off = align256(off + 1024 * 8);
  G.scal = off; off = align256(off + 64 * 8);
  G.ints = off; off = align256(off + 64 * 4);
  G.lb = off; off = align256(off + 64 * 8);
  G.wb = off; off = align256(off + (size_t)N1 * 64 * 8);
  G.abtmp = off; off = align256(off + (size_t)MN1 * 8);
  G.cbar64 = off; off = align256(off + (size_t)N1 * 64 * 8);
  G.symnb = off; off = align256(off + (size_t)N1 * N1 * 8);
  G.err3 = off; off = align256(off + 3 * 8);
  G.errws = off; off = align256(off + tt_error_ws_bytes(P.d, P.dims, P.ranks));
  G.total = off;
  pl->pub.grad_workspace_bytes = pl->grad_ok ? off : 0;
}

int make_plan(int32_t d, const int64_t* dims, const int64_t* target_ranks, int32_t q, int32_t p,
              int32_t x_dtype, const ttr_options* opt, Plan* out) {
  if (!out || !dims || !target_ranks) { set_error("null pointer argument"); return TTR_EINVAL; }
  if (d < 2 || d > TTR_MAX_D) { set_error("d must be in [2, 64]"); return TTR_EINVAL; }
  if (q < 0 || p < 0) { set_error("q and p must be >= 0"); return TTR_EINVAL; }
  if (x_dtype != TTR_F64 && x_dtype != TTR_F32 && x_dtype != TTR_BF16) {
    set_error("unknown dtype"); return TTR_EINVAL;
  }
  const int method = opt ? opt->method : TTR_METHOD_RBKI;
  const int literal = opt ? opt->literal : 0;
  if (method < TTR_METHOD_RBKI || method > TTR_METHOD_RSVD || (literal != 0 && literal != 1)) {
    set_error("unknown method or literal flag"); return TTR_EINVAL;
  }
  if (method == TTR_METHOD_RBKI && literal && q < 1) {
    set_error("TT-RBKI as printed needs q >= 1 (its Krylov matrix has q blocks)"); return TTR_EINVAL;
  }
  std::memset(out, 0, sizeof(*out));
  ttr_plan_t& P = out->pub;
  P.d = d; P.q = q; P.p = p; P.x_dtype = x_dtype;
  P.method = method; P.literal = literal;
  const bool krylov_rr = method == TTR_METHOD_RBKI && !literal;
  const int kform = opt ? opt->krylov_form : TTR_KRYLOV_AUTO;
  if (kform < TTR_KRYLOV_AUTO || kform > TTR_KRYLOV_GRAM) { set_error("unknown krylov_form"); return TTR_EINVAL; }
  P.carry_dtype = x_dtype == TTR_F64 ? TTR_F64 : TTR_F32;
  const bool user_tau = opt && opt->tau > 0;
  P.tau = user_tau ? opt->tau : default_tau(x_dtype);
  int64_t numel = 1;
  for (int i = 0; i < d; ++i) {
    if (dims[i] <= 0) { set_error("dims must be positive"); return TTR_EINVAL; }
    if (!mul_ok(numel, dims[i], &numel)) { set_error("numel overflows int64"); return TTR_EINVAL; }
    P.dims[i] = dims[i];
  }
  for (int i = 0; i < d - 1; ++i)
    if (target_ranks[i] <= 0) { set_error("target ranks must be positive"); return TTR_EINVAL; }

  P.ranks[0] = 1;
  int64_t rest = numel;
  int a_dtype = x_dtype;
  size_t max_carry = 0, max_wbuf = 0, max_part = 0, max_zs = 0, max_ms = 0, max_mq = 0, max_mw = 0, max_gram = 0;
  size_t max_orth_len = 0;  // largest partial of a tall block's orthonormalisation step (doubles)
  int max_small = 1;
  int64_t max_m = 1;
  for (int k = 1; k < d; ++k) {
    ModeGeom& g = out->modes[k - 1];
    g.k = k;
    rest /= dims[k - 1];
    g.n = rest;
    if (!mul_ok(P.ranks[k - 1], dims[k - 1], &g.m)) { set_error("m overflows"); return TTR_EINVAL; }
    int64_t r = std::min<int64_t>(target_ranks[k - 1], std::min<int64_t>(g.m, g.n));
    if (r > 64) { set_error("ranks above 64 are not supported"); return TTR_EUNSUPPORTED; }
    g.r = (int)r;
    g.s = g.r + p;
    g.method = method;
    g.literal = literal;
    // width of the final basis: the block Krylov space, or one block of the power driver
    g.b = literal ? g.r : g.s;
    g.iters = method == TTR_METHOD_RSVD ? 0 : (method == TTR_METHOD_RBKI ? 1 : q);
    g.w = krylov_rr ? (q + 1) * g.s : g.b;
    g.S = pad16(g.s);
    g.a_dtype = a_dtype;
    g.tau = user_tau ? opt->tau : default_tau(a_dtype);
    g.m_pad = pad_rows(g.m, a_dtype);
    // identity: G = I; saturated: the final basis spans range(A), so the exact truncated SVD
    // gives the same tensor (for the printed truncation this needs r = n < m)
    if (r == g.m) g.kind = TTR_MODE_IDENTITY;
    else if (literal ? r == g.n : (int64_t)g.w >= std::min(g.m, g.n)) g.kind = TTR_MODE_SATURATED;
    else g.kind = TTR_MODE_REGULAR;
    if (g.kind == TTR_MODE_REGULAR) {
      if (g.S > 64) { set_error("r + p above 64 is not supported"); return TTR_EUNSUPPORTED; }
      if (g.w > kMaxSmall) { set_error("(q+1)(r+p) above 256 is not supported"); return TTR_EUNSUPPORTED; }
      g.two_pass = fused_fits(g.m_pad, krylov_rr ? g.S : pad16(g.b), a_dtype) ? 0 : 1;
      // Gram-first: one pass forms A A^T (about m_pad (m_pad + 16) n flops on 16 x 16 blocks),
      // against q + 1 streamed products of 4 S m n flops; float32 input takes the Gram in
      // float64 products, at half the float32 matrix-core rate
      const int64_t krylov_flops = (int64_t)4 * g.S * (q + 1) / (a_dtype == TTR_F32 ? 2 : 1);
      if (krylov_rr && g.m_pad <= kGramBigM && kform != TTR_KRYLOV_STREAMED)
        g.gram_first = (kform == TTR_KRYLOV_GRAM || g.m_pad + 16 <= krylov_flops) ? 1 : 0;
      if (g.gram_first) max_gram = std::max(max_gram, (size_t)g.m * g.m * 8);
      if (orth_big_rows(g.m)) max_orth_len = std::max(max_orth_len, (size_t)g.w * std::max(g.s, g.b));
      max_wbuf = std::max(max_wbuf, split_f32_mode(a_dtype, g.m_pad, g.n) ? (size_t)6 * g.S * split_w_ld(g.n) : (size_t)g.n * g.S * dtype_bytes(a_dtype));
      max_mq = std::max(max_mq, (size_t)g.m * g.w * 8);
      max_small = std::max(max_small, g.w);
    } else if (g.kind == TTR_MODE_SATURATED) {
      const int64_t sh = std::min(g.m, g.n);
      if (g.m <= g.n && g.m_pad > kGramBigM) {
        set_error("saturated modes with m <= n need m <= 256"); return TTR_EUNSUPPORTED;
      }
      if (sh > kMaxSmall) { set_error("saturated short side above 256"); return TTR_EUNSUPPORTED; }
      max_small = std::max<int>(max_small, (int)sh);
      if (g.m > g.n) max_mw = std::max(max_mw, (size_t)g.m * g.n * 8);
    }
    P.m[k - 1] = g.m; P.n[k - 1] = g.n; P.s[k - 1] = g.s; P.w[k - 1] = g.w;
    P.kind[k - 1] = g.kind; P.two_pass[k - 1] = g.two_pass; P.gram_first[k - 1] = g.gram_first;
    P.ranks[k] = g.r;
    if (g.kind != TTR_MODE_IDENTITY) {
      max_carry = std::max(max_carry, (size_t)g.r * g.n);
      a_dtype = P.carry_dtype;
      max_zs = std::max(max_zs, (size_t)g.m_pad * 64 * dtype_bytes(g.a_dtype));
      max_ms = std::max(max_ms, (size_t)g.m * 64 * 8);
      max_part = std::max(max_part, mode_partials(g));
      max_m = std::max(max_m, g.m);
    }
  }
  P.ranks[d] = 1;
  for (int k = 1; k <= d; ++k) P.core_elems[k - 1] = P.ranks[k - 1] * dims[k - 1] * P.ranks[k];

  Layout& L = out->lay;
  size_t off = align256(kStatusOffset + sizeof(int));
  const size_t cb = (size_t)dtype_bytes(P.carry_dtype);
  L.carry[0] = off; off = align256(off + max_carry * cb);
  L.carry[1] = off; off = align256(off + max_carry * cb);
  L.wbuf = off; off = align256(off + max_wbuf);
  L.partials = off; off = align256(off + max_part);
  L.partials_bytes = max_part;
  L.zs = off; off = align256(off + max_zs);
  L.ybuf = off; off = align256(off + max_ms);
  L.yall = off; off = align256(off + std::max(max_mq, max_mw));
  L.qbuf = off; off = align256(off + max_mq);
  L.gram = off; off = align256(off + max_gram);
  L.pbuf = off; off = align256(off + max_ms);
  // small: 6 square n_e x n_e float64 matrices (eigen work takes two), 15 for split-K partials, scalars
  const size_t ne = (size_t)std::max(max_small, 64);
  L.small_ne = (int)ne;
  L.small_bytes = align256((21 * ne * ne + 3 * kMaxSmall) * 8 + 4096 * 8);
  L.small = off; off = align256(off + L.small_bytes);
  L.orth_big_bytes = max_orth_len ? align256(((size_t)kOrthBigGroups * (max_orth_len + 1) + 64 * 64) * 8) : 0;
  L.orth_big = off; off = align256(off + L.orth_big_bytes);
  L.total = off;
  P.workspace_bytes = off;
  (void)max_m;
  grad_layout(out);
  return TTR_OK;
}

int error_split(int32_t d, const int64_t* dims, int64_t* inner_out) {
  // smallest split s >= 1 whose inner block prod_{k>s} I_k is at most 2^20 entries
  int s = d - 1;
  for (int cand = 1; cand <= d - 1; ++cand) {
    int64_t inner = 1;
    for (int k = cand; k < d; ++k) inner *= dims[k];
    if (inner <= (int64_t(1) << 20)) { s = cand; break; }
  }
  int64_t inner = 1;
  for (int k = s; k < d; ++k) inner *= dims[k];
  *inner_out = inner;
  return s;
}

size_t tt_error_ws_bytes(int32_t d, const int64_t* dims, const int64_t* ranks) {
  int64_t inner = 0;
  const int s = error_split(d, dims, &inner);
  int64_t rmax = 1;
  for (int k = s; k <= d; ++k) rmax = std::max(rmax, ranks[k]);
  int64_t outer = 1;
  for (int k = 0; k < s; ++k) outer *= dims[k];
  return 2 * align256((size_t)rmax * inner * 8) + align256((size_t)outer * 3 * 8);
}

size_t block_workspace(int64_t m, int64_t n, int cols, int dt) {
  const int S = pad16(std::max(cols, 1));
  const int64_t m_pad = pad_rows(m, dt);
  size_t off = 0;
  off = align256(off + (size_t)n * S * dtype_bytes(dt));                         // wbuf
  size_t part = stream_partial_bytes(n, m_pad, S, dt, m_pad <= kGramBigM);
  if (m_pad <= kGramBigM) part = std::max(part, gram_sketch_partial_bytes(n, m_pad, S, dt));
  off = align256(off + part);                                                    // partials
  off = align256(off + (size_t)m_pad * S * dtype_bytes(dt));                     // zs
  return off;
}

}  // namespace ttr

extern "C" {

int ttr_plan(int32_t d, const int64_t* dims, const int64_t* target_ranks, int32_t q, int32_t p,
             int32_t x_dtype, const ttr_options* opt, ttr_plan_t* out) {
  if (!out) { ttr::set_error("null plan output"); return TTR_EINVAL; }
  ttr::Plan pl;
  int rc = ttr::make_plan(d, dims, target_ranks, q, p, x_dtype, opt, &pl);
  if (rc == TTR_OK) *out = pl.pub;
  return rc;
}

size_t ttr_block_workspace(int64_t m, int64_t n, int32_t cols, int32_t a_dtype) {
  if (m <= 0 || n <= 0 || cols <= 0 || cols > 64) return 0;
  return ttr::block_workspace(m, n, cols, a_dtype);
}

const char* ttr_strerror(int code) {
  switch (code) {
    case TTR_OK: return "ok";
    case TTR_EINVAL: return "invalid argument";
    case TTR_EWORKSPACE: return "workspace too small";
    case TTR_EHIP: return "HIP runtime error";
    case TTR_ENUMERIC: return "non-finite values";
    case TTR_EUNSUPPORTED: return "unsupported shape";
    default: return "unknown error";
  }
}

const char* ttr_last_error_detail(void) { return ttr::g_detail.c_str(); }

}  // extern "C"
