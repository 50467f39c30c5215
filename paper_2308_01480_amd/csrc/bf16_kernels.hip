// bfloat16 storage: the streaming kernels on v_mfma_f32_16x16x32_bf16 (float32 accumulation).
//
// A bf16 matrix-core operand holds 8 consecutive k values per lane.  The A tile is kept
// in LDS once, row-major (Ar: rows x TT+8, k = column), and read two ways:
//   products contracting over columns read one 16-byte load per operand (ld8);
//   products contracting over rows read it with the gfx950 LDS transpose load (ld8_tr),
//   so no transposed copy of the tile is written.
// Zt is transposed Z (S x rows+8), Wt transposed W (S x TT+8).
// The tile is TT = 64 columns; rows are padded to a multiple of 32.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "omega.h"

namespace ttr {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16;

constexpr int BT = 64;            // tile columns
constexpr int BRP = BT + 8;       // row-major tile pitch (bf16 elements)

__device__ inline f4_t mma_bf16(const bf8_t& a, const bf8_t& b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline bf8_t ld8(const bf16* p) { return *reinterpret_cast<const bf8_t*>(p); }
__device__ inline f4_t fzero() { return f4_t{0.f, 0.f, 0.f, 0.f}; }
__device__ inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Register staging of a rows x 64 tile: 8 bf16 (16 bytes) per vector, 8 vectors per row.
template <int MAXV, int NTH = kThreads>
struct BTile {
  u4_t v[MAXV];
  __device__ void fetch(const bf16* __restrict__ A, int64_t m, int64_t n, int64_t row0, int rows, int64_t col0,
                        bool aligned) {
    const int nv = rows * 8;
    const bool full = aligned && (col0 + BT <= n);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = (int)threadIdx.x + i * NTH;
      u4_t val = u4_t{0u, 0u, 0u, 0u};
      if (idx < nv) {
        const int rr = idx >> 3, cv = idx & 7;
        const int64_t row = row0 + rr;
        if (row < m) {
          const bf16* src = A + row * n + col0 + cv * 8;
          if (full) {
            val = *reinterpret_cast<const u4_t*>(src);
          } else {
            bf16 tmp[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) tmp[e] = (col0 + cv * 8 + e < n) ? src[e] : (bf16)0.0f;
            val = *reinterpret_cast<u4_t*>(tmp);
          }
        }
      }
      v[i] = val;
    }
  }
  // Ar (rows x BRP).
  __device__ void commit(bf16* __restrict__ Ar, int rows) const {
    const int nv = rows * 8;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = (int)threadIdx.x + i * NTH;
      if (idx < nv) *reinterpret_cast<u4_t*>(Ar + (idx >> 3) * BRP + (idx & 7) * 8) = v[i];
    }
  }
};

// Operand of 8 consecutive rows of one tile column per lane, from the row-major tile,
// with the gfx950 LDS transpose load: within each group of 16 lanes, lane 4a + b receives
// element b of the 64-bit words loaded by lanes a, a + 4, a + 8, a + 12.  So lane (e, a)
// of the group passes the address of columns 4a..4a+3 of row e, and lane 4a + b comes out
// holding column 4a + b of rows 0..3; a second load 4 rows further gives rows 4..7.
__device__ inline bf8_t ld8_tr(const bf16* p) {
  typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) bf4_t lds_bf4;
  const bf4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf4*)(p));
  const bf4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf4*)(p + 4 * BRP));
  return bf8_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// Phase 1, per wave: acc1[sb] (16 beta x 16 c) += A_J^T Zt^T over the tile rows, for the
// tile columns [16 wave, 16 wave + 16) (A_J read from the row-major tile by transpose
// loads).  Lane (q, i) holds W[16 wave + 4 q + r][16 sb + i] in acc1[sb][r].
template <int SB>
__device__ inline void b_phase1_wave(const bf16* __restrict__ Ar, const bf16* __restrict__ Zt, int rows, int zp,
                                     f4_t (&acc1)[SB]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bf16* Asrc = Ar + (8 * (lane >> 4) + ((lane >> 2) & 3)) * BRP + wave * 16 + 4 * (lane & 3);
  for (int ks = 0; ks < rows / 32; ++ks) {
    const int k0 = ks * 32 + 8 * (lane >> 4);
    const bf8_t av = ld8_tr(Asrc + ks * 32 * BRP);
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc1[sb] = mma_bf16(av, ld8(Zt + (sb * 16 + (lane & 15)) * zp + k0), acc1[sb]);
  }
}

// Phase 2: acc2[i][sb] (16 rows x 16 c) += Ar (rows x BT) Wt^T (BT x S).
template <int SB, int APW>
__device__ inline void b_phase2(const bf16* __restrict__ Ar, const bf16* __restrict__ Wt, int rows,
                                f4_t (&acc2)[APW][SB]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int ks = 0; ks < BT / 32; ++ks) {
    const int k0 = ks * 32 + 8 * (lane >> 4);
    bf8_t b[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) b[sb] = ld8(Wt + (sb * 16 + (lane & 15)) * BRP + k0);
#pragma unroll
    for (int i = 0; i < APW; ++i) {
      const int ab = wave + kWaves * i;
      if (ab * 16 < rows) {
        const bf8_t a = ld8(Ar + (ab * 16 + (lane & 15)) * BRP + k0);
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = mma_bf16(a, b[sb], acc2[i][sb]);
      }
    }
  }
}

template <int SB, int APW>
__device__ inline void b_store_rows(f4_t (&acc2)[APW][SB], float* __restrict__ out, int rows, int row_off) {
  constexpr int S = SB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < APW; ++i) {
    const int ab = wave + kWaves * i;
    if (ab * 16 < rows)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(int64_t)(row_off + ab * 16 + 4 * (lane >> 4) + r) * S + sb * 16 + (lane & 15)] = acc2[i][sb][r];
  }
}

// Z (rows x S, row-major, global) -> Zt (S x rows+8) in LDS.
template <int S>
__device__ inline void load_zt(const bf16* __restrict__ Zg, int rows, int zp, bf16* __restrict__ Zt) {
  for (int e = threadIdx.x; e < rows * S; e += kThreads) {
    const int rr = e / S, c = e % S;
    Zt[c * zp + rr] = Zg[e];
  }
}

// ----------------------------------------------------------------------------------
// Fused single pass: partial[g] (m_pad x S, float) = sum_J A_J (A_J^T Z).
// ----------------------------------------------------------------------------------
template <int SB, int APW>
__global__ __launch_bounds__(kThreads) void kb_fused(const bf16* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                     const bf16* __restrict__ Zg, float* __restrict__ part,
                                                     int64_t tiles_per_group, int64_t ntiles) {
  constexpr int S = SB * 16;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tp = m_pad + 8;
  bf16* Ar = reinterpret_cast<bf16*>(smem);
  bf16* Zt = Ar + m_pad * BRP;
  bf16* Wt = Zt + S * tp;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = aligned16(A) && ((n * 2) % 16 == 0);

  load_zt<S>(Zg, m_pad, tp, Zt);
  f4_t acc2[APW][SB];
#pragma unroll
  for (int i = 0; i < APW; ++i)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = fzero();
  BTile<2 * APW> regs;
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad, t0 * BT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(Ar, m_pad);
    __syncthreads();
    if (t + 1 < t1) regs.fetch(A, m, n, 0, m_pad, (t + 1) * BT, aligned);
    static_assert(BT == 16 * kWaves, "one 16-column block of W per wave");
    // Phase 1 without a cross-wave sum: wave w forms W for tile columns [16 w, 16 w + 16)
    // over all rows, and stores it rounded to bf16 into Wt, two columns per 32-bit word.
    {
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      // transpose-load source: row 8 (lane / 16) + (lane / 4) % 4 of the K-step, columns
      // 16 wave + 4 (lane % 4) .. + 3
      const bf16* Asrc = Ar + (8 * (lane >> 4) + ((lane >> 2) & 3)) * BRP + wave * 16 + 4 * (lane & 3);
      f4_t acc1[SB];
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc1[sb] = fzero();
      for (int ks = 0; ks < m_pad / 32; ++ks) {
        const int k0 = ks * 32 + 8 * (lane >> 4);
        const bf8_t av = ld8_tr(Asrc + ks * 32 * BRP);
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc1[sb] = mma_bf16(av, ld8(Zt + (sb * 16 + (lane & 15)) * tp + k0), acc1[sb]);
      }
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int rp = 0; rp < 2; ++rp) {
          const int bb = wave * 16 + 4 * (lane >> 4) + 2 * rp, c = sb * 16 + (lane & 15);
          bf16 two[2];
          two[0] = (bf16)acc1[sb][2 * rp];
          two[1] = (bf16)acc1[sb][2 * rp + 1];
          *reinterpret_cast<uint32_t*>(Wt + c * BRP + bb) = *reinterpret_cast<const uint32_t*>(two);
        }
    }
    __syncthreads();
    b_phase2<SB, APW>(Ar, Wt, m_pad, acc2);
  }
  b_store_rows<SB, APW>(acc2, part + g * (int64_t)m_pad * S, m_pad, 0);
}

// ----------------------------------------------------------------------------------
// Sketch A Omega_k inside the Gram pass of a Gram-first mode.  The Omega rows of a tile
// are drawn (omega.h) straight into a transposed LDS tile Ot (S x BRP, the layout of Wt),
// double-buffered so that the next tile's rows are drawn while the current one is used.
// Sketch tile p = rank + nranks i of the (m_pad / 16) x SKB grid accumulates in float32
// over the work-group's columns, as the A W kernel does.
// ----------------------------------------------------------------------------------
// Zero the rows c >= 8 ceil(s / 8) of both transposed Omega tiles (never drawn); the
// `nthr` calling threads have ids tid = 0 .. nthr-1.
template <int SKB>
__device__ inline void b_sketch_init(bf16* __restrict__ Ot, int s, int tid, int nthr) {
  constexpr int S = SKB * 16;
  const int cz = 8 * ((s + 7) / 8);
  for (int e = tid; e < 2 * S * BRP; e += nthr)
    if ((e / BRP) % S >= cz) Ot[e] = (bf16)0.0f;
}

template <int SKB, int SPW>
__device__ inline void b_sketch_tiles(const bf16* __restrict__ Ar, const bf16* __restrict__ Ot, int MB, int rank,
                                      int nranks, f4_t (&yacc)[SPW]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int ks = 0; ks < BT / 32; ++ks) {
    const int k0 = ks * 32 + 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
      const int p = rank + nranks * i;
      if (p < MB * SKB) {
        const int rb = p / SKB, cb = p - rb * SKB;
        yacc[i] = mma_bf16(ld8(Ar + (rb * 16 + (lane & 15)) * BRP + k0), ld8(Ot + (cb * 16 + (lane & 15)) * BRP + k0),
                           yacc[i]);
      }
    }
  }
}

template <int SKB, int SPW>
__device__ inline void b_sketch_store(const f4_t (&yacc)[SPW], float* __restrict__ out, int MB, int rank, int nranks) {
  constexpr int S = SKB * 16;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < SPW; ++i) {
    const int p = rank + nranks * i;
    if (p < MB * SKB) {
      const int rb = p / SKB, cb = p - rb * SKB;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(rb * 16 + 4 * (lane >> 4) + r) * S + cb * 16 + (lane & 15)] = yacc[i][r];
    }
  }
}

// ----------------------------------------------------------------------------------
// Row-blocked A W: partial[g] rows [rb*256, +256) += A_J W_J, W (n x S) bf16.  With OM
// the W tile is Omega_k drawn inside the kernel (omega.h) into a double-buffered
// transposed LDS tile (one row block: m_pad <= 256), so Omega never reaches HBM.
// ----------------------------------------------------------------------------------
template <int SB, bool OM = false>
__global__ __launch_bounds__(kThreads) void kb_aw(const bf16* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                  const bf16* __restrict__ W, float* __restrict__ part,
                                                  int64_t tiles_per_group, int64_t ntiles, uint64_t seed, int kmode,
                                                  int s) {
  constexpr int S = SB * 16;
  constexpr int APW = kAwRows / (16 * kWaves);
  constexpr int OT = S * BRP;
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* Ar = reinterpret_cast<bf16*>(smem);
  bf16* Wt = Ar + kAwRows * BRP;  // OM: two transposed Omega tiles
  const int64_t g = blockIdx.x;
  const int row0 = blockIdx.y * kAwRows;
  const int rows = (m_pad - row0) < kAwRows ? (m_pad - row0) : kAwRows;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = aligned16(A) && ((n * 2) % 16 == 0);
  f4_t acc2[APW][SB];
#pragma unroll
  for (int i = 0; i < APW; ++i)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = fzero();
  if constexpr (OM) {
    b_sketch_init<SB>(Wt, s, threadIdx.x, kThreads);
    if (t0 < t1) omega_tile<bf16>(seed, kmode, t0 * BT, BT, n, s, Wt + (t0 & 1) * OT, 1, BRP, threadIdx.x, kThreads);
  }
  BTile<2 * APW> regs;
  if (t0 < t1) regs.fetch(A, m, n, row0, rows, t0 * BT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(Ar, rows);
    if constexpr (!OM) {
      const int64_t w0 = t * BT;
      for (int e = threadIdx.x; e < BT * S; e += kThreads) {
        const int bb = e / S, c = e % S;
        Wt[c * BRP + bb] = (w0 + bb < n) ? W[(w0 + bb) * S + c] : (bf16)0.0f;
      }
    }
    __syncthreads();
    if (t + 1 < t1) {
      regs.fetch(A, m, n, row0, rows, (t + 1) * BT, aligned);
      if constexpr (OM)
        omega_tile<bf16>(seed, kmode, (t + 1) * BT, BT, n, s, Wt + ((t + 1) & 1) * OT, 1, BRP, threadIdx.x, kThreads);
    }
    b_phase2<SB, APW>(Ar, OM ? Wt + (t & 1) * OT : Wt, rows, acc2);
  }
  b_store_rows<SB, APW>(acc2, part + g * (int64_t)m_pad * S, rows, row0);
}

// ----------------------------------------------------------------------------------
// A^T Z per tile, rows in chunks of RC: out mode 0 -> out[beta * ldo + c] (n x S, TO),
// mode 1 -> out[c * ldo + beta] for c < s_out (the S x n carry).
// ----------------------------------------------------------------------------------
template <typename TO, int SB, int OUTMODE, int RC>
__global__ __launch_bounds__(kThreads) void kb_atz(const bf16* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                   const bf16* __restrict__ Zg, TO* __restrict__ out, int64_t ldo,
                                                   int s_out, int64_t tiles_per_group, int64_t ntiles) {
  constexpr int S = SB * 16;
  constexpr int TP = RC + 8;
  constexpr int MAXV = 2 * (RC / (16 * kWaves));
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* Ar = reinterpret_cast<bf16*>(smem);
  bf16* Zt = Ar + RC * BRP;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = aligned16(A) && ((n * 2) % 16 == 0);
  const int nchunks = (m_pad + RC - 1) / RC;
  if (nchunks == 1) load_zt<S>(Zg, m_pad, TP, Zt);
  BTile<MAXV> regs;
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad < RC ? m_pad : RC, t0 * BT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    f4_t acc1[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc1[sb] = fzero();
    for (int c = 0; c < nchunks; ++c) {
      const int row0 = c * RC;
      const int rows = (m_pad - row0) < RC ? (m_pad - row0) : RC;
      __syncthreads();
      regs.commit(Ar, rows);
      if (nchunks > 1) load_zt<S>(Zg + (int64_t)row0 * S, rows, TP, Zt);
      __syncthreads();
      if (c + 1 < nchunks) {
        const int nr0 = (c + 1) * RC;
        regs.fetch(A, m, n, nr0, (m_pad - nr0) < RC ? (m_pad - nr0) : RC, t * BT, aligned);
      } else if (t + 1 < t1) {
        regs.fetch(A, m, n, 0, m_pad < RC ? m_pad : RC, (t + 1) * BT, aligned);
      }
      b_phase1_wave<SB>(Ar, Zt, rows, TP, acc1);
    }
    // each wave writes its own 16 columns of W straight from the accumulators
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t b0 = t * BT + wave * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int c = sb * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (b0 + r < n) {
          if (OUTMODE == 0) out[(b0 + r) * ldo + c] = (TO)acc1[sb][r];
          else if (c < s_out) out[(int64_t)c * ldo + b0 + r] = (TO)acc1[sb][r];
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------------
// A^T Z for m_pad <= 256 (one row chunk) with Z in registers: every wave holds all of Z as
// matrix-core B operands (KS K-steps x SB column blocks, zb[ks][sb] = Z[32 ks + 8 (lane /
// 16) + 0..7][16 sb + lane % 16]), so LDS holds only A: two adjacent tiles, staged
// through two register sets whose loads go out together.  Output
// modes as kb_atz; the carry (mode 1) stores four consecutive columns per lane at once.
// ----------------------------------------------------------------------------------
//
// SK2 > 0 (float32 carry, OUTMODE 1): the next mode's sketch rides along.  The carry
// C (r x n, row-major) read as the next unfolding is (r n2) x nc with row c n2 + i2 and
// column j - i2 nc of C's column j; work-group g takes tiles of block i2 = g / gpb only
// (tiles_per_group of its tb = nc / BT, part u = g mod gpb), so its tiles add
// C[:, block cols] Omega[cols, :] to one (r x 16 SK2) block of Y, formed on the float32
// matrix cores straight from the carry accumulators: for k-step r of the 16 x 16 x 4
// product lane l supplies acc1[mb][r] = C[16 mb + l%16][16 w + 4 (l/16) + r] and the
// matching rows of the transposed Omega (omt: 16 SK2 x nc float32).  The waves' sums are
// added in LDS and written as the group's partial (part_y[g]: S x 16 SK2).
template <typename TO, int SB, int OUTMODE, int KS, int SK2 = 0>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void kb_atz_zr(const bf16* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                      const bf16* __restrict__ Zg, TO* __restrict__ out, int64_t ldo,
                                                      int s_out, int64_t tiles_per_group, int64_t ntiles,
                                                      const float* __restrict__ omt, int64_t nc, int gpb,
                                                      float* __restrict__ part_y) {
  constexpr int S = SB * 16;
  constexpr int MAXV = KS * 32 * 8 / kThreads;  // 16-byte vectors of one tile per thread
  static_assert(SK2 == 0 || (OUTMODE == 1 && std::is_same<TO, float>::value), "sketch of a float32 carry");
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* Ar = reinterpret_cast<bf16*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  int64_t t0 = g * tiles_per_group;
  int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  int64_t tb0 = 0;  // SK2: first tile of the block
  if constexpr (SK2 > 0) {
    const int64_t tb = nc / BT;
    tb0 = (g / gpb) * tb;
    t0 = tb0 + (g % gpb) * tiles_per_group;
    t1 = t0 + tiles_per_group < tb0 + tb ? t0 + tiles_per_group : tb0 + tb;
  }
  f4_t yacc[SB][SK2 > 0 ? SK2 : 1];
#pragma unroll
  for (int mb = 0; mb < SB; ++mb)
#pragma unroll
    for (int nb = 0; nb < (SK2 > 0 ? SK2 : 1); ++nb) yacc[mb][nb] = fzero();
  const bool aligned = aligned16(A) && ((n * 2) % 16 == 0);
  const int nks = m_pad / 32;
  BTile<MAXV> ra, rb;
  if (t0 < t1) ra.fetch(A, m, n, 0, m_pad, t0 * BT, aligned);
  if (t0 + 1 < t1) rb.fetch(A, m, n, 0, m_pad, (t0 + 1) * BT, aligned);
  bf8_t zb[KS][SB];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      bf16 z8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = ks * 32 + 8 * (lane >> 4) + e;
        z8[e] = ks < nks ? Zg[(int64_t)k * S + sb * 16 + (lane & 15)] : (bf16)0.0f;
      }
      zb[ks][sb] = bf8_t{z8[0], z8[1], z8[2], z8[3], z8[4], z8[5], z8[6], z8[7]};
    }
  const int Aoff = (8 * (lane >> 4) + ((lane >> 2) & 3)) * BRP + wave * 16 + 4 * (lane & 3);
  const bool vec_out = OUTMODE == 1 && ((ldo & 3) == 0) && ((reinterpret_cast<uintptr_t>(out) & (4 * sizeof(TO) - 1)) == 0);
  // SK2: the transposed Omega rows of tile t, loaded one tile ahead of their use
  constexpr int NOM = SK2 > 0 ? SK2 : 1;
  auto load_om = [&](int64_t t, f4_t (&om)[NOM]) {
    if constexpr (SK2 > 0) {
      const int64_t jc0 = (t - tb0) * BT + wave * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int nb = 0; nb < SK2; ++nb)
        om[nb] = *reinterpret_cast<const f4_t*>(omt + (int64_t)(nb * 16 + (lane & 15)) * nc + jc0);
    }
  };
  // tile t from LDS tile Ab: products, then the outputs
  auto tile = [&](int64_t t, const bf16* Ab, const f4_t (&om)[NOM]) {
    const bf16* Asrc = Ab + Aoff;
    f4_t acc1[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc1[sb] = fzero();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ks < nks) {
        const bf8_t av = ld8_tr(Asrc + ks * 32 * BRP);
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc1[sb] = mma_bf16(av, zb[ks][sb], acc1[sb]);
      }
    }
    const int64_t b0 = t * BT + wave * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int c = sb * 16 + (lane & 15);
      if (OUTMODE == 1 && vec_out && b0 + 3 < n) {
        if (c < s_out) {
          typedef TO to4_t __attribute__((ext_vector_type(4)));
          *reinterpret_cast<to4_t*>(out + (int64_t)c * ldo + b0) =
              to4_t{(TO)acc1[sb][0], (TO)acc1[sb][1], (TO)acc1[sb][2], (TO)acc1[sb][3]};
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (b0 + r < n) {
            if (OUTMODE == 0) out[(b0 + r) * ldo + c] = (TO)acc1[sb][r];
            else if (c < s_out) out[(int64_t)c * ldo + b0 + r] = (TO)acc1[sb][r];
          }
        }
      }
    }
    if constexpr (SK2 > 0) {
      // rows c >= s_out of acc1 are zero (zero columns of Z), as in the stored carry
#pragma unroll
      for (int nb = 0; nb < SK2; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int mb = 0; mb < SB; ++mb)
            yacc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(acc1[mb][r], om[nb][r], yacc[mb][nb], 0, 0, 0);
    }
  };
  // adjacent tiles t, t + 1 in two LDS tiles: their loads go out together (two 128-byte
  // row segments side by side) and one barrier pair serves both
  bf16* Ar1 = Ar + KS * 32 * BRP;
  f4_t omA[NOM], omB[NOM];
  if (SK2 > 0 && t0 < t1) load_om(t0, omA);
  for (int64_t t = t0; t < t1; t += 2) {
    __syncthreads();
    ra.commit(Ar, m_pad);
    if (t + 1 < t1) rb.commit(Ar1, m_pad);
    __syncthreads();
    if (t + 2 < t1) ra.fetch(A, m, n, 0, m_pad, (t + 2) * BT, aligned);
    if (t + 3 < t1) rb.fetch(A, m, n, 0, m_pad, (t + 3) * BT, aligned);
    if (SK2 > 0 && t + 1 < t1) load_om(t + 1, omB);
    tile(t, Ar, omA);
    if (SK2 > 0 && t + 2 < t1) load_om(t + 2, omA);
    if (t + 1 < t1) tile(t + 1, Ar1, omB);
  }
  if constexpr (SK2 > 0) {
    // the four waves' sums added in LDS (the A tiles are no longer read), then written
    constexpr int YC = SK2 * 16, YN = S * YC;
    __syncthreads();
    float* Ysum = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int mb = 0; mb < SB; ++mb)
#pragma unroll
      for (int nb = 0; nb < SK2; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Ysum[wave * YN + (mb * 16 + 4 * (lane >> 4) + r) * YC + nb * 16 + (lane & 15)] = yacc[mb][nb][r];
    __syncthreads();
    for (int e = threadIdx.x; e < YN; e += kThreads)
      part_y[g * YN + e] = ((Ysum[e] + Ysum[YN + e]) + Ysum[2 * YN + e]) + Ysum[3 * YN + e];
  }
}

// ----------------------------------------------------------------------------------
// Gram A A^T (m_pad <= 128 on NT = 256 threads, m_pad <= 256 on NT = 1024): per tile in
// float32 on the matrix cores, folded into float64 accumulators after every tile.
// ----------------------------------------------------------------------------------
template <int PPW, int NT = kThreads, int SKB = 0>
__global__ __launch_bounds__(NT) void kb_gram(const bf16* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                              double* __restrict__ part, int64_t tiles_per_group, int64_t ntiles,
                                              uint64_t seed, int kmode, int s, float* __restrict__ part_y) {
  constexpr int NW = NT / 64;
  constexpr int MAXM = NT == kThreads ? kGramMaxM : kGramBigM;
  constexpr int SPW = SKB > 0 ? (MAXM / 16 * SKB + NW - 1) / NW : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* Ar = reinterpret_cast<bf16*>(smem);
  bf16* Ot = Ar + m_pad * BRP;  // SKB > 0: two transposed Omega tiles of SKB * 16 x BRP
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = aligned16(A) && ((n * 2) % 16 == 0);
  const int MB = m_pad / 16;
  const int npairs = MB * (MB + 1) / 2;
  // block pair i of this wave: p = wave + NW i in the row-major upper triangle of MB x MB
  // blocks, decoded into (block row, block column) when used (no per-pair registers)
  auto pair_of = [&](int i, int* pa, int* pb) {
    int p = wave + NW * i, a = 0;
    if (p >= npairs) return false;
    while (p >= MB - a) { p -= MB - a; ++a; }
    *pa = a; *pb = a + p;
    return true;
  };
  double acc[PPW][4];
#pragma unroll
  for (int i = 0; i < PPW; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[i][r] = 0.0;
  constexpr int OT = SKB * 16 * BRP;  // one Omega tile
  f4_t yacc[SPW];
#pragma unroll
  for (int i = 0; i < SPW; ++i) yacc[i] = fzero();
  if constexpr (SKB > 0) {
    b_sketch_init<SKB>(Ot, s, threadIdx.x, NT);
    if (t0 < t1) omega_tile<bf16>(seed, kmode, t0 * BT, BT, n, s, Ot + (t0 & 1) * OT, 1, BRP, threadIdx.x, NT);
  }
  BTile<MAXM * 8 / NT, NT> regs;
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad, t0 * BT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(Ar, m_pad);
    __syncthreads();
    if (t + 1 < t1) {
      regs.fetch(A, m, n, 0, m_pad, (t + 1) * BT, aligned);
      if constexpr (SKB > 0)
        omega_tile<bf16>(seed, kmode, (t + 1) * BT, BT, n, s, Ot + ((t + 1) & 1) * OT, 1, BRP, threadIdx.x, NT);
    }
    if constexpr (SKB > 0) b_sketch_tiles<SKB, SPW>(Ar, Ot + (t & 1) * OT, MB, wave, NW, yacc);
#pragma unroll
    for (int i = 0; i < PPW; ++i) {
      int pa, pb;
      if (pair_of(i, &pa, &pb)) {
        f4_t c = fzero();
#pragma unroll
        for (int ks = 0; ks < BT / 32; ++ks) {
          const int k0 = ks * 32 + 8 * (lane >> 4);
          c = mma_bf16(ld8(Ar + (pa * 16 + (lane & 15)) * BRP + k0), ld8(Ar + (pb * 16 + (lane & 15)) * BRP + k0), c);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][r] += (double)c[r];
      }
    }
  }
  double* out = part + g * (int64_t)m_pad * m_pad;
#pragma unroll
  for (int i = 0; i < PPW; ++i) {
    int pa, pb;
    if (pair_of(i, &pa, &pb))
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(pa * 16 + 4 * (lane >> 4) + r) * m_pad + pb * 16 + (lane & 15)] = acc[i][r];
  }
  if constexpr (SKB > 0) b_sketch_store<SKB, SPW>(yacc, part_y + g * (int64_t)m_pad * SKB * 16, MB, wave, NW);
}

// ----------------------------------------------------------------------------------
// Gram A A^T for 128 < m_pad <= 256 on 1024 threads, register-blocked: active wave w
// owns the 64 x 64 super-block kSuperBlocks[w] of the upper triangle (a 4 x 4 grid of
// 16 x 16 tiles), so per 32-column step it loads the operands of its 4 row blocks and 4
// column blocks once for 16 products (the pair kernel loads two per product).  The ten
// upper super-blocks go to waves 0..9, which the round-robin wave placement spreads 3, 3,
// 2, 2 over the four SIMDs.  Products of bfloat16 are exact in float32; the sums stay in
// float32 over the work-group's columns and the partial is written in float64.  The tile
// is staged with its rows padded to 64 (zeros beyond m).
// ----------------------------------------------------------------------------------
__constant__ int kSuperBlocks[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1},
                                        {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};

// With SKB > 0 the six waves left over (10..15) draw the Omega rows of the next tile and
// form the sketch tiles of a Gram-first mode.  The two roles run separate copies of the
// tile loop (the same loads, LDS commits and barriers in the same order), so each copy
// keeps only its own registers live; the sketch sums stay in LDS (Ys, m_pad x S float32,
// each 16 x 16 tile owned by one wave), which leaves the generator's registers free.
// TPI tiles per barrier interval: the A tiles of an interval sit side by side in LDS
// (TPI x rows x BRP) and its Omega rows form one transposed tile of pitch TPI BT + 8.  Two
// tiles give 10 generator passes of 64 items per interval at s = 40, which the six
// generator waves (two of them share a SIMD with another) split 3/3/2/2 over the SIMDs,
// instead of 5 passes per tile of which one SIMD takes 2.
template <int TPI, int SKB>
__device__ __host__ constexpr int gram_sb_op() { return TPI * BT + 8; }

template <int SKB, int TPI, bool GRAM>
__device__ inline void gram_sb_loop(const bf16* __restrict__ A, int64_t m, int64_t n, int m_pad, int64_t g,
                                    int64_t G, int64_t ntiles, bool aligned, bf16* __restrict__ Ar, bf16* __restrict__ Ot,
                                    float* __restrict__ Ys, uint64_t seed, int kmode, int s, f4_t (&acc)[4][4]) {
  constexpr int SW = kGramBigThreads / 64 - 10;  // sketch waves
  constexpr int S = SKB * 16;
  constexpr int SPW = SKB > 0 ? (kGramBigM / 16 * SKB + SW - 1) / SW : 1;
  constexpr int OP = gram_sb_op<TPI, SKB>();  // Omega tile pitch
  constexpr int OT = S * OP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows64 = (m_pad + 63) / 64 * 64;
  const int MB = m_pad / 16;
  const int sr = (GRAM && wave < 10) ? kSuperBlocks[wave][0] : 0, sc = (GRAM && wave < 10) ? kSuperBlocks[wave][1] : 0;
  const bool active = GRAM && wave < 10 && sc * 64 < m_pad;
  const int gtid = (int)threadIdx.x - 640, gthr = kGramBigThreads - 640;
  // intervals g, g + G, g + 2G, ... (tiles TPI j .. TPI j + TPI - 1 of interval j): the
  // work-groups walk the columns side by side
  const int64_t nint = (ntiles + TPI - 1) / TPI;
  const int64_t kc = g < nint ? (nint - g + G - 1) / G : 0;
  if constexpr (!GRAM) {
    // Omega rows c >= 8 ceil(s / 8) are never drawn: zero them in both buffers once
    const int cz = 8 * ((s + 7) / 8);
    for (int e = gtid; e < 2 * OT; e += gthr)
      if ((e / OP) % S >= cz) Ot[e] = (bf16)0.0f;
    // each wave zeroes the sketch tiles it owns
    for (int p = wave - 10; p < MB * SKB; p += SW) {
      const int rb = p / SKB, cb = p - rb * SKB;
#pragma unroll
      for (int r = 0; r < 4; ++r) Ys[(rb * 16 + 4 * (lane >> 4) + r) * S + cb * 16 + (lane & 15)] = 0.0f;
    }
    if (kc > 0) omega_tile<bf16>(seed, kmode, g * TPI * BT, TPI * BT, n, s, Ot, 1, OP, gtid, gthr);
  }
  BTile<kGramBigM * 8 / kGramBigThreads, kGramBigThreads> regs[TPI];
  if (kc > 0)
#pragma unroll
    for (int u = 0; u < TPI; ++u) regs[u].fetch(A, m, n, 0, rows64, (g * TPI + u) * BT, aligned);
  for (int64_t k = 0; k < kc; ++k) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TPI; ++u) regs[u].commit(Ar + u * rows64 * BRP, rows64);
    __syncthreads();
    if (k + 1 < kc) {
      const int64_t jn = g + (k + 1) * G;
#pragma unroll
      for (int u = 0; u < TPI; ++u) regs[u].fetch(A, m, n, 0, rows64, (jn * TPI + u) * BT, aligned);
      if constexpr (!GRAM)
        omega_tile<bf16>(seed, kmode, jn * TPI * BT, TPI * BT, n, s, Ot + ((k + 1) & 1) * OT, 1, OP, gtid, gthr);
    }
    if constexpr (GRAM) {
      if (active) {
#pragma unroll 1
        for (int u = 0; u < TPI; ++u) {
          const bf16* At = Ar + u * rows64 * BRP;
#pragma unroll
          for (int ks = 0; ks < BT / 32; ++ks) {
            const int k0 = ks * 32 + 8 * (lane >> 4);
            bf8_t av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              av[i] = ld8(At + (sr * 64 + i * 16 + (lane & 15)) * BRP + k0);
              bv[i] = ld8(At + (sc * 64 + i * 16 + (lane & 15)) * BRP + k0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[i][j] = mma_bf16(av[i], bv[j], acc[i][j]);
          }
        }
      }
    } else {
      const bf16* Oc = Ot + (k & 1) * OT;
#pragma unroll
      for (int i = 0; i < SPW; ++i) {
        const int p = (wave - 10) + SW * i;
        if (p < MB * SKB) {
          const int rb = p / SKB, cb = p - rb * SKB;
          f4_t c = fzero();
#pragma unroll
          for (int ks = 0; ks < TPI * BT / 32; ++ks) {
            const bf16* At = Ar + (ks / (BT / 32)) * rows64 * BRP;
            const int k0 = (ks % (BT / 32)) * 32 + 8 * (lane >> 4);
            c = mma_bf16(ld8(At + (rb * 16 + (lane & 15)) * BRP + k0),
                         ld8(Oc + (cb * 16 + (lane & 15)) * OP + ks * 32 + 8 * (lane >> 4)), c);
          }
          float* yt = Ys + (rb * 16 + 4 * (lane >> 4)) * S + cb * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) yt[r * S] += c[r];
        }
      }
    }
  }
}

template <int SKB = 0, int TPI = 1>
__global__ __launch_bounds__(kGramBigThreads) void kb_gram_sb(const bf16* __restrict__ A, int64_t m, int64_t n,
                                                              int m_pad, double* __restrict__ part,
                                                              int64_t tiles_per_group, int64_t ntiles, uint64_t seed,
                                                              int kmode, int s, float* __restrict__ part_y) {
  constexpr int S = SKB * 16;
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* Ar = reinterpret_cast<bf16*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  (void)tiles_per_group;
  const bool aligned = aligned16(A) && ((n * 2) % 16 == 0);
  const int rows64 = (m_pad + 63) / 64 * 64;
  bf16* Ot = Ar + TPI * rows64 * BRP;                        // SKB > 0: two transposed Omega tiles
  float* Ys = reinterpret_cast<float*>(Ot + 2 * S * gram_sb_op<TPI, SKB>());  // SKB > 0: m_pad x S sketch sums
  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = fzero();
  if (SKB == 0 || wave < 10)
    gram_sb_loop<SKB, TPI, true>(A, m, n, m_pad, g, gridDim.x, ntiles, aligned, Ar, Ot, Ys, seed, kmode, s, acc);
  else
    gram_sb_loop<SKB, TPI, false>(A, m, n, m_pad, g, gridDim.x, ntiles, aligned, Ar, Ot, Ys, seed, kmode, s, acc);
  if (SKB > 0 && wave >= 10) {
    // each wave copies the sketch tiles it owns (no other wave wrote them)
    constexpr int SW = kGramBigThreads / 64 - 10;
    const int MB = m_pad / 16;
    float* outy = part_y + g * (int64_t)m_pad * S;
    for (int p = wave - 10; p < MB * SKB; p += SW) {
      const int rb = p / SKB, cb = p - rb * SKB;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = (rb * 16 + 4 * (lane >> 4) + r) * S + cb * 16 + (lane & 15);
        outy[e] = Ys[e];
      }
    }
    return;
  }
  if (wave >= 10) return;
  const int sr = kSuperBlocks[wave][0], sc = kSuperBlocks[wave][1];
  if (sc * 64 >= m_pad) return;
  double* out = part + g * (int64_t)m_pad * m_pad;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = sc * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = sr * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (row < m_pad && col < m_pad) out[(int64_t)row * m_pad + col] = (double)acc[i][j][r];
      }
    }
}

// ----------------------------------------------------------------------------------
// Float32 operands on the bf16 matrix cores (the two-pass Krylov products and carries of
// tall float32 unfoldings).  Each float32 x is split into three bf16 values
// x1 = bf16(x), x2 = bf16(x - x1), x3 = bf16(x - x1 - x2): both differences are exact in
// float32 and |x - x1 - x2 - x3| <= 2^-24 |x| (|x| below the largest bf16, 3.39e38).  A
// product a b is formed as a1 b1 + a1 b2 + a2 b1 + a1 b3 + a2 b2 + a3 b1, each term exact
// in float32 and summed in the float32 accumulators; the dropped terms a2 b3, a3 b2, a3 b3
// stay below 2^-23 |a b|, the order of float32 rounding.  Six bf16 products take 2.7 times
// less matrix-core time than the float32 one, which leaves these passes bound by HBM.
// ----------------------------------------------------------------------------------
__device__ inline float bf16_to_f32(bf16 h) {
  return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, h) << 16);
}
__device__ inline void split3(float x, bf16& x1, bf16& x2, bf16& x3) {
  x1 = (bf16)x;
  const float r1 = x - bf16_to_f32(x1);
  x2 = (bf16)r1;
  x3 = (bf16)(r1 - bf16_to_f32(x2));
}
// acc += a b over one K-step from the split operands a[3], b[3]
__device__ inline f4_t mma_split(const bf8_t (&a)[3], const bf8_t (&b)[3], f4_t acc) {
  acc = mma_bf16(a[0], b[0], acc);
  acc = mma_bf16(a[0], b[1], acc);
  acc = mma_bf16(a[1], b[0], acc);
  acc = mma_bf16(a[0], b[2], acc);
  acc = mma_bf16(a[1], b[1], acc);
  return mma_bf16(a[2], b[0], acc);
}
// ld8_tr on a plane of row pitch `pitch` (bf16 elements)
__device__ inline bf8_t ld8_trp(const bf16* p, int pitch) {
  typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) bf4_t lds_bf4;
  const bf4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf4*)(p));
  const bf4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf4*)(p + 4 * pitch));
  return bf8_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}
// Rows [row0, row0 + ROWS) x columns [col0, col0 + 4 VPR) of a float32 matrix in 16-byte
// vectors (NV per thread); rows >= m and columns >= n read as zero.
template <int NV, int VPR>
__device__ inline void fetch_f32(u4_t (&v)[NV], const float* __restrict__ A, int64_t m, int64_t n, int64_t row0,
                                 int rows, int64_t col0, bool full) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int idx = (int)threadIdx.x + i * kThreads;
    const int rr = idx / VPR, cv = idx % VPR;
    const int64_t row = row0 + rr;
    u4_t val = u4_t{0u, 0u, 0u, 0u};
    if (rr < rows && row < m) {
      const float* src = A + row * n + col0 + 4 * cv;
      if (full) {
        val = *reinterpret_cast<const u4_t*>(src);
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (col0 + 4 * cv + e < n) ? src[e] : 0.0f;
        val = *reinterpret_cast<u4_t*>(t);
      }
    }
    v[i] = val;
  }
}
// The vectors of fetch_f32 split into three row-major bf16 planes (pitch P, plane stride PS).
template <int NV, int VPR, int P, int PS>
__device__ inline void commit_split_rows(const u4_t (&v)[NV], bf16* __restrict__ planes) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int idx = (int)threadIdx.x + i * kThreads;
    const int rr = idx / VPR, cv = idx % VPR;
    const float* f = reinterpret_cast<const float*>(&v[i]);
    bf16 h[3][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split3(f[e], h[0][e], h[1][e], h[2][e]);
#pragma unroll
    for (int p = 0; p < 3; ++p)
      *reinterpret_cast<uint2*>(planes + p * PS + rr * P + 4 * cv) = *reinterpret_cast<const uint2*>(h[p]);
  }
}
// A row-major float32 block (rows x S, 16-byte vectors, NV per thread) split into three
// transposed bf16 planes: plane p element (c, r) at planes[p * PS + c * P + r].
template <int NV, int S, int P, int PS>
__device__ inline void commit_split_cols(const u4_t (&v)[NV], int rows, bf16* __restrict__ planes) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int idx = (int)threadIdx.x + i * kThreads;
    if (idx < rows * S / 4) {
      const int r = idx / (S / 4), c0 = 4 * (idx % (S / 4));
      const float* f = reinterpret_cast<const float*>(&v[i]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        bf16 h0, h1, h2;
        split3(f[e], h0, h1, h2);
        planes[(c0 + e) * P + r] = h0;
        planes[PS + (c0 + e) * P + r] = h1;
        planes[2 * PS + (c0 + e) * P + r] = h2;
      }
    }
  }
}

// W = A^T Z (OUTMODE 0: out[beta ldo + c], all S columns; OUTMODE 2: three transposed bf16
// planes, plane p row c at out + (p S + c) ldo in bf16 elements) or the carry (OUTMODE 1:
// out[c ldo + beta], c < s_out) for float32 A (m_pad rows in chunks of kSplitRC).  Z comes
// split once per launch (k_split_planes): three transposed bf16 planes, plane p row c at
// Zp[(p S + c) ldz], ldz = m_pad rounded up to kSplitRC, so each chunk of Z is a plain copy.
// A tile: kSplitTC columns, split into three planes as it is staged; wave w owns the
// tile's column blocks 2w and 2w + 1 for all S columns.
constexpr int kSplitTC = kSplitTCols, kSplitRC = 64;
constexpr int kSplitAP = kSplitTC + 24;  // plane pitch: transposed loads of 4 rows hit distinct banks
constexpr int kSplitZP = kSplitRC + 8;
inline size_t atz_split_lds_bytes(int S) {
  return ((size_t)3 * kSplitRC * kSplitAP + (size_t)3 * S * kSplitZP) * sizeof(bf16);
}

// Z (rows x S float32, row-major) into three transposed bf16 planes of pitch ldz (rows
// rows .. ldz - 1 zero).
__global__ __launch_bounds__(256) void k_split_planes(const float* __restrict__ Z, int rows, int S, int ldz,
                                                      bf16* __restrict__ Zp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)ldz * S) return;
  const int r = (int)(e / S), c = (int)(e % S);
  bf16 h0, h1, h2;
  split3(r < rows ? Z[e] : 0.0f, h0, h1, h2);
  Zp[(int64_t)c * ldz + r] = h0;
  Zp[(int64_t)(S + c) * ldz + r] = h1;
  Zp[(int64_t)(2 * S + c) * ldz + r] = h2;
}

template <typename TO, int SB, int OUTMODE>
__global__ __launch_bounds__(kThreads) void kb_atz_s(const float* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                     const bf16* __restrict__ Zp, int ldz, TO* __restrict__ out,
                                                     int64_t ldo, int s_out, int64_t tiles_per_group,
                                                     int64_t ntiles) {
  constexpr int S = SB * 16, TC = kSplitTC, RC = kSplitRC, AP = kSplitAP, ZP = kSplitZP;
  constexpr int VPR = TC / 4;                                       // vectors per A row
  constexpr int AV = RC * VPR / kThreads;                           // A vectors per thread
  constexpr int ZV = (3 * S * (RC / 8) + kThreads - 1) / kThreads;  // Z plane vectors per thread
  static_assert(TC == 32 * kWaves, "two column blocks per wave");
  extern __shared__ __align__(16) unsigned char smem[];
  bf16* Ap = reinterpret_cast<bf16*>(smem);  // 3 planes RC x AP
  bf16* Zt = Ap + 3 * RC * AP;                // 3 planes S x ZP (transposed)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = aligned16(A) && (n % 4 == 0);
  const int nchunks = (m_pad + RC - 1) / RC;
  u4_t av[AV], zv[ZV];
  auto fetch = [&](int64_t t, int c) {
    const int64_t col0 = t * TC;
    const int row0 = c * RC;
    const int rows = (m_pad - row0) < RC ? (m_pad - row0) : RC;
    fetch_f32<AV, VPR>(av, A, m, n, row0, rows, col0, aligned && col0 + TC <= n);
    // plane row pc = p S + cc: its RC entries of this chunk are RC / 8 16-byte vectors
#pragma unroll
    for (int i = 0; i < ZV; ++i) {
      const int idx = (int)threadIdx.x + i * kThreads;
      zv[i] = idx < 3 * S * (RC / 8)
                  ? *reinterpret_cast<const u4_t*>(Zp + (int64_t)(idx / (RC / 8)) * ldz + row0 + 8 * (idx % (RC / 8)))
                  : u4_t{0u, 0u, 0u, 0u};
    }
  };
  if (t0 < t1) fetch(t0, 0);
  for (int64_t t = t0; t < t1; ++t) {
    f4_t acc[2][SB];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc[j][sb] = fzero();
    for (int c = 0; c < nchunks; ++c) {
      __syncthreads();
      commit_split_rows<AV, VPR, AP, RC * AP>(av, Ap);
#pragma unroll
      for (int i = 0; i < ZV; ++i) {
        const int idx = (int)threadIdx.x + i * kThreads;
        if (idx < 3 * S * (RC / 8))
          *reinterpret_cast<u4_t*>(Zt + (idx / (RC / 8)) * ZP + 8 * (idx % (RC / 8))) = zv[i];
      }
      __syncthreads();
      if (c + 1 < nchunks) fetch(t, c + 1);
      else if (t + 1 < t1) fetch(t + 1, 0);
#pragma unroll 1
      for (int ks = 0; ks < RC / 32; ++ks) {
        const int k0 = ks * 32 + 8 * (lane >> 4);
        bf8_t zb[SB][3];
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
#pragma unroll
          for (int p = 0; p < 3; ++p) zb[sb][p] = ld8(Zt + p * S * ZP + (sb * 16 + (lane & 15)) * ZP + k0);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const bf16* src = Ap + (ks * 32 + 8 * (lane >> 4) + ((lane >> 2) & 3)) * AP + (2 * wave + j) * 16 + 4 * (lane & 3);
          bf8_t a[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) a[p] = ld8_trp(src + p * RC * AP, AP);
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) acc[j][sb] = mma_split(a, zb[sb], acc[j][sb]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t b0 = t * TC + (2 * wave + j) * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        const int c = sb * 16 + (lane & 15);
        if constexpr (OUTMODE == 2) {
          // W as three transposed bf16 planes: plane p row c at out + (p S + c) ldo
          bf16 h[3][4];
#pragma unroll
          for (int r = 0; r < 4; ++r) split3(acc[j][sb][r], h[0][r], h[1][r], h[2][r]);
          bf16* wp = reinterpret_cast<bf16*>(out);
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            bf16* dst = wp + (int64_t)(p * S + c) * ldo + b0;
            if (b0 + 3 < n) {
              *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(h[p]);
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (b0 + r < n) dst[r] = h[p][r];
            }
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (b0 + r < n) {
              if (OUTMODE == 0) out[(b0 + r) * ldo + c] = (TO)acc[j][sb][r];
              else if (c < s_out) out[(int64_t)c * ldo + b0 + r] = (TO)acc[j][sb][r];
            }
          }
        }
      }
    }
  }
}

// partial[g] rows [rb kAwRows, +kAwRows) += A_J W_J for float32 A: tiles of kSplitTT
// columns kept in float32 in LDS and split when a wave loads its operand (each element of
// A is loaded by one wave).  The W tile reaches LDS as three transposed bf16 planes:
// WM 0: split from a float32 W (n x S); WM 1: Omega_k drawn inside the kernel (float32
// entries, split as they are written) into a double-buffered set of planes (one row
// block: m_pad <= kAwRows); WM 2: copied from the planes kb_atz_s wrote (plane p row c at
// W + (p S + c) ldw, bf16).
constexpr int kSplitTT = 32;
constexpr int kSplitWP = kSplitTT + 8;   // bf16 pitch of a transposed W plane
constexpr int kSplitAFP = kSplitTT + 4;  // float32 pitch of the A tile
inline size_t aw_split_lds_bytes(int S, bool om) {
  return (size_t)kAwRows * kSplitAFP * sizeof(float) + (om ? 2 : 1) * (size_t)3 * S * kSplitWP * sizeof(bf16);
}

// Omega_k rows [beta0, beta0 + rows) drawn and split into the three transposed planes of
// pitch P (plane stride PS): plane p element (c, b) at planes[p * PS + c * P + b].
template <int P, int PS>
__device__ inline void omega_tile_split(uint64_t seed, int k, int64_t beta0, int rows, int64_t n, int s,
                                        bf16* __restrict__ planes, int tid, int nthr) {
  const int g8 = (s + 7) / 8;
  for (int id = tid; id < rows * g8; id += nthr) {
    const int b = id / g8, g = id - b * g8;
    float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (beta0 + b < n) omega8(seed, k, beta0 + b, g, z);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = 8 * g + j;
      bf16 h0, h1, h2;
      split3(c < s ? z[j] : 0.0f, h0, h1, h2);
      planes[c * P + b] = h0;
      planes[PS + c * P + b] = h1;
      planes[2 * PS + c * P + b] = h2;
    }
  }
}

template <int SB, int WM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void kb_aw_s(
    const float* __restrict__ A, int64_t m, int64_t n, int m_pad, const void* __restrict__ Wv, int64_t ldw,
    float* __restrict__ part, int64_t tiles_per_group, int64_t ntiles, uint64_t seed, int kmode, int s) {
  constexpr bool OM = WM == 1;
  const float* __restrict__ W = static_cast<const float*>(Wv);
  const bf16* __restrict__ Wp = static_cast<const bf16*>(Wv);
  constexpr int S = SB * 16, TT = kSplitTT, P = kSplitWP, AFP = kSplitAFP;
  constexpr int APW = kAwRows / (16 * kWaves);
  constexpr int VPR = TT / 4;
  constexpr int AV = kAwRows * VPR / kThreads;
  constexpr int WV = OM ? 1 : (WM == 2 ? (3 * S * (TT / 8) + kThreads - 1) / kThreads
                                       : (TT * S / 4 + kThreads - 1) / kThreads);
  constexpr int WPL = 3 * S * P;  // one set of W planes
  extern __shared__ __align__(16) unsigned char smem[];
  float* As = reinterpret_cast<float*>(smem);                  // kAwRows x AFP
  bf16* Wt = reinterpret_cast<bf16*>(As + kAwRows * AFP);      // 3 planes S x P (OM: two sets)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int row0 = blockIdx.y * kAwRows;
  const int rows = (m_pad - row0) < kAwRows ? (m_pad - row0) : kAwRows;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = aligned16(A) && (n % 4 == 0);
  f4_t acc[APW][SB];
#pragma unroll
  for (int i = 0; i < APW; ++i)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc[i][sb] = fzero();
  // NST register stages (two without Omega for S <= 48: the loads of tiles t + 1 and t + 2
  // in flight)
  constexpr int NST = (OM || SB > 3) ? 1 : 2;
  u4_t av[NST][AV], wv[NST][WV];
  auto fetch = [&](int st, int64_t t) {
    const int64_t col0 = t * TT;
    fetch_f32<AV, VPR>(av[st], A, m, n, row0, rows, col0, aligned && col0 + TT <= n);
    if constexpr (WM == 0) {
      const int wrows = (n - col0) < TT ? (int)(n - col0) : TT;
      const u4_t* ws = reinterpret_cast<const u4_t*>(W + col0 * S);
#pragma unroll
      for (int i = 0; i < WV; ++i) {
        const int idx = (int)threadIdx.x + i * kThreads;
        wv[st][i] = idx < wrows * S / 4 ? ws[idx] : u4_t{0u, 0u, 0u, 0u};
      }
    } else if constexpr (WM == 2) {
      // plane row pc = p S + c: the tile's TT entries are TT / 8 16-byte vectors
      const bool wfull = col0 + TT <= n;
#pragma unroll
      for (int i = 0; i < WV; ++i) {
        const int idx = (int)threadIdx.x + i * kThreads;
        u4_t val = u4_t{0u, 0u, 0u, 0u};
        if (idx < 3 * S * (TT / 8)) {
          const bf16* src = Wp + (int64_t)(idx / (TT / 8)) * ldw + col0 + 8 * (idx % (TT / 8));
          if (wfull) {
            val = *reinterpret_cast<const u4_t*>(src);
          } else {
            bf16 t8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) t8[e] = (col0 + 8 * (idx % (TT / 8)) + e < n) ? src[e] : (bf16)0.0f;
            val = *reinterpret_cast<u4_t*>(t8);
          }
        }
        wv[st][i] = val;
      }
    }
  };
  if constexpr (OM) {
    // Omega rows c >= 8 ceil(s / 8) are never drawn: zero them in both sets once
    const int cz = 8 * ((s + 7) / 8);
    for (int e = threadIdx.x; e < 2 * WPL; e += kThreads)
      if ((e % (S * P)) / P >= cz) Wt[e] = (bf16)0.0f;
    if (t0 < t1) omega_tile_split<P, S * P>(seed, kmode, t0 * TT, TT, n, s, Wt + (t0 & 1) * WPL, threadIdx.x, kThreads);
  }
#pragma unroll
  for (int st = 0; st < NST; ++st)
    if (t0 + st < t1) fetch(st, t0 + st);
  for (int64_t tb = t0; tb < t1; tb += NST)
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    const int64_t t = tb + st;
    if (t >= t1) break;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int idx = (int)threadIdx.x + i * kThreads;
      *reinterpret_cast<u4_t*>(As + (idx / VPR) * AFP + 4 * (idx % VPR)) = av[st][i];
    }
    if constexpr (WM == 0) commit_split_cols<WV, S, P, S * P>(wv[st], TT, Wt);
    if constexpr (WM == 2) {
#pragma unroll
      for (int i = 0; i < WV; ++i) {
        const int idx = (int)threadIdx.x + i * kThreads;
        if (idx < 3 * S * (TT / 8)) *reinterpret_cast<u4_t*>(Wt + (idx / (TT / 8)) * P + 8 * (idx % (TT / 8))) = wv[st][i];
      }
    }
    __syncthreads();
    if (t + NST < t1) fetch(st, t + NST);
    if constexpr (OM)
      if (t + 1 < t1)
        omega_tile_split<P, S * P>(seed, kmode, (t + 1) * TT, TT, n, s, Wt + ((t + 1) & 1) * WPL, threadIdx.x, kThreads);
    const bf16* Wc = OM ? Wt + (t & 1) * WPL : Wt;
    const int k0 = 8 * (lane >> 4);
    bf8_t wb[SB][3];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int p = 0; p < 3; ++p) wb[sb][p] = ld8(Wc + p * S * P + (sb * 16 + (lane & 15)) * P + k0);
#pragma unroll
    for (int i = 0; i < APW; ++i) {
      const int ab = wave + kWaves * i;
      if (ab * 16 < rows) {
        const float* src = As + (ab * 16 + (lane & 15)) * AFP + k0;
        const u4_t lo = *reinterpret_cast<const u4_t*>(src), hi = *reinterpret_cast<const u4_t*>(src + 4);
        const float* fl = reinterpret_cast<const float*>(&lo);
        const float* fh = reinterpret_cast<const float*>(&hi);
        bf16 h[3][8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          split3(fl[e], h[0][e], h[1][e], h[2][e]);
          split3(fh[e], h[0][e + 4], h[1][e + 4], h[2][e + 4]);
        }
        bf8_t a[3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
          a[p] = bf8_t{h[p][0], h[p][1], h[p][2], h[p][3], h[p][4], h[p][5], h[p][6], h[p][7]};
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc[i][sb] = mma_split(a, wb[sb], acc[i][sb]);
      }
    }
  }
  b_store_rows<SB, APW>(acc, part + g * (int64_t)m_pad * S, rows, row0);
}

// ----------------------------------------------------------------------------------
// Launchers.
// ----------------------------------------------------------------------------------
template <typename F>
static hipError_t b_set_lds(F kernel, size_t bytes) {
  if (bytes > kLdsBytes) return hipErrorInvalidValue;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

hipError_t launch_reduce_f32(const float* part, int64_t groups, int64_t stride, int m, int S, int s, double* y,
                             int ldy, hipStream_t st);
hipError_t launch_reduce_gram(const double* part, int64_t groups, int m_pad, int m, double* out, hipStream_t st);

static void grid_of(int64_t n, int64_t cap, int64_t* tpg, int64_t* gu, int64_t* ntiles) {
  *ntiles = (n + BT - 1) / BT;
  const int64_t G = groups_for(*ntiles, cap);
  *tpg = (*ntiles + G - 1) / G;
  *gu = (*ntiles + *tpg - 1) / *tpg;
}

template <int SB, int APW>
static hipError_t fused_b(const StreamArgs& a) {
  int64_t tpg, gu, nt;
  grid_of(a.n, kMaxGroups, &tpg, &gu, &nt);
  const size_t lds = fused_lds_bytes(a.m_pad, SB * 16, TTR_BF16);
  auto kern = kb_fused<SB, APW>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  if (!part_fits(a, gu, a.m_pad * SB * 16, sizeof(float))) return hipErrorInvalidValue;
  if ((e = mark_event(a.ev_begin, a.stream)) != hipSuccess) return e;
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)gu), dim3(kThreads), lds, a.stream, (const bf16*)a.A, a.m, a.n,
                       (int)a.m_pad, (const bf16*)a.Z, (float*)a.part, tpg, nt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = mark_event(a.ev_end, a.stream)) != hipSuccess) return e;
  return launch_reduce_f32((const float*)a.part, gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y,
                           a.ldy, a.stream);
}

template <int SB, bool OM = false>
static hipError_t aw_b(const StreamArgs& a) {
  int64_t tpg, gu, nt;
  const int64_t rb = (a.m_pad + kAwRows - 1) / kAwRows;
  if (OM && rb != 1) return hipErrorInvalidValue;
  grid_of(a.n, std::max<int64_t>(1, kMaxGroups / rb), &tpg, &gu, &nt);
  // OM: a second transposed W tile (the Omega tiles are double-buffered)
  const size_t lds = aw_lds_bytes(SB * 16, TTR_BF16) + (OM ? (size_t)SB * 16 * BRP * 2 : 0);
  auto kern = kb_aw<SB, OM>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  if (!part_fits(a, gu, a.m_pad * SB * 16, sizeof(float))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)gu, (unsigned)rb), dim3(kThreads), lds, a.stream, (const bf16*)a.A, a.m,
                     a.n, (int)a.m_pad, (const bf16*)a.W, (float*)a.part, tpg, nt, a.seed, a.kmode, a.s);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_f32((const float*)a.part, gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y,
                           a.ldy, a.stream);
}

template <typename TO, int SB, int OUTMODE, int KS>
static hipError_t atz_zr_b(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  int64_t tpg, gu, nt;
  grid_of(a.n, kMaxGroups, &tpg, &gu, &nt);
  const size_t lds = (size_t)2 * KS * 32 * BRP * sizeof(bf16);
  auto kern = kb_atz_zr<TO, SB, OUTMODE, KS>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)gu), dim3(kThreads), lds, a.stream, (const bf16*)a.A, a.m, a.n,
                     (int)a.m_pad, (const bf16*)a.Z, (TO*)out, ldo, s_out, tpg, nt, (const float*)nullptr, (int64_t)0,
                     1, (float*)nullptr);
  return hipGetLastError();
}

// The carry with the next mode's sketch (kb_atz_zr<float, SB, 1, KS, SK2>): n2 blocks of
// nc columns, gpb work-groups per block.
template <int SB, int KS, int SK2>
static hipError_t carry_sketch_b(const StreamArgs& a, float* out, int64_t ldo, int s_out, const float* omt, int64_t nc,
                                 int64_t n2, float* part_y) {
  const int64_t tb = nc / BT;
  const int64_t gpb = std::max<int64_t>(1, std::min<int64_t>(tb, kMaxGroups / n2));
  const int64_t tpg = (tb + gpb - 1) / gpb;
  const size_t lds = (size_t)2 * KS * 32 * BRP * sizeof(bf16);
  static_assert((size_t)4 * SB * 16 * SK2 * 16 * sizeof(float) <= (size_t)2 * KS * 32 * BRP * sizeof(bf16),
                "wave sums fit the tile LDS");
  auto kern = kb_atz_zr<float, SB, 1, KS, SK2>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)(n2 * gpb)), dim3(kThreads), lds, a.stream, (const bf16*)a.A, a.m, a.n,
                     (int)a.m_pad, (const bf16*)a.Z, out, ldo, s_out, tpg, tb * n2, omt, nc, (int)gpb, part_y);
  return hipGetLastError();
}

template <typename TO, int SB, int OUTMODE>
static hipError_t atz_b(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  constexpr int RC = atz_row_chunk(SB * 16, TTR_BF16);
  // Z in registers when it takes at most 16 operands per lane (m_pad <= 256, S <= 32; or
  // m_pad <= 128, S <= 64)
  if (a.m_pad <= 128) return atz_zr_b<TO, SB, OUTMODE, 4>(a, out, ldo, s_out);
  if constexpr (SB <= 2)
    if (a.m_pad <= 256) return atz_zr_b<TO, SB, OUTMODE, 8>(a, out, ldo, s_out);
  int64_t tpg, gu, nt;
  grid_of(a.n, kMaxGroups, &tpg, &gu, &nt);
  const size_t lds = atz_lds_bytes(SB * 16, TTR_BF16);
  auto kern = kb_atz<TO, SB, OUTMODE, RC>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)gu), dim3(kThreads), lds, a.stream, (const bf16*)a.A, a.m, a.n,
                     (int)a.m_pad, (const bf16*)a.Z, (TO*)out, ldo, s_out, tpg, nt);
  return hipGetLastError();
}

template <int PPW, int NT = kThreads, int SKB = 0>
static hipError_t gram_b(const StreamArgs& a, double* gm) {
  int64_t tpg, gu, nt;
  grid_of(a.n, kGramGroups, &tpg, &gu, &nt);
  const size_t lds = gram_lds_bytes(a.m_pad, TTR_BF16) + (SKB > 0 ? gram_sketch_lds_bytes(SKB * 16, TTR_BF16) : 0);
  auto kern = kb_gram<PPW, NT, SKB>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  if (!part_fits(a, gu, a.m_pad * a.m_pad, sizeof(double))) return hipErrorInvalidValue;
  float* part_y = nullptr;
  if (SKB > 0) {
    const size_t off = gram_part_bytes(gu, a.m_pad);
    if (off + (size_t)gu * a.m_pad * SKB * 16 * sizeof(float) > a.part_bytes) return hipErrorInvalidValue;
    part_y = reinterpret_cast<float*>(static_cast<char*>(a.part) + off);
  }
  if ((e = mark_event(a.ev_begin, a.stream)) != hipSuccess) return e;
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)gu), dim3(NT), lds, a.stream, (const bf16*)a.A, a.m, a.n,
                       (int)a.m_pad, (double*)a.part, tpg, nt, a.seed, a.kmode, a.s, part_y);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = mark_event(a.ev_end, a.stream)) != hipSuccess) return e;
  e = launch_reduce_gram((const double*)a.part, gu, (int)a.m_pad, (int)a.m, gm, a.stream);
  if (e != hipSuccess || SKB == 0) return e;
  return launch_reduce_f32(part_y, gu, a.m_pad * (int64_t)(SKB * 16), (int)a.m, SKB * 16, a.s, a.y, a.ldy, a.stream);
}

hipError_t launch_fused_bf16(const StreamArgs& a) {
  const int SB = a.S / 16;
  const int apw = (int)((a.m_pad / 16 + kWaves - 1) / kWaves);
#define TTR_B(SBv, APWv) \
  if (SB == SBv && apw <= APWv) return fused_b<SBv, APWv>(a);
#define TTR_BA(SBv) TTR_B(SBv, 2) TTR_B(SBv, 4) TTR_B(SBv, 6) TTR_B(SBv, 8)
  TTR_BA(1) TTR_BA(2) TTR_BA(3) TTR_BA(4)
#undef TTR_BA
#undef TTR_B
  return hipErrorInvalidValue;
}

hipError_t launch_aw_bf16(const StreamArgs& a) {
  switch (a.S / 16) {
    case 1: return aw_b<1>(a);
    case 2: return aw_b<2>(a);
    case 3: return aw_b<3>(a);
    case 4: return aw_b<4>(a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_aw_omega_bf16(const StreamArgs& a) {
  switch (a.S / 16) {
    case 1: return aw_b<1, true>(a);
    case 2: return aw_b<2, true>(a);
    case 3: return aw_b<3, true>(a);
    case 4: return aw_b<4, true>(a);
  }
  return hipErrorInvalidValue;
}

template <typename TO, int OUTMODE>
static hipError_t atz_b_dispatch(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  switch (a.S / 16) {
    case 1: return atz_b<TO, 1, OUTMODE>(a, out, ldo, s_out);
    case 2: return atz_b<TO, 2, OUTMODE>(a, out, ldo, s_out);
    case 3: return atz_b<TO, 3, OUTMODE>(a, out, ldo, s_out);
    case 4: return atz_b<TO, 4, OUTMODE>(a, out, ldo, s_out);
  }
  return hipErrorInvalidValue;
}

// y[(c n2 + i2) ldy + j] = sum over u < gpb of part_y[i2 gpb + u][c][j] (c < r1, j < s2), in
// float64 and in group order.
__global__ __launch_bounds__(256) void k_carry_sketch_reduce(const float* __restrict__ part_y, int gpb, int64_t n2,
                                                             int R, int YC, int r1, int s2, double* __restrict__ y,
                                                             int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r1 * n2 * s2) return;
  const int j = (int)(idx % s2);
  const int64_t row = idx / s2;  // c n2 + i2
  const int c = (int)(row / n2);
  const int64_t i2 = row - (int64_t)c * n2;
  const float* p = part_y + (i2 * gpb) * (int64_t)R * YC + c * YC + j;
  double acc = 0.0;
  for (int u = 0; u < gpb; ++u) acc += (double)p[(int64_t)u * R * YC];
  y[row * ldy + j] = acc;
}

bool carry_sketch_fits(int dtype, int64_t m_pad, int S, int64_t n, int64_t nc, int S2) {
  return dtype == TTR_BF16 && m_pad <= 256 && S >= 16 && S <= 32 && S % 16 == 0 && S2 >= 16 && S2 <= 48 &&
         S2 % 16 == 0 && nc >= BT && nc % BT == 0 && n % nc == 0;
}

size_t carry_sketch_part_bytes(int64_t n, int64_t nc, int S, int S2) {
  const int64_t n2 = n / nc, tb = nc / BT;
  const int64_t gpb = std::max<int64_t>(1, std::min<int64_t>(tb, kMaxGroups / n2));
  return (size_t)(n2 * gpb) * S * S2 * sizeof(float);
}

hipError_t launch_carry_sketch_bf16(const StreamArgs& a, float* out, int64_t ldo, int s_out, const float* omt, int64_t nc,
                                    int S2, int s2, double* y, int64_t ldy) {
  if (!carry_sketch_fits(a.dtype, a.m_pad, a.S, a.n, nc, S2) || s_out > a.S || s2 > S2) return hipErrorInvalidValue;
  const int64_t n2 = a.n / nc, tb = nc / BT;
  const int64_t gpb = std::max<int64_t>(1, std::min<int64_t>(tb, kMaxGroups / n2));
  if (!a.part || carry_sketch_part_bytes(a.n, nc, a.S, S2) > a.part_bytes) return hipErrorInvalidValue;
  float* part_y = static_cast<float*>(a.part);
  const bool k4 = a.m_pad <= 128;
  hipError_t e = hipErrorInvalidValue;
#define TTR_CS(SBv, SK2v) \
  e = k4 ? carry_sketch_b<SBv, 4, SK2v>(a, out, ldo, s_out, omt, nc, n2, part_y) \
         : carry_sketch_b<SBv, 8, SK2v>(a, out, ldo, s_out, omt, nc, n2, part_y);
  if (a.S == 16) {
    if (S2 == 16) { TTR_CS(1, 1) } else if (S2 == 32) { TTR_CS(1, 2) } else { TTR_CS(1, 3) }
  } else {
    if (S2 == 16) { TTR_CS(2, 1) } else if (S2 == 32) { TTR_CS(2, 2) } else { TTR_CS(2, 3) }
  }
#undef TTR_CS
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)s_out * n2 * s2;
  hipLaunchKernelGGL(k_carry_sketch_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, a.stream, part_y,
                     (int)gpb, n2, a.S, S2, s_out, s2, y, ldy);
  return hipGetLastError();
}

hipError_t launch_atz_bf16(const StreamArgs& a, void* out, int out_dtype, int64_t ldo, int s_out, int outmode) {
  if (out_dtype == TTR_BF16)
    return outmode == 0 ? atz_b_dispatch<bf16, 0>(a, out, ldo, s_out) : atz_b_dispatch<bf16, 1>(a, out, ldo, s_out);
  if (out_dtype == TTR_F32)
    return outmode == 0 ? atz_b_dispatch<float, 0>(a, out, ldo, s_out) : atz_b_dispatch<float, 1>(a, out, ldo, s_out);
  return hipErrorInvalidValue;
}

// LDS of kb_gram_sb<SKB, TPI>: TPI A tiles, two transposed Omega tiles of pitch TPI BT + 8
// and the m_pad x S float32 sketch sums (SKB > 0)
template <int SKB, int TPI>
static size_t gram_sb_lds(int64_t m_pad) {
  return (size_t)TPI * gram_lds_bytes((m_pad + 63) / 64 * 64, TTR_BF16) +
         (SKB > 0 ? (size_t)2 * SKB * 16 * gram_sb_op<TPI, SKB>() * 2 + (size_t)m_pad * SKB * 16 * 4 : 0);
}

template <int SKB = 0>
static hipError_t gram_sb(const StreamArgs& a, double* gm) {
  int64_t tpg, gu, nt;
  grid_of(a.n, kGramGroups, &tpg, &gu, &nt);
  // two tiles per barrier interval when their LDS fits
  const bool two = gram_sb_lds<SKB, 2>(a.m_pad) <= kLdsBytes;
  const size_t lds = two ? gram_sb_lds<SKB, 2>(a.m_pad) : gram_sb_lds<SKB, 1>(a.m_pad);
  auto kern = two ? kb_gram_sb<SKB, 2> : kb_gram_sb<SKB, 1>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  if (!part_fits(a, gu, a.m_pad * a.m_pad, sizeof(double))) return hipErrorInvalidValue;
  float* part_y = nullptr;
  if (SKB > 0) {
    const size_t off = gram_part_bytes(gu, a.m_pad);
    if (off + (size_t)gu * a.m_pad * SKB * 16 * sizeof(float) > a.part_bytes) return hipErrorInvalidValue;
    part_y = reinterpret_cast<float*>(static_cast<char*>(a.part) + off);
  }
  if ((e = mark_event(a.ev_begin, a.stream)) != hipSuccess) return e;
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)gu), dim3(kGramBigThreads), lds, a.stream, (const bf16*)a.A, a.m,
                       a.n, (int)a.m_pad, (double*)a.part, tpg, nt, a.seed, a.kmode, a.s, part_y);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = mark_event(a.ev_end, a.stream)) != hipSuccess) return e;
  e = launch_reduce_gram((const double*)a.part, gu, (int)a.m_pad, (int)a.m, gm, a.stream);
  if (e != hipSuccess || SKB == 0) return e;
  return launch_reduce_f32(part_y, gu, a.m_pad * (int64_t)(SKB * 16), (int)a.m, SKB * 16, a.s, a.y, a.ldy, a.stream);
}

hipError_t launch_gram_bf16(const StreamArgs& a, double* gm) {
  const int MB = (int)(a.m_pad / 16);
  if (MB > kGramMaxM / 16) {  // 128 < m_pad <= 256: register-blocked super-blocks
    if (MB > kGramBigM / 16) return hipErrorInvalidValue;
    return gram_sb(a, gm);
  }
  const int ppw = (MB * (MB + 1) / 2 + kWaves - 1) / kWaves;
  if (ppw <= 1) return gram_b<1>(a, gm);
  if (ppw <= 3) return gram_b<3>(a, gm);
  if (ppw <= 5) return gram_b<5>(a, gm);
  if (ppw <= 9) return gram_b<9>(a, gm);
  return hipErrorInvalidValue;
}

template <int SKB>
static hipError_t gram_sketch_b(const StreamArgs& a, double* gm) {
  const int MB = (int)(a.m_pad / 16);
  if (MB > kGramMaxM / 16) {
    if (MB > kGramBigM / 16) return hipErrorInvalidValue;
    return gram_sb<SKB>(a, gm);
  }
  const int ppw = (MB * (MB + 1) / 2 + kWaves - 1) / kWaves;
  if (ppw <= 3) return gram_b<3, kThreads, SKB>(a, gm);
  return gram_b<9, kThreads, SKB>(a, gm);
}

hipError_t launch_gram_sketch_bf16(const StreamArgs& a, double* gm) {
  switch (a.S / 16) {
    case 1: return gram_sketch_b<1>(a, gm);
    case 2: return gram_sketch_b<2>(a, gm);
    case 3: return gram_sketch_b<3>(a, gm);
    case 4: return gram_sketch_b<4>(a, gm);
  }
  return hipErrorInvalidValue;
}

// Float32 A W and A^T Z / carry on the bf16 matrix cores (split operands).
template <int SB, int WM>
static hipError_t aw_split_b(const StreamArgs& a) {
  constexpr bool OM = WM == 1;
  const int64_t ntiles = (a.n + kSplitTT - 1) / kSplitTT;
  const int64_t rb = (a.m_pad + kAwRows - 1) / kAwRows;
  if (OM && rb != 1) return hipErrorInvalidValue;
  const size_t lds = aw_split_lds_bytes(SB * 16, OM);
  auto kern = kb_aw_s<SB, WM>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int64_t G = groups_for(ntiles, std::max<int64_t>(1, kMaxGroups / rb));
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t gu = (ntiles + tpg - 1) / tpg;
  if (!part_fits(a, gu, a.m_pad * SB * 16, sizeof(float))) return hipErrorInvalidValue;
  if ((e = mark_event(a.ev_begin, a.stream)) != hipSuccess) return e;
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)gu, (unsigned)rb), dim3(kThreads), lds, a.stream, (const float*)a.A, a.m,
                       a.n, (int)a.m_pad, a.W, split_w_ld(a.n), (float*)a.part, tpg, ntiles, a.seed, a.kmode, a.s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = mark_event(a.ev_end, a.stream)) != hipSuccess) return e;
  return launch_reduce_f32((const float*)a.part, gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y,
                           a.ldy, a.stream);
}

template <int OUTMODE, int SB>
static hipError_t atz_split_b(const StreamArgs& a, float* out, int64_t ldo, int s_out) {
  const int64_t ntiles = (a.n + kSplitTC - 1) / kSplitTC;
  const int64_t G = groups_for(ntiles, kMaxGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = atz_split_lds_bytes(SB * 16);
  auto kern = kb_atz_s<float, SB, OUTMODE>;
  hipError_t e = b_set_lds(kern, lds);
  if (e != hipSuccess) return e;
  // Z split into its planes in the partials region (this kernel writes no partials)
  const int ldz = (int)((a.m_pad + kSplitRC - 1) / kSplitRC * kSplitRC);
  if (!a.part || (size_t)3 * SB * 16 * ldz * sizeof(bf16) > a.part_bytes) return hipErrorInvalidValue;
  bf16* zp = static_cast<bf16*>(a.part);
  hipLaunchKernelGGL(k_split_planes, dim3((unsigned)(((int64_t)ldz * SB * 16 + 255) / 256)), dim3(256), 0, a.stream,
                     (const float*)a.Z, (int)a.m_pad, SB * 16, ldz, zp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = mark_event(a.ev_begin, a.stream)) != hipSuccess) return e;
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)gu), dim3(kThreads), lds, a.stream, (const float*)a.A, a.m, a.n,
                       (int)a.m_pad, (const bf16*)zp, ldz, out, ldo, s_out, tpg, ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return mark_event(a.ev_end, a.stream);
}

hipError_t launch_aw_split(const StreamArgs& a, bool omega) {
  if (a.dtype != TTR_F32) return hipErrorInvalidValue;
  const int wm = omega ? 1 : (a.w_f32 ? 0 : 2);
#define TTR_AWS(SBv) \
  return wm == 1 ? aw_split_b<SBv, 1>(a) : (wm == 0 ? aw_split_b<SBv, 0>(a) : aw_split_b<SBv, 2>(a));
  switch (a.S / 16) {
    case 1: TTR_AWS(1)
    case 2: TTR_AWS(2)
    case 3: TTR_AWS(3)
    case 4: TTR_AWS(4)
  }
#undef TTR_AWS
  return hipErrorInvalidValue;
}

hipError_t launch_atz_split(const StreamArgs& a, void* out, int64_t ldo, int s_out, int outmode) {
  if (a.dtype != TTR_F32) return hipErrorInvalidValue;
  float* o = static_cast<float*>(out);
  // outmode 0 writes W as the three bf16 planes launch_aw_split reads (row pitch split_w_ld(n))
  const int64_t lw = split_w_ld(a.n);
  switch (a.S / 16) {
    case 1: return outmode == 0 ? atz_split_b<2, 1>(a, o, lw, s_out) : atz_split_b<1, 1>(a, o, ldo, s_out);
    case 2: return outmode == 0 ? atz_split_b<2, 2>(a, o, lw, s_out) : atz_split_b<1, 2>(a, o, ldo, s_out);
    case 3: return outmode == 0 ? atz_split_b<2, 3>(a, o, lw, s_out) : atz_split_b<1, 3>(a, o, ldo, s_out);
    case 4: return outmode == 0 ? atz_split_b<2, 4>(a, o, lw, s_out) : atz_split_b<1, 4>(a, o, ldo, s_out);
  }
  return hipErrorInvalidValue;
}

}  // namespace ttr
