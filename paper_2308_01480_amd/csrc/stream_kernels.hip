// Streaming kernels over the wide unfolding A (m x n, row-major, n >> m).
//
// Every kernel walks A in column tiles of TT columns (16 float64 / 32 float32 /
// 64 bfloat16), stages each tile once through LDS and feeds the matrix cores
// (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x32_bf16).
// A work-group owns a contiguous range of tiles and keeps its results in
// registers; per-work-group partial sums are reduced afterwards in a fixed order,
// so every result is bitwise reproducible.  All index arithmetic is 64-bit.
//
//   k_fused   Y = A (A^T Z)      one pass: W_J = A_J^T Z stays on chip, Y += A_J W_J
//                                (the Krylov block product of Algorithm 3, step 4)
//   k_aw      Y = A W            W (n x S) streamed with A (sketch A Omega; second
//                                half of the two-pass Krylov product for tall A)
//   k_atz     W = A^T Z          written out as n x S (two-pass) or as the S x n
//                                carry G^T A (Algorithm 3, step 10)
//   k_gram    A A^T              short-side Gram of saturated modes
//   k_omega   Omega_k            Philox4x64-10 + Box-Muller (Algorithm 3, step 3)
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace ttr {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// ----------------------------------------------------------------------------------
// Matrix-core traits.  For 16x16x4 (float32/float64) lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; the 16x16 result lands as 4 values per lane in column l%16 and
// rows orow(l, r).  For 16x16x32 bfloat16 lane l supplies 8 consecutive k values
// 8*(l/16) .. 8*(l/16)+7 of row (A) / column (B) l%16.
// ----------------------------------------------------------------------------------
template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef f4_t acc;
  typedef float scalar;
  static constexpr int K = 4;
  __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mma<double> {
  typedef d4_t acc;
  typedef double scalar;
  static constexpr int K = 4;
  __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int orow(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T> __device__ __host__ constexpr int tile_cols_t() { return sizeof(T) == 8 ? 16 : 32; }

// ----------------------------------------------------------------------------------
// Tile staging.  A tile is `rows` (multiple of 16) x TT columns starting at (row0, col0).
// fetch() issues the global loads into registers (16-byte vectors when the tile is
// whole and aligned, guarded scalar loads otherwise); commit() writes them to LDS
// with row pitch TT+1.  Rows >= m and columns >= n are zero.
// ----------------------------------------------------------------------------------
template <typename T, int MAXV>
struct TileRegs {
  static constexpr int VEC = 16 / sizeof(T);
  static constexpr int TT = tile_cols_t<T>();
  static constexpr int VPR = TT / VEC;
  u4_t v[MAXV];

  __device__ void fetch(const T* __restrict__ A, int64_t m, int64_t n, int64_t row0, int rows, int64_t col0,
                        bool aligned) {
    const int nv = rows * VPR;
    const bool full = aligned && (col0 + TT <= n);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = (int)threadIdx.x + i * kThreads;
      u4_t val = u4_t{0u, 0u, 0u, 0u};
      if (idx < nv) {
        const int rr = idx / VPR, cv = idx % VPR;
        const int64_t row = row0 + rr;
        if (row < m) {
          const T* src = A + row * n + col0 + (int64_t)cv * VEC;
          if (full) {
            val = *reinterpret_cast<const u4_t*>(src);
          } else {
            T tmp[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) tmp[e] = (col0 + cv * VEC + e < n) ? src[e] : T(0);
            val = *reinterpret_cast<u4_t*>(tmp);
          }
        }
      }
      v[i] = val;
    }
  }

  __device__ void commit(T* __restrict__ As, int rows) const {
    constexpr int AP = TT + 1;
    const int nv = rows * VPR;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = (int)threadIdx.x + i * kThreads;
      if (idx < nv) {
        const int rr = idx / VPR, cv = idx % VPR;
        T tmp[VEC];
        *reinterpret_cast<u4_t*>(tmp) = v[i];
#pragma unroll
        for (int e = 0; e < VEC; ++e) As[rr * AP + cv * VEC + e] = tmp[e];
      }
    }
  }
};

__device__ inline bool ptr_aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// ----------------------------------------------------------------------------------
// Phase 1: W (TT x S) = A_J^T Z over LDS rows [0, rows): the K (row) dimension is split
// across the waves; each wave leaves its partial W in Wp[wave] and the waves' partials
// are summed in a fixed order into Wp[0].
// ----------------------------------------------------------------------------------
template <typename T, int SB>
__device__ inline void phase1_accumulate(const T* __restrict__ As, const T* __restrict__ Zs, int rows,
                                         typename Mma<T>::acc (&acc1)[tile_cols_t<T>() / 16][SB]) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), TB = TT / 16, S = SB * 16, AP = TT + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int ks = wave; ks < rows / 4; ks += kWaves) {
    const int row = ks * 4 + (lane >> 4);
    T a[TB], b[SB];
#pragma unroll
    for (int tb = 0; tb < TB; ++tb) a[tb] = As[row * AP + tb * 16 + (lane & 15)];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) b[sb] = Zs[row * S + sb * 16 + (lane & 15)];
#pragma unroll
    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc1[tb][sb] = M::mma(a[tb], b[sb], acc1[tb][sb]);
  }
}

template <typename T, int SB>
__device__ inline void phase1_reduce(typename Mma<T>::acc (&acc1)[tile_cols_t<T>() / 16][SB], T* __restrict__ Wp) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), TB = TT / 16, S = SB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* Wme = Wp + wave * TT * S;
#pragma unroll
  for (int tb = 0; tb < TB; ++tb)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Wme[(tb * 16 + M::orow(lane, r)) * S + sb * 16 + (lane & 15)] = acc1[tb][sb][r];
  __syncthreads();
  for (int e = threadIdx.x; e < TT * S; e += kThreads)
    Wp[e] = ((Wp[e] + Wp[TT * S + e]) + Wp[2 * TT * S + e]) + Wp[3 * TT * S + e];
  __syncthreads();
}

// Phase 2: Y (APW row blocks of 16 per wave x S) += A_J (rows x TT) W (TT x S).
template <typename T, int SB, int APW>
__device__ inline void phase2_accumulate(const T* __restrict__ As, const T* __restrict__ Ws, int rows,
                                         typename Mma<T>::acc (&acc2)[APW][SB]) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), S = SB * 16, AP = TT + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int ks = 0; ks < TT / 4; ++ks) {
    const int col = ks * 4 + (lane >> 4);
    T b[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) b[sb] = Ws[col * S + sb * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < APW; ++i) {
      const int ab = wave + kWaves * i;
      if (ab * 16 < rows) {
        const T a = As[(ab * 16 + (lane & 15)) * AP + col];
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = M::mma(a, b[sb], acc2[i][sb]);
      }
    }
  }
}

template <typename T, int SB, int APW>
__device__ inline void store_rows(typename Mma<T>::acc (&acc2)[APW][SB], T* __restrict__ out, int rows, int row_off) {
  using M = Mma<T>;
  constexpr int S = SB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < APW; ++i) {
    const int ab = wave + kWaves * i;
    if (ab * 16 < rows) {
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(int64_t)(row_off + ab * 16 + M::orow(lane, r)) * S + sb * 16 + (lane & 15)] = acc2[i][sb][r];
    }
  }
}

// ----------------------------------------------------------------------------------
// k_fused: partial[g] (m_pad x S) = sum over the group's tiles of A_J (A_J^T Z).
// LDS: A tile (m_pad x TT+1) | Z (m_pad x S) | W partials (4 x TT x S).
// The next tile's global loads are issued before the current tile is computed.
// ----------------------------------------------------------------------------------
template <typename T, int SB, int APW>
__global__ __launch_bounds__(kThreads) void k_fused(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                    const T* __restrict__ Zg, T* __restrict__ part,
                                                    int64_t tiles_per_group, int64_t ntiles) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), TB = TT / 16, S = SB * 16, AP = TT + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Zs = As + m_pad * AP;
  T* Wp = Zs + m_pad * S;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(T)) % 16 == 0);

  for (int e = threadIdx.x; e < m_pad * S; e += kThreads) Zs[e] = Zg[e];
  typename M::acc acc2[APW][SB];
#pragma unroll
  for (int i = 0; i < APW; ++i)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = M::zero();

  TileRegs<T, 2 * APW> regs;
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad, t0 * TT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(As, m_pad);
    __syncthreads();
    if (t + 1 < t1) regs.fetch(A, m, n, 0, m_pad, (t + 1) * TT, aligned);
    typename M::acc acc1[TB][SB];
#pragma unroll
    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc1[tb][sb] = M::zero();
    phase1_accumulate<T, SB>(As, Zs, m_pad, acc1);
    phase1_reduce<T, SB>(acc1, Wp);
    phase2_accumulate<T, SB, APW>(As, Wp, m_pad, acc2);
  }
  store_rows<T, SB, APW>(acc2, part + g * (int64_t)m_pad * S, m_pad, 0);
}

// ----------------------------------------------------------------------------------
// k_aw: partial[g] rows [rb*256, rb*256+256) += A_J W_J, W (n x S) streamed from HBM.
// Grid (column group g, row block rb).
// ----------------------------------------------------------------------------------
template <typename T, int SB>
__global__ __launch_bounds__(kThreads) void k_aw(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                 const T* __restrict__ W, T* __restrict__ part,
                                                 int64_t tiles_per_group, int64_t ntiles) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), S = SB * 16, AP = TT + 1;
  constexpr int APW = kAwRows / (16 * kWaves);
  constexpr int WVEC = 16 / sizeof(T);
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Ws = As + kAwRows * AP;
  const int64_t g = blockIdx.x;
  const int row0 = blockIdx.y * kAwRows;
  const int rows = (m_pad - row0) < kAwRows ? (m_pad - row0) : kAwRows;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(T)) % 16 == 0);

  typename M::acc acc2[APW][SB];
#pragma unroll
  for (int i = 0; i < APW; ++i)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = M::zero();

  TileRegs<T, 2 * APW> regs;
  if (t0 < t1) regs.fetch(A, m, n, row0, rows, t0 * TT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(As, rows);
    // W tile rows [t*TT, t*TT+TT) are one contiguous TT x S block
    const int64_t wrow0 = t * TT;
    for (int e = threadIdx.x; e < TT * S / WVEC; e += kThreads) {
      const int rr = e / (S / WVEC);
      u4_t val = u4_t{0u, 0u, 0u, 0u};
      if (wrow0 + rr < n) val = reinterpret_cast<const u4_t*>(W + wrow0 * S)[e];
      reinterpret_cast<u4_t*>(Ws)[e] = val;
    }
    __syncthreads();
    if (t + 1 < t1) regs.fetch(A, m, n, row0, rows, (t + 1) * TT, aligned);
    phase2_accumulate<T, SB, APW>(As, Ws, rows, acc2);
  }
  store_rows<T, SB, APW>(acc2, part + g * (int64_t)m_pad * S, rows, row0);
}

// ----------------------------------------------------------------------------------
// k_atz: W_J = A_J^T Z for every tile; rows processed in chunks of kRowChunk with
// Z chunk and A chunk in LDS.  Output mode 0: out[(beta) * ldo + c] (n x S, all S
// columns); mode 1: out[c * ldo + beta] for c < s_out (the S x n carry, transposed).
// ----------------------------------------------------------------------------------
template <typename T, typename TO, int SB, int OUTMODE, int RC>
__global__ __launch_bounds__(kThreads) void k_atz(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                  const T* __restrict__ Zg, TO* __restrict__ out, int64_t ldo,
                                                  int s_out, int64_t tiles_per_group, int64_t ntiles) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), TB = TT / 16, S = SB * 16;
  constexpr int kRowChunk = RC;
  constexpr int MAXV = 2 * (kRowChunk / (16 * kWaves));
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Zs = As + kRowChunk * (TT + 1);
  T* Wp = Zs + kRowChunk * S;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(T)) % 16 == 0);
  const int nchunks = (m_pad + kRowChunk - 1) / kRowChunk;

  if (nchunks == 1)
    for (int e = threadIdx.x; e < m_pad * S; e += kThreads) Zs[e] = Zg[e];
  TileRegs<T, MAXV> regs;
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad < kRowChunk ? m_pad : kRowChunk, t0 * TT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    typename M::acc acc1[TB][SB];
#pragma unroll
    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc1[tb][sb] = M::zero();
    for (int c = 0; c < nchunks; ++c) {
      const int row0 = c * kRowChunk;
      const int rows = (m_pad - row0) < kRowChunk ? (m_pad - row0) : kRowChunk;
      __syncthreads();
      regs.commit(As, rows);
      if (nchunks > 1)
        for (int e = threadIdx.x; e < rows * S; e += kThreads) Zs[e] = Zg[(int64_t)row0 * S + e];
      __syncthreads();
      // prefetch the next (tile, chunk) block
      if (c + 1 < nchunks) {
        const int nr0 = (c + 1) * kRowChunk;
        regs.fetch(A, m, n, nr0, (m_pad - nr0) < kRowChunk ? (m_pad - nr0) : kRowChunk, t * TT, aligned);
      } else if (t + 1 < t1) {
        regs.fetch(A, m, n, 0, m_pad < kRowChunk ? m_pad : kRowChunk, (t + 1) * TT, aligned);
      }
      phase1_accumulate<T, SB>(As, Zs, rows, acc1);
    }
    phase1_reduce<T, SB>(acc1, Wp);
    const int64_t b0 = t * TT;
    if (OUTMODE == 0) {
      for (int e = threadIdx.x; e < TT * S; e += kThreads) {
        const int bb = e / S, c = e % S;
        if (b0 + bb < n) out[(b0 + bb) * ldo + c] = (TO)Wp[e];
      }
    } else {
      for (int e = threadIdx.x; e < TT * s_out; e += kThreads) {
        const int c = e / TT, bb = e % TT;
        if (b0 + bb < n) out[(int64_t)c * ldo + b0 + bb] = (TO)Wp[bb * S + c];
      }
    }
  }
}

// ----------------------------------------------------------------------------------
// k_gram: partial[g] (m_pad x m_pad, upper 16x16 blocks) = sum_J A_J A_J^T, m_pad <= 128.
// float32 / bfloat16 products are summed per tile on the matrix cores in float32 and
// folded into float64 accumulators after every tile.
// ----------------------------------------------------------------------------------
template <typename T, int PPW>
__global__ __launch_bounds__(kThreads) void k_gram(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                   double* __restrict__ part, int64_t tiles_per_group,
                                                   int64_t ntiles) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), AP = TT + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(T)) % 16 == 0);
  const int MB = m_pad / 16;
  const int npairs = MB * (MB + 1) / 2;
  int pa[PPW], pb[PPW];
#pragma unroll
  for (int i = 0; i < PPW; ++i) {
    int p = wave + kWaves * i, a = 0;
    pa[i] = -1; pb[i] = -1;
    if (p < npairs) {
      while (p >= MB - a) { p -= MB - a; ++a; }
      pa[i] = a; pb[i] = a + p;
    }
  }
  double acc[PPW][4];
#pragma unroll
  for (int i = 0; i < PPW; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[i][r] = 0.0;

  TileRegs<T, kGramMaxM * TileRegs<T, 1>::VPR / kThreads> regs;  // m_pad <= 128 rows per tile
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad, t0 * TT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(As, m_pad);
    __syncthreads();
    if (t + 1 < t1) regs.fetch(A, m, n, 0, m_pad, (t + 1) * TT, aligned);
#pragma unroll
    for (int i = 0; i < PPW; ++i) {
      if (pa[i] >= 0) {
        typename M::acc c = M::zero();
#pragma unroll
        for (int ks = 0; ks < TT / 4; ++ks) {
          const T a = As[(pa[i] * 16 + (lane & 15)) * AP + ks * 4 + (lane >> 4)];
          const T b = As[(pb[i] * 16 + (lane & 15)) * AP + ks * 4 + (lane >> 4)];
          c = M::mma(a, b, c);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][r] += (double)c[r];
      }
    }
  }
  double* out = part + g * (int64_t)m_pad * m_pad;
#pragma unroll
  for (int i = 0; i < PPW; ++i)
    if (pa[i] >= 0)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(pa[i] * 16 + M::orow(lane, r)) * m_pad + pb[i] * 16 + (lane & 15)] = acc[i][r];
}

// ----------------------------------------------------------------------------------
// Omega: Philox4x64-10 (Salmon et al. 2011) and Box-Muller in float64.
// ----------------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t hi0 = __umul64hi(M0, x[0]), lo0 = M0 * x[0];
    const uint64_t hi1 = __umul64hi(M1, x[2]), lo1 = M1 * x[2];
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = lo1; x[2] = y2; x[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

__device__ inline double unit_open(uint64_t x) { return ((double)(x >> 12) + 0.5) * 0x1p-52; }

// Four normals of group g (entries c = 4g .. 4g+3) of row beta of Omega_k.
__device__ inline void omega4(uint64_t seed, int k, int64_t beta, int g, double (&z)[4]) {
  uint64_t x[4] = {(uint64_t)beta, (uint64_t)g, 0ull, 0ull};
  philox4x64_10(x, seed, (uint64_t)k);
  const double two_pi = 6.283185307179586;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double rad = sqrt(-2.0 * log(unit_open(x[2 * h])));
    const double th = two_pi * unit_open(x[2 * h + 1]);
    double sn, cs;
    sincos(th, &sn, &cs);
    z[2 * h] = rad * cs;
    z[2 * h + 1] = rad * sn;
  }
}

template <typename TO>
__global__ __launch_bounds__(256) void k_omega(uint64_t seed, int k, int64_t beta0, int64_t nrows, int s, int ldo,
                                               TO* __restrict__ out) {
  const int G4 = (ldo + 3) / 4;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrows * G4) return;
  const int64_t rr = idx / G4;
  const int g = (int)(idx % G4);
  double z[4];
  omega4(seed, k, beta0 + rr, g, z);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * g + j;
    if (c < ldo) out[rr * ldo + c] = c < s ? (TO)z[j] : (TO)0;
  }
}

// ----------------------------------------------------------------------------------
// Deterministic reductions of per-work-group partials.
// ----------------------------------------------------------------------------------
// Eight interleaved accumulators keep eight loads in flight per thread; they are
// combined in a fixed order, so the sum is bitwise reproducible.
template <typename P>
__device__ inline double strided_sum(const P* __restrict__ p, int64_t groups, int64_t stride) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t g = 0;
  for (; g + 8 <= groups; g += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += (double)p[(g + u) * stride];
  for (int u = 0; g < groups; ++g, ++u) a[u] += (double)p[g * stride];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

template <typename P>
__global__ __launch_bounds__(256) void k_reduce(const P* __restrict__ part, int64_t groups, int64_t stride, int m,
                                                int S, int s, double* __restrict__ y, int ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * s) return;
  const int i = (int)(idx / s), c = (int)(idx % s);
  y[(int64_t)i * ldy + c] = strided_sum(part + (int64_t)i * S + c, groups, stride);
}

__global__ __launch_bounds__(256) void k_reduce_gram(const double* __restrict__ part, int64_t groups, int m_pad,
                                                     int m, double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  int i = (int)(idx / m), j = (int)(idx % m);
  if (i / 16 > j / 16) { const int t = i; i = j; j = t; }
  out[idx] = strided_sum(part + (int64_t)i * m_pad + j, groups, (int64_t)m_pad * m_pad);
}

// ----------------------------------------------------------------------------------
// Host launchers.
// ----------------------------------------------------------------------------------
template <typename F>
static hipError_t set_lds(F kernel, size_t bytes) {
  if (bytes > kLdsBytes) return hipErrorInvalidValue;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) (void)hipGetLastError();  // do not leave a sticky error behind
  return e;
}

#define TTR_HIP(x)                                   \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return e_;                 \
  } while (0)

template <typename T, int SB, int APW>
static hipError_t launch_fused_t(const StreamArgs& a) {
  constexpr int TT = tile_cols_t<T>();
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t G = groups_for(ntiles, kMaxGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = fused_lds_bytes(a.m_pad, SB * 16, sizeof(T) == 8 ? TTR_F64 : TTR_F32);
  auto kern = k_fused<T, SB, APW>;
  TTR_HIP(set_lds(kern, lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m, a.n, (int)a.m_pad,
                     (const T*)a.Z, (T*)a.part, tpg, ntiles);
  TTR_HIP(hipGetLastError());
  const int64_t total = a.m * a.s;
  hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, a.stream, (const T*)a.part,
                     Gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y, a.ldy);
  return hipGetLastError();
}

template <typename T, int SB>
static hipError_t launch_aw_t(const StreamArgs& a) {
  constexpr int TT = tile_cols_t<T>();
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t rb = (a.m_pad + kAwRows - 1) / kAwRows;
  const int64_t G = groups_for(ntiles, std::max<int64_t>(1, kMaxGroups / rb));
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = aw_lds_bytes(SB * 16, sizeof(T) == 8 ? TTR_F64 : TTR_F32);
  auto kern = k_aw<T, SB>;
  TTR_HIP(set_lds(kern, lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu, (unsigned)rb), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m, a.n,
                     (int)a.m_pad, (const T*)a.W, (T*)a.part, tpg, ntiles);
  TTR_HIP(hipGetLastError());
  const int64_t total = a.m * a.s;
  hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, a.stream, (const T*)a.part,
                     Gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y, a.ldy);
  return hipGetLastError();
}

template <typename T, typename TO, int SB, int OUTMODE>
static hipError_t launch_atz_t(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  constexpr int TT = tile_cols_t<T>();
  constexpr int DT = sizeof(T) == 8 ? TTR_F64 : TTR_F32;
  constexpr int RC = atz_row_chunk(SB * 16, DT);
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t G = groups_for(ntiles, kMaxGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = atz_lds_bytes(SB * 16, DT);
  auto kern = k_atz<T, TO, SB, OUTMODE, RC>;
  TTR_HIP(set_lds(kern, lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m, a.n,
                     (int)a.m_pad, (const T*)a.Z, (TO*)out, ldo, s_out, tpg, ntiles);
  return hipGetLastError();
}

template <typename T, int PPW>
static hipError_t launch_gram_t(const StreamArgs& a, double* gm) {
  constexpr int TT = tile_cols_t<T>();
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t G = groups_for(ntiles, kGramGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = gram_lds_bytes(a.m_pad, sizeof(T) == 8 ? TTR_F64 : TTR_F32);
  auto kern = k_gram<T, PPW>;
  TTR_HIP(set_lds(kern, lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m, a.n,
                     (int)a.m_pad, (double*)a.part, tpg, ntiles);
  TTR_HIP(hipGetLastError());
  const int64_t total = a.m * a.m;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, a.stream,
                     (const double*)a.part, Gu, (int)a.m_pad, (int)a.m, gm);
  return hipGetLastError();
}

// Dispatch on (dtype, S/16, rows per wave).
template <typename T>
static hipError_t fused_dispatch(const StreamArgs& a) {
  const int SB = a.S / 16;
  const int apw = (int)((a.m_pad / 16 + kWaves - 1) / kWaves);
#define TTR_F(SBv, APWv) \
  if (SB == SBv && apw <= APWv) return launch_fused_t<T, SBv, APWv>(a);
#define TTR_FA(SBv) TTR_F(SBv, 1) TTR_F(SBv, 2) TTR_F(SBv, 4) TTR_F(SBv, 6) TTR_F(SBv, 8)
  TTR_FA(1) TTR_FA(2) TTR_FA(3) TTR_FA(4)
#undef TTR_FA
#undef TTR_F
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t aw_dispatch(const StreamArgs& a) {
  switch (a.S / 16) {
    case 1: return launch_aw_t<T, 1>(a);
    case 2: return launch_aw_t<T, 2>(a);
    case 3: return launch_aw_t<T, 3>(a);
    case 4: return launch_aw_t<T, 4>(a);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename TO, int OUTMODE>
static hipError_t atz_dispatch(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  switch (a.S / 16) {
    case 1: return launch_atz_t<T, TO, 1, OUTMODE>(a, out, ldo, s_out);
    case 2: return launch_atz_t<T, TO, 2, OUTMODE>(a, out, ldo, s_out);
    case 3: return launch_atz_t<T, TO, 3, OUTMODE>(a, out, ldo, s_out);
    case 4: return launch_atz_t<T, TO, 4, OUTMODE>(a, out, ldo, s_out);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t gram_dispatch(const StreamArgs& a, double* gm) {
  const int MB = (int)(a.m_pad / 16);
  const int ppw = (MB * (MB + 1) / 2 + kWaves - 1) / kWaves;
  if (ppw <= 1) return launch_gram_t<T, 1>(a, gm);
  if (ppw <= 3) return launch_gram_t<T, 3>(a, gm);
  if (ppw <= 5) return launch_gram_t<T, 5>(a, gm);
  if (ppw <= 9) return launch_gram_t<T, 9>(a, gm);
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_f32(const float* part, int64_t groups, int64_t stride, int m, int S, int s, double* y,
                             int ldy, hipStream_t st) {
  const int64_t total = (int64_t)m * s;
  hipLaunchKernelGGL(k_reduce<float>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, groups, stride,
                     m, S, s, y, ldy);
  return hipGetLastError();
}

hipError_t launch_reduce_gram(const double* part, int64_t groups, int m_pad, int m, double* out, hipStream_t st) {
  const int64_t total = (int64_t)m * m;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, groups, m_pad, m,
                     out);
  return hipGetLastError();
}

hipError_t launch_fused(const StreamArgs& a) {
  if (a.dtype == TTR_F64) return fused_dispatch<double>(a);
  if (a.dtype == TTR_F32) return fused_dispatch<float>(a);
  return launch_fused_bf16(a);
}

hipError_t launch_aw(const StreamArgs& a) {
  if (a.dtype == TTR_F64) return aw_dispatch<double>(a);
  if (a.dtype == TTR_F32) return aw_dispatch<float>(a);
  return launch_aw_bf16(a);
}

hipError_t launch_atz(const StreamArgs& a, void* out, int out_dtype, int64_t ldo, int s_out, int outmode) {
  if (a.dtype == TTR_F64) {
    if (out_dtype != TTR_F64) return hipErrorInvalidValue;
    return outmode == 0 ? atz_dispatch<double, double, 0>(a, out, ldo, s_out)
                        : atz_dispatch<double, double, 1>(a, out, ldo, s_out);
  }
  if (a.dtype == TTR_F32) {
    if (out_dtype != TTR_F32) return hipErrorInvalidValue;
    return outmode == 0 ? atz_dispatch<float, float, 0>(a, out, ldo, s_out)
                        : atz_dispatch<float, float, 1>(a, out, ldo, s_out);
  }
  return launch_atz_bf16(a, out, out_dtype, ldo, s_out, outmode);
}

hipError_t launch_gram(const StreamArgs& a, double* gm) {
  if (a.dtype == TTR_F64) return gram_dispatch<double>(a, gm);
  if (a.dtype == TTR_F32) return gram_dispatch<float>(a, gm);
  return launch_gram_bf16(a, gm);
}

hipError_t launch_omega(uint64_t seed, int k, int64_t beta0, int64_t nrows, int s, int ldo, void* out, int out_dtype,
                        hipStream_t st) {
  const int64_t total = nrows * ((ldo + 3) / 4);
  const dim3 grid((unsigned)((total + 255) / 256));
  if (out_dtype == TTR_F64)
    hipLaunchKernelGGL(k_omega<double>, grid, dim3(256), 0, st, seed, k, beta0, nrows, s, ldo, (double*)out);
  else if (out_dtype == TTR_F32)
    hipLaunchKernelGGL(k_omega<float>, grid, dim3(256), 0, st, seed, k, beta0, nrows, s, ldo, (float*)out);
  else
    hipLaunchKernelGGL(k_omega<__bf16>, grid, dim3(256), 0, st, seed, k, beta0, nrows, s, ldo, (__bf16*)out);
  return hipGetLastError();
}

}  // namespace ttr
