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

#include <algorithm>
#include <type_traits>

#include "common.h"
#include "convert.h"
#include "kernels.h"
#include "omega.h"

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
template <typename T, int MAXV, int NTH = kThreads, int TTC = tile_cols_t<T>()>
struct TileRegs {
  static constexpr int VEC = 16 / sizeof(T);
  static constexpr int TT = TTC;
  static constexpr int VPR = TT / VEC;
  u4_t v[MAXV];

  __device__ void fetch(const T* __restrict__ A, int64_t m, int64_t n, int64_t row0, int rows, int64_t col0,
                        bool aligned) {
    if (aligned && col0 + TT <= n) fetch_full(A, m, n, row0, rows, col0);
    else fetch_guarded(A, m, n, row0, rows, col0, false);
  }

  // Whole, 16-byte aligned tile: lane (r, cv) loads rows r, r + RSTEP, ... with one
  // 16-byte vector each; the row stride is uniform, so addresses stay per-lane base +
  // scalar offset.
  __device__ void fetch_full(const T* __restrict__ A, int64_t m, int64_t n, int64_t row0, int rows, int64_t col0) {
    constexpr int RSTEP = NTH / VPR;
    const int r_in = (int)threadIdx.x / VPR, cv = (int)threadIdx.x % VPR;
    const T* base = A + (row0 + r_in) * n + col0 + cv * VEC;
    const int64_t lim = (m - row0 < (int64_t)rows ? m - row0 : (int64_t)rows) - r_in;  // valid i * RSTEP < lim
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      u4_t val = u4_t{0u, 0u, 0u, 0u};
      if ((int64_t)i * RSTEP < lim) val = *reinterpret_cast<const u4_t*>(base + (int64_t)i * RSTEP * n);
      v[i] = val;
    }
  }

  __device__ void fetch_guarded(const T* __restrict__ A, int64_t m, int64_t n, int64_t row0, int rows, int64_t col0,
                                bool full) {
    const int nv = rows * VPR;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = (int)threadIdx.x + i * NTH;
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

  template <int PAD = 1>
  __device__ void commit(T* __restrict__ As, int rows) const {
    constexpr int AP = TT + PAD;
    const int nv = rows * VPR;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int idx = (int)threadIdx.x + i * NTH;
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
// k_fused_zr: the fused product for taller float32 unfoldings (512 < m_pad <= 1024,
// S <= 32), where the A tile alone fills LDS.  Z stays in registers instead: the
// K-steps (4 rows each) of A_J^T Z are dealt to the NWV = 8 waves round-robin, so
// wave w keeps the Z rows of its own K-steps, KPW = MPK / 32 of them.  The A tile
// (MPK x 16 columns) is staged in LDS once per tile and read by both products; the Y
// accumulators (MPK / 16 / NWV row blocks per wave) stay in registers.  Two waves per
// SIMD let one wave's matrix-core work cover the other's LDS reads.  Each wave leaves its
// partial W in its own LDS slot; one barrier later they are summed in a fixed order.
// ----------------------------------------------------------------------------------
constexpr int kZrWaves = 8;
constexpr int kZrThreads = 64 * kZrWaves;
constexpr int kZrTileCols = kFusedZrTileCols;

// CARRY = 1 stops after the first product and writes W_J^T into the carry C = Z^T A
// (s_out x n, leading dimension ldo) instead of accumulating A_J W_J.
template <int SB, int KPW, int CARRY>
__global__ __launch_bounds__(kZrThreads) void k_fused_zr(const float* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                         const float* __restrict__ Zg, float* __restrict__ part,
                                                         int64_t tiles_per_group, int64_t ntiles, int64_t ldo,
                                                         int s_out) {
  using M = Mma<float>;
  constexpr int NWV = kZrWaves;
  constexpr int TT = kZrTileCols, S = SB * 16, AP = TT + 1;
  constexpr int MPK = KPW * 4 * NWV;
  constexpr int APW = (MPK / 16 + NWV - 1) / NWV;
  extern __shared__ __align__(16) unsigned char smem[];
  float* As = reinterpret_cast<float*>(smem);
  float* Wp = As + MPK * AP;  // 8 slots of TT x S (one per wave), then the summed W
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(float)) % 16 == 0);

  float zr[KPW][SB];
#pragma unroll
  for (int i = 0; i < KPW; ++i) {
    const int row = 4 * (wave + NWV * i) + (lane >> 4);
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) zr[i][sb] = row < m_pad ? Zg[row * S + sb * 16 + (lane & 15)] : 0.f;
  }
  constexpr int NACC = CARRY ? 1 : APW;
  M::acc acc2[NACC][SB];
#pragma unroll
  for (int i = 0; i < NACC; ++i)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = M::zero();

  TileRegs<float, (MPK * TT / 4 + kZrThreads - 1) / kZrThreads, kZrThreads, TT> regs;
  if (t0 < t1) regs.fetch(A, m, n, 0, MPK, t0 * TT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(As, MPK);
    __syncthreads();
    if (t + 1 < t1) regs.fetch(A, m, n, 0, MPK, (t + 1) * TT, aligned);
    M::acc acc1[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc1[sb] = M::zero();
#pragma unroll
    for (int i = 0; i < KPW; ++i) {
      const float av = As[(4 * (wave + NWV * i) + (lane >> 4)) * AP + (lane & 15)];
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc1[sb] = M::mma(av, zr[i][sb], acc1[sb]);
    }
    // W = sum of the 8 wave partials in the order (((P0 + P4) + (P1 + P5)) + (P2 + P6)) + (P3 + P7)
    float* slot = Wp + wave * TT * S;
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int r = 0; r < 4; ++r) slot[M::orow(lane, r) * S + sb * 16 + (lane & 15)] = acc1[sb][r];
    __syncthreads();
    for (int e = threadIdx.x; e < TT * S; e += kZrThreads) {
      const float s0 = Wp[e] + Wp[4 * TT * S + e], s1 = Wp[TT * S + e] + Wp[5 * TT * S + e];
      const float s2 = Wp[2 * TT * S + e] + Wp[6 * TT * S + e], s3 = Wp[3 * TT * S + e] + Wp[7 * TT * S + e];
      Wp[8 * TT * S + e] = ((s0 + s1) + s2) + s3;
    }
    __syncthreads();
    const float* Ws = Wp + 8 * TT * S;
    if (CARRY) {
      const int64_t b0 = t * TT;
      for (int e = threadIdx.x; e < TT * s_out; e += kZrThreads) {
        const int c = e / TT, bb = e % TT;
        if (b0 + bb < n) part[(int64_t)c * ldo + b0 + bb] = Ws[bb * S + c];
      }
      continue;
    }
#pragma unroll
    for (int ks = 0; ks < TT / 4; ++ks) {
      const int col = ks * 4 + (lane >> 4);
      float b[SB];
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) b[sb] = Ws[col * S + sb * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < NACC; ++i) {
        const int ab = wave + NWV * i;
        if (ab * 16 < m_pad) {
          const float av = As[(ab * 16 + (lane & 15)) * AP + col];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) acc2[i][sb] = M::mma(av, b[sb], acc2[i][sb]);
        }
      }
    }
  }
  if (CARRY) return;
  float* out = part + g * (int64_t)m_pad * S;
#pragma unroll
  for (int i = 0; i < NACC; ++i) {
    const int ab = wave + NWV * i;
    if (ab * 16 < m_pad) {
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(int64_t)(ab * 16 + M::orow(lane, r)) * S + sb * 16 + (lane & 15)] = acc2[i][sb][r];
    }
  }
}

// ----------------------------------------------------------------------------------
// Short unfoldings (m_pad <= 64): every wave streams its own blocks of 16 * VEC columns
// (VEC = 16-byte vector length) with no LDS and no barriers.  Lane (j, q) loads the
// vector A[4 ks + q][c0 + VEC j .. c0 + VEC j + VEC - 1]; element e of that vector is
// column j of the e-th matrix-core product, so each block is VEC products whose output
// columns interleave back into whole 16-byte vectors.
//
// k_carry_small: C (s_out x n) = Z^T A with Z^T as the A operand held in registers
// (Z = G rounded to A's dtype, m_pad x S).
// ----------------------------------------------------------------------------------
// FULL = true: every block [b0, b1) is whole and A, out are 16-byte aligned with n and
// ldo multiples of VEC, so loads and stores are whole vectors with no column guards (its
// register footprint stays small enough for four waves per SIMD); FULL = false handles
// any block with guarded scalar accesses.
template <typename T, int SB, int KS, bool FULL>
__global__ __launch_bounds__(kThreads) void k_carry_small(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                          const T* __restrict__ Zg, T* __restrict__ out, int64_t ldo,
                                                          int s_out, int64_t b0, int64_t b1) {
  using M = Mma<T>;
  constexpr int VEC = 16 / sizeof(T), CB = 16 * VEC, S = SB * 16;
  const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
  T gr[KS][SB];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int row = 4 * ks + q;
      gr[ks][sb] = row < m_pad ? Zg[row * S + sb * 16 + j] : T(0);
    }
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t blk = b0 + (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); blk < b1; blk += nw) {
    const int64_t col = blk * CB + VEC * j;
    T av[KS][VEC];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int64_t row = 4 * ks + q;
      if (FULL) {
        // rows beyond m read row m - 1 and are zeroed after the load (no divergent load)
        const int64_t rc = row < m ? row : m - 1;
        u4_t v = *reinterpret_cast<const u4_t*>(A + rc * n + col);
        if (row >= m) v = u4_t{0u, 0u, 0u, 0u};
        *reinterpret_cast<u4_t*>(av[ks]) = v;
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) av[ks][e] = (row < m && col + e < n) ? A[row * n + col + e] : T(0);
      }
    }
    typename M::acc acc[VEC][SB];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc[e][sb] = M::zero();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc[e][sb] = M::mma(gr[ks][sb], av[ks][e], acc[e][sb]);
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = sb * 16 + M::orow(lane, r);
        if (c < s_out) {
          T v[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) v[e] = acc[e][sb][r];
          T* dst = out + (int64_t)c * ldo + col;
          if (FULL) {
            *reinterpret_cast<u4_t*>(dst) = *reinterpret_cast<u4_t*>(v);
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              if (col + e < n) dst[e] = v[e];
          }
        }
      }
  }
}

// k_gram_small: per-work-group partial A A^T (upper block pairs, float64).  Lane (i, q)
// holds row rb*16 + i of 4 consecutive vectors; element e of vector t is the
// k = q column of product (t, e), for the A and the A^T operand alike.  Blocks [b0, b1);
// FULL as for k_carry_small.  The group's waves are summed as (w0 + w2) + (w1 + w3).
template <typename T, int MB, bool FULL>
__global__ __launch_bounds__(kThreads) void k_gram_small(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                         double* __restrict__ part, int64_t b0, int64_t b1) {
  using M = Mma<T>;
  constexpr int VEC = 16 / sizeof(T), NT4 = 4, CB = 4 * VEC * NT4, NP = MB * (MB + 1) / 2;
  __shared__ double red[2][NP][64][4];
  const int lane = threadIdx.x & 63, i16 = lane & 15, q = lane >> 4, wave = threadIdx.x >> 6;
  double sum[NP][4];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum[p][r] = 0.0;
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t blk = b0 + (int64_t)blockIdx.x * kWaves + wave; blk < b1; blk += nw) {
    const int64_t c0 = blk * CB;
    T av[MB][NT4][VEC];
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
      for (int t = 0; t < NT4; ++t) {
        const int64_t row = rb * 16 + i16, col = c0 + (int64_t)t * 4 * VEC + VEC * q;
        if (FULL) {
          // rows beyond m read row m - 1 and are zeroed after the load (no divergent load)
          const int64_t rc = row < m ? row : m - 1;
          u4_t v = *reinterpret_cast<const u4_t*>(A + rc * n + col);
          if (row >= m) v = u4_t{0u, 0u, 0u, 0u};
          *reinterpret_cast<u4_t*>(av[rb][t]) = v;
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) av[rb][t][e] = (row < m && col + e < n) ? A[row * n + col + e] : T(0);
        }
      }
    int p = 0;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = a; b < MB; ++b, ++p) {
        typename M::acc c = M::zero();
#pragma unroll
        for (int t = 0; t < NT4; ++t)
#pragma unroll
          for (int e = 0; e < VEC; ++e) c = M::mma(av[a][t][e], av[b][t][e], c);
#pragma unroll
        for (int r = 0; r < 4; ++r) sum[p][r] += (double)c[r];
      }
  }
  if (wave >= 2) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave - 2][p][lane][r] = sum[p][r];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][p][lane][r] += sum[p][r];
  }
  __syncthreads();
  if (wave == 0) {
    double* outp = part + (int64_t)blockIdx.x * m_pad * m_pad;
    int pp = 0;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = a; b < MB; ++b, ++pp)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double v = red[0][pp][lane][r] + red[1][pp][lane][r];
          outp[(a * 16 + M::orow(lane, r)) * m_pad + b * 16 + i16] = v;
        }
  }
}

// ----------------------------------------------------------------------------------
// k_aw: partial[g] rows [rb*256, rb*256+256) += A_J W_J, W (n x S) streamed from HBM.
// Grid (column group g, row block rb).  With OM the W tile is the sketch's Omega_k,
// drawn inside the kernel (omega.h) into a double-buffered LDS tile while the previous
// tile is multiplied, so Omega never reaches HBM (one row block: m_pad <= 256).
// ----------------------------------------------------------------------------------
template <typename T, int SB, bool OM = false>
__global__ __launch_bounds__(kThreads) void k_aw(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                 const T* __restrict__ W, T* __restrict__ part,
                                                 int64_t tiles_per_group, int64_t ntiles, uint64_t seed, int kmode,
                                                 int s) {
  using M = Mma<T>;
  constexpr int TT = tile_cols_t<T>(), S = SB * 16, AP = TT + 1;
  constexpr int APW = kAwRows / (16 * kWaves);
  constexpr int WVEC = 16 / sizeof(T);
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Ws = As + kAwRows * AP;  // OM: two Omega tiles of TT x S
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

  // W tile rows [t TT, t TT + TT) are one contiguous TT x S block: its 16-byte vectors are
  // loaded into registers together with the next A tile and written to LDS after the barrier
  constexpr int WV = OM ? 1 : (TT * S / WVEC + kThreads - 1) / kThreads;
  u4_t wv[WV];
  auto wfetch = [&](int64_t t) {
    const int64_t wrow0 = t * TT;
#pragma unroll
    for (int i = 0; i < WV; ++i) {
      const int e = (int)threadIdx.x + i * kThreads;
      const int rr = e / (S / WVEC);
      u4_t val = u4_t{0u, 0u, 0u, 0u};
      if (e < TT * S / WVEC && wrow0 + rr < n) val = reinterpret_cast<const u4_t*>(W + wrow0 * S)[e];
      wv[i] = val;
    }
  };
  if constexpr (OM) {
    // columns at and beyond 8 ceil(s / 8) are never drawn: zero them in both buffers once
    const int cz = 8 * ((s + 7) / 8);
    for (int e = threadIdx.x; e < 2 * TT * S; e += kThreads)
      if (e % S >= cz) Ws[e] = T(0);
  }
  TileRegs<T, 2 * APW> regs;
  if (t0 < t1) {
    regs.fetch(A, m, n, row0, rows, t0 * TT, aligned);
    if constexpr (OM) omega_tile<T>(seed, kmode, t0 * TT, TT, n, s, Ws + (t0 & 1) * TT * S, S, 1, threadIdx.x, kThreads);
    else wfetch(t0);
  }
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.commit(As, rows);
    if constexpr (!OM) {
#pragma unroll
      for (int i = 0; i < WV; ++i) {
        const int e = (int)threadIdx.x + i * kThreads;
        if (e < TT * S / WVEC) reinterpret_cast<u4_t*>(Ws)[e] = wv[i];
      }
    }
    __syncthreads();
    if (t + 1 < t1) {
      regs.fetch(A, m, n, row0, rows, (t + 1) * TT, aligned);
      if constexpr (OM)
        omega_tile<T>(seed, kmode, (t + 1) * TT, TT, n, s, Ws + ((t + 1) & 1) * TT * S, S, 1, threadIdx.x, kThreads);
      else wfetch(t + 1);
    }
    phase2_accumulate<T, SB, APW>(As, OM ? Ws + (t & 1) * TT * S : Ws, rows, acc2);
  }
  store_rows<T, SB, APW>(acc2, part + g * (int64_t)m_pad * S, rows, row0);
}

// ----------------------------------------------------------------------------------
// k_atz: W_J = A_J^T Z for every tile; rows processed in chunks of kRowChunk with
// Z chunk and A chunk in LDS.  When Z spans several chunks, the next Z chunk is loaded
// into registers together with the next A block, so neither load waits at the barrier.
// Output mode 0: out[(beta) * ldo + c] (n x S, all S columns); mode 1: out[c * ldo + beta]
// for c < s_out (the S x n carry, transposed).
// ----------------------------------------------------------------------------------
// Rows [row0, row0 + rows) of the m_pad x S block Z (row-major, 16-byte aligned) in
// 16-byte vectors, staged through registers into a contiguous LDS copy.
template <typename T, int S, int RC>
struct ZChunkRegs {
  static constexpr int VEC = 16 / sizeof(T);
  static constexpr int NV = (RC * S / VEC + kThreads - 1) / kThreads;
  u4_t v[NV];
  __device__ void fetch(const T* __restrict__ Zg, int row0, int rows) {
    const u4_t* src = reinterpret_cast<const u4_t*>(Zg + (int64_t)row0 * S);
    const int nv = rows * S / VEC;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int idx = (int)threadIdx.x + i * kThreads;
      if (idx < nv) v[i] = src[idx];
    }
  }
  __device__ void commit(T* __restrict__ Zs, int rows) const {
    u4_t* dst = reinterpret_cast<u4_t*>(Zs);
    const int nv = rows * S / VEC;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int idx = (int)threadIdx.x + i * kThreads;
      if (idx < nv) dst[idx] = v[i];
    }
  }
};

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

  const bool zvec = nchunks > 1 && ptr_aligned16(Zg);
  if (nchunks == 1)
    for (int e = threadIdx.x; e < m_pad * S; e += kThreads) Zs[e] = Zg[e];
  TileRegs<T, MAXV> regs;
  ZChunkRegs<T, S, kRowChunk> zregs;
  if (t0 < t1) {
    regs.fetch(A, m, n, 0, m_pad < kRowChunk ? m_pad : kRowChunk, t0 * TT, aligned);
    if (zvec) zregs.fetch(Zg, 0, kRowChunk);
  }
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
      if (zvec) zregs.commit(Zs, rows);
      else if (nchunks > 1)
        for (int e = threadIdx.x; e < rows * S; e += kThreads) Zs[e] = Zg[(int64_t)row0 * S + e];
      __syncthreads();
      // prefetch the next (tile, chunk) block and its Z chunk
      if (c + 1 < nchunks) {
        const int nr0 = (c + 1) * kRowChunk;
        const int nrows = (m_pad - nr0) < kRowChunk ? (m_pad - nr0) : kRowChunk;
        regs.fetch(A, m, n, nr0, nrows, t * TT, aligned);
        if (zvec) zregs.fetch(Zg, nr0, nrows);
      } else if (t + 1 < t1) {
        regs.fetch(A, m, n, 0, m_pad < kRowChunk ? m_pad : kRowChunk, (t + 1) * TT, aligned);
        if (zvec) zregs.fetch(Zg, 0, kRowChunk);
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
// k_atz_wide: W_J = A_J^T Z over wide column tiles (TC = 128 float32 / 64 float64
// columns) and 64-row chunks, so one staged chunk of Z serves TC columns (a quarter of
// the Z traffic of 32-column tiles when m is tall).  Wave w owns the output blocks of
// tile columns [w TC/4, (w+1) TC/4) for all S columns, so no cross-wave sum is needed.
// With ZRES the whole of Z (m_pad x S) stays in LDS for the work-group's life.  The next
// chunk of A (and of Z) is loaded into registers while the current one is multiplied.
// Output mode 0: out[beta * ldo + c] (n x S); mode 1: out[c * ldo + beta] for c < s_out
// (the S x n carry), written through an LDS transpose in whole rows.
// ----------------------------------------------------------------------------------
template <typename T> __device__ __host__ constexpr int wide_cols_t() { return sizeof(T) == 8 ? 64 : 128; }
constexpr int kWideRows = 64;
// Elements of the A tile's LDS region, which also holds the transposed output tile (mode 1),
// rounded up to whole 16-byte vectors so that the Z region after it stays aligned.
__device__ __host__ constexpr int wide_tile_elems(int tc, int S) {
  return ((kWideRows * (tc + 1) > tc * (S + 1) ? kWideRows * (tc + 1) : tc * (S + 1)) + 7) / 8 * 8;
}

template <typename T, typename TO, int SB, int OUTMODE, bool ZRES>
__global__ __launch_bounds__(kThreads) void k_atz_wide(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                                       const T* __restrict__ Zg, TO* __restrict__ out, int64_t ldo,
                                                       int s_out, int64_t tiles_per_group, int64_t ntiles, int cps,
                                                       T* __restrict__ rpart) {
  using M = Mma<T>;
  constexpr int TC = wide_cols_t<T>(), CBW = TC / 16 / kWaves, RC = kWideRows;
  constexpr int S = SB * 16, AP = TC + 1, WP = S + 1;
  constexpr int MAXV = RC * TC * (int)sizeof(T) / 16 / kThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Zs = As + wide_tile_elems(TC, S);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(T)) % 16 == 0);
  const int nchunks = (m_pad + RC - 1) / RC;
  auto chunk_rows = [&](int c) { return (m_pad - c * RC) < RC ? (m_pad - c * RC) : RC; };
  // row split (gridDim.y > 1, short unfoldings): chunks [c0, c1) into partial y of rpart
  const int c0 = (int)blockIdx.y * cps, c1 = c0 + cps < nchunks ? c0 + cps : nchunks;
  const bool split = gridDim.y > 1;
  if constexpr (ZRES) {
    const u4_t* src = reinterpret_cast<const u4_t*>(Zg);
    u4_t* dst = reinterpret_cast<u4_t*>(Zs);
    for (int e = threadIdx.x; e < m_pad * S * (int)sizeof(T) / 16; e += kThreads) dst[e] = src[e];
  }
  TileRegs<T, MAXV, kThreads, TC> regs;
  ZChunkRegs<T, S, RC> zregs;
  if (t0 < t1 && c0 < c1) {
    regs.fetch(A, m, n, (int64_t)c0 * RC, chunk_rows(c0), t0 * TC, aligned);
    if constexpr (!ZRES) zregs.fetch(Zg, c0 * RC, chunk_rows(c0));
  }
  // with at most two output tiles per wave, even and odd k-steps go to separate
  // accumulators (summed at the end), so consecutive products never wait on each other
  constexpr int KH = CBW * SB <= 2 ? 2 : 1;
  for (int64_t t = t0; t < t1; ++t) {
    typename M::acc acc[CBW][SB], acch[KH > 1 ? CBW : 1][KH > 1 ? SB : 1];
#pragma unroll
    for (int i = 0; i < CBW; ++i)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc[i][sb] = M::zero();
#pragma unroll
    for (int i = 0; i < (KH > 1 ? CBW : 1); ++i)
#pragma unroll
      for (int sb = 0; sb < (KH > 1 ? SB : 1); ++sb) acch[i][sb] = M::zero();
    for (int c = c0; c < c1; ++c) {
      const int rows = chunk_rows(c);
      __syncthreads();
      regs.commit(As, rows);
      if constexpr (!ZRES) zregs.commit(Zs, rows);
      __syncthreads();
      if (c + 1 < c1) {
        regs.fetch(A, m, n, (int64_t)(c + 1) * RC, chunk_rows(c + 1), t * TC, aligned);
        if constexpr (!ZRES) zregs.fetch(Zg, (c + 1) * RC, chunk_rows(c + 1));
      } else if (t + 1 < t1) {
        regs.fetch(A, m, n, (int64_t)c0 * RC, chunk_rows(c0), (t + 1) * TC, aligned);
        if constexpr (!ZRES) zregs.fetch(Zg, c0 * RC, chunk_rows(c0));
      }
      const T* Zc = ZRES ? Zs + (int64_t)c * RC * S : Zs;
      // rows is a multiple of 16: an even number of k-steps
      for (int ks = 0; ks < rows / 4; ks += KH) {
#pragma unroll
        for (int h = 0; h < KH; ++h) {
          const int row = (ks + h) * 4 + (lane >> 4);
          T av[CBW], bv[SB];
#pragma unroll
          for (int i = 0; i < CBW; ++i) av[i] = As[row * AP + (wave * CBW + i) * 16 + (lane & 15)];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) bv[sb] = Zc[row * S + sb * 16 + (lane & 15)];
#pragma unroll
          for (int i = 0; i < CBW; ++i)
#pragma unroll
            for (int sb = 0; sb < SB; ++sb) {
              if (h == 0) acc[i][sb] = M::mma(av[i], bv[sb], acc[i][sb]);
              else acch[KH > 1 ? i : 0][KH > 1 ? sb : 0] = M::mma(av[i], bv[sb], acch[KH > 1 ? i : 0][KH > 1 ? sb : 0]);
            }
        }
      }
    }
    if constexpr (KH > 1) {
#pragma unroll
      for (int i = 0; i < CBW; ++i)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc[i][sb] += acch[KH > 1 ? i : 0][KH > 1 ? sb : 0];
    }
    const int64_t b0 = t * TC;
    if (split) {
      // partial y in the n x S layout, summed by k_atz_split_reduce
      T* rp = rpart + (int64_t)blockIdx.y * n * S;
#pragma unroll
      for (int i = 0; i < CBW; ++i)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t col = b0 + (wave * CBW + i) * 16 + M::orow(lane, r);
            if (col < n) rp[col * S + sb * 16 + (lane & 15)] = acc[i][sb][r];
          }
    } else if constexpr (OUTMODE == 0) {
#pragma unroll
      for (int i = 0; i < CBW; ++i)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t col = b0 + (wave * CBW + i) * 16 + M::orow(lane, r);
            if (col < n) out[col * ldo + sb * 16 + (lane & 15)] = (TO)acc[i][sb][r];
          }
    } else {
      // transpose through LDS (the A tile's space) so that each carry row is written whole
      __syncthreads();
      T* Ws = As;
#pragma unroll
      for (int i = 0; i < CBW; ++i)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Ws[((wave * CBW + i) * 16 + M::orow(lane, r)) * WP + sb * 16 + (lane & 15)] = acc[i][sb][r];
      __syncthreads();
      for (int e = threadIdx.x; e < s_out * TC; e += kThreads) {
        const int cc = e / TC, j = e - cc * TC;
        if (b0 + j < n) out[(int64_t)cc * ldo + b0 + j] = (TO)Ws[j * WP + cc];
      }
    }
  }
}

// Sum of the row-split partials of k_atz_wide (in split order): out[beta * ldo + c]
// (mode 0, c < S) or out[c * ldo + beta] (mode 1, c < s_out); beta runs fastest.
template <typename T, typename TO, int OUTMODE>
__global__ __launch_bounds__(256) void k_atz_split_reduce(const T* __restrict__ rpart, int nsplit, int64_t n, int S,
                                                          TO* __restrict__ out, int64_t ldo, int s_out) {
  const int cols = OUTMODE == 0 ? S : s_out;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)cols * n) return;
  const int c = (int)(e / n);
  const int64_t beta = e - (int64_t)c * n;
  double acc = 0.0;
  for (int y = 0; y < nsplit; ++y) acc += (double)rpart[((int64_t)y * n + beta) * S + c];
  if (OUTMODE == 0) out[beta * ldo + c] = (TO)acc;
  else out[(int64_t)c * ldo + beta] = (TO)acc;
}

// ----------------------------------------------------------------------------------
// k_gram: partial[g] (m_pad x m_pad, upper 16x16 blocks) = sum_J A_J A_J^T, m_pad <= 128
// on NT = 256 threads, m_pad <= 256 on NT = 1024 (16 waves share the 136 block pairs).
// float32 / bfloat16 products are summed per tile on the matrix cores in float32 and
// folded into float64 accumulators after every tile.
// ----------------------------------------------------------------------------------
// MT: type of the matrix-core products.  float32 input can take float64 products (MT =
// double): f32 x f32 is exact in float64 and the sums are float64, so the Gram is accurate
// to float64 rounding rather than float32's (its small eigen-directions need that).
// Row pitch padding of k_gram's tile: float32 input with float64 products on many pairs
// (the interleaved loop below) reads each operand pair as one 8-byte load, so its rows
// take an even pitch, TT + 4, whose 16 rows x 4 lanes of a read hit distinct banks.
template <typename T, int PPW, typename MT>
__host__ __device__ constexpr int gram_pad() {
  return (sizeof(T) == 4 && std::is_same<MT, double>::value && PPW >= 5) ? 4 : 1;
}

template <typename T, int PPW, int NT = kThreads, typename MT = T>
__global__ __launch_bounds__(NT) void k_gram(const T* __restrict__ A, int64_t m, int64_t n, int m_pad,
                                             double* __restrict__ part, int64_t tiles_per_group, int64_t ntiles) {
  using M = Mma<MT>;
  constexpr int TT = tile_cols_t<T>(), AP = TT + gram_pad<T, PPW, MT>();
  constexpr int NW = NT / 64;
  constexpr int MAXM = NT == kThreads ? kGramMaxM : kGramBigM;
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t t0 = g * tiles_per_group;
  const int64_t t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  const bool aligned = ptr_aligned16(A) && ((n * (int64_t)sizeof(T)) % 16 == 0);
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
  // the wave's block pairs, decoded once: LDS offsets of their two row blocks (uniform)
  constexpr bool F64ACC = std::is_same<MT, double>::value && PPW >= 5;  // (few pairs: per-pair chains)
  int pba[F64ACC ? PPW : 1], pbb[F64ACC ? PPW : 1];
  bool pval[F64ACC ? PPW : 1];
#pragma unroll
  for (int i = 0; i < (F64ACC ? PPW : 1); ++i) {
    int pa = 0, pb = 0;
    pval[i] = pair_of(i, &pa, &pb);
    pba[i] = pa * 16 * AP;
    pbb[i] = pb * 16 * AP;
  }
  const int lofs = (lane & 15) * AP + (lane >> 4);
  // float64 products accumulate on the matrix cores across all tiles; float32 products are
  // summed per tile and folded into float64
  typename M::acc cacc[F64ACC ? PPW : 1];
  double acc[F64ACC ? 1 : PPW][4];
#pragma unroll
  for (int i = 0; i < (F64ACC ? PPW : 1); ++i) cacc[i] = M::zero();
#pragma unroll
  for (int i = 0; i < (F64ACC ? 1 : PPW); ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[i][r] = 0.0;

  TileRegs<T, MAXM * TileRegs<T, 1>::VPR / NT, NT> regs;  // m_pad <= MAXM rows per tile
  if (t0 < t1) regs.fetch(A, m, n, 0, m_pad, t0 * TT, aligned);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    regs.template commit<AP - TT>(As, m_pad);
    __syncthreads();
    if (t + 1 < t1) regs.fetch(A, m, n, 0, m_pad, (t + 1) * TT, aligned);
    if constexpr (F64ACC && sizeof(T) == 4) {
      // float32 input: lane q = l / 16 takes columns 8 j + 2 q and 8 j + 2 q + 1 of the tile
      // (one 8-byte load per operand) for k-steps 2 j and 2 j + 1 (the sum over a tile's
      // columns does not depend on which k-step takes which column)
      const int lofs2 = (lane & 15) * AP + 2 * (lane >> 4);
#pragma unroll
      for (int j = 0; j < TT / 8; ++j)
#pragma unroll
        for (int i = 0; i < PPW; ++i)
          if (pval[i]) {
            const float2 av = *reinterpret_cast<const float2*>(As + pba[i] + lofs2 + 8 * j);
            const float2 bv = *reinterpret_cast<const float2*>(As + pbb[i] + lofs2 + 8 * j);
            cacc[i] = M::mma((MT)av.x, (MT)bv.x, cacc[i]);
            cacc[i] = M::mma((MT)av.y, (MT)bv.y, cacc[i]);
          }
    } else if constexpr (F64ACC) {
      // k-steps outside, pairs inside: consecutive products go to different accumulators
#pragma unroll
      for (int ks = 0; ks < TT / 4; ++ks)
#pragma unroll
        for (int i = 0; i < PPW; ++i)
          if (pval[F64ACC ? i : 0]) {
            const MT a = (MT)As[pba[F64ACC ? i : 0] + lofs + ks * 4];
            const MT b = (MT)As[pbb[F64ACC ? i : 0] + lofs + ks * 4];
            cacc[F64ACC ? i : 0] = M::mma(a, b, cacc[F64ACC ? i : 0]);
          }
    } else {
#pragma unroll
      for (int i = 0; i < PPW; ++i) {
        int pa, pb;
        if (pair_of(i, &pa, &pb)) {
          typename M::acc c = M::zero();
#pragma unroll
          for (int ks = 0; ks < TT / 4; ++ks) {
            const MT a = (MT)As[(pa * 16 + (lane & 15)) * AP + ks * 4 + (lane >> 4)];
            const MT b = (MT)As[(pb * 16 + (lane & 15)) * AP + ks * 4 + (lane >> 4)];
            c = M::mma(a, b, c);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][r] += (double)c[r];
        }
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
        out[(pa * 16 + M::orow(lane, r)) * m_pad + pb * 16 + (lane & 15)] =
            F64ACC ? (double)cacc[F64ACC ? i : 0][r] : acc[F64ACC ? 0 : i][r];
  }
}

// ----------------------------------------------------------------------------------
// Omega_k materialised (n x ldo, zero padded); the entries come from omega.h.
// ----------------------------------------------------------------------------------
template <typename TO>
__global__ __launch_bounds__(256) void k_omega(uint64_t seed, int k, int64_t beta0, int64_t nrows, int s, int ldo,
                                               TO* __restrict__ out) {
  const int G8 = (ldo + 7) / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrows * G8) return;
  const int64_t rr = idx / G8;
  const int g = (int)(idx % G8);
  float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (8 * g < s) omega8(seed, k, beta0 + rr, g, z);  // groups wholly in the zero padding draw nothing
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = 8 * g + j;
    if (c < ldo) out[rr * ldo + c] = round_from_f64<TO>(c < s ? (double)z[j] : 0.0);
  }
}

// Omega_k rows [0, nrows) transposed, float32: out[c ldt + beta] for c < S (zero for c >= s).
// Consecutive threads take consecutive rows beta, so each of the eight stores of a group is
// coalesced.
__global__ __launch_bounds__(256) void k_omega_t(uint64_t seed, int k, int64_t nrows, int s, int S, int64_t ldt,
                                                 float* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int G8 = (S + 7) / 8;
  if (idx >= nrows * G8) return;
  const int g = (int)(idx / nrows);
  const int64_t beta = idx - (int64_t)g * nrows;
  float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (8 * g < s) omega8(seed, k, beta, g, z);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = 8 * g + j;
    if (c < S) out[(int64_t)c * ldt + beta] = c < s ? z[j] : 0.0f;
  }
}

hipError_t launch_omega_t(uint64_t seed, int k, int64_t nrows, int s, int S, int64_t ldt, float* out, hipStream_t st) {
  if (S % 8 != 0 || ldt < nrows) return hipErrorInvalidValue;
  const int64_t total = nrows * (S / 8);
  hipLaunchKernelGGL(k_omega_t, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, seed, k, nrows, s, S, ldt, out);
  return hipGetLastError();
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

// Reductions of the per-group partials.  A work-group takes kRedOuts outputs; its
// kRedSeg thread slices each sum a contiguous range of the groups, and the slices are
// added in slice order, so every output has one fixed summation order.
constexpr int kRedSeg = 8;
constexpr int kRedOuts = 256 / kRedSeg;

template <typename P>
__device__ inline double seg_partial(const P* __restrict__ p, int64_t groups, int64_t stride, int seg) {
  const int64_t per = (groups + kRedSeg - 1) / kRedSeg;
  const int64_t g0 = seg * per, g1 = g0 + per < groups ? g0 + per : groups;
  return g0 < g1 ? strided_sum(p + g0 * stride, g1 - g0, stride) : 0.0;
}

__device__ inline double seg_combine(double v, double (&red)[kRedSeg][kRedOuts], int seg, int o) {
  red[seg][o] = v;
  __syncthreads();
  double t = red[0][o];
#pragma unroll
  for (int k = 1; k < kRedSeg; ++k) t += red[k][o];
  return t;
}

template <typename P>
__global__ __launch_bounds__(256) void k_reduce(const P* __restrict__ part, int64_t groups, int64_t stride, int m,
                                                int S, int s, double* __restrict__ y, int ldy) {
  __shared__ double red[kRedSeg][kRedOuts];
  const int o = threadIdx.x % kRedOuts, seg = threadIdx.x / kRedOuts;
  const int64_t idx = (int64_t)blockIdx.x * kRedOuts + o;
  const bool ok = idx < (int64_t)m * s;
  const int i = ok ? (int)(idx / s) : 0, c = ok ? (int)(idx % s) : 0;
  const double v = ok ? seg_partial(part + (int64_t)i * S + c, groups, stride, seg) : 0.0;
  const double t = seg_combine(v, red, seg, o);
  if (ok && seg == 0) y[(int64_t)i * ldy + c] = t;
}

__global__ __launch_bounds__(256) void k_reduce_gram(const double* __restrict__ part, int64_t groups, int m_pad,
                                                     int m, double* __restrict__ out) {
  __shared__ double red[kRedSeg][kRedOuts];
  const int o = threadIdx.x % kRedOuts, seg = threadIdx.x / kRedOuts;
  const int64_t idx = (int64_t)blockIdx.x * kRedOuts + o;
  const bool ok = idx < (int64_t)m * m;
  int i = ok ? (int)(idx / m) : 0, j = ok ? (int)(idx % m) : 0;
  if (i / 16 > j / 16) { const int t = i; i = j; j = t; }
  const double v = ok ? seg_partial(part + (int64_t)i * m_pad + j, groups, (int64_t)m_pad * m_pad, seg) : 0.0;
  const double t = seg_combine(v, red, seg, o);
  if (ok && seg == 0) out[idx] = t;
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

// Work-groups of `kernel` (threads, dynamic LDS) resident on the whole device at once.
template <typename F>
static int64_t resident_groups(F kernel, int threads, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), threads, lds) !=
          hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return (int64_t)cus * per_cu;
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
  if (!part_fits(a, Gu, a.m_pad * SB * 16, sizeof(T))) return hipErrorInvalidValue;
  TTR_HIP(mark_event(a.ev_begin, a.stream));
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m, a.n,
                       (int)a.m_pad, (const T*)a.Z, (T*)a.part, tpg, ntiles);
    TTR_HIP(hipGetLastError());
  }
  TTR_HIP(mark_event(a.ev_end, a.stream));
  const int64_t total = a.m * a.s;
  hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, a.stream, (const T*)a.part,
                     Gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y, a.ldy);
  return hipGetLastError();
}

template <typename T, int SB, bool OM = false>
static hipError_t launch_aw_t(const StreamArgs& a) {
  constexpr int TT = tile_cols_t<T>();
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t rb = (a.m_pad + kAwRows - 1) / kAwRows;
  if (OM && rb != 1) return hipErrorInvalidValue;
  // OM: a second W tile (the Omega tiles are double-buffered)
  const size_t lds = aw_lds_bytes(SB * 16, sizeof(T) == 8 ? TTR_F64 : TTR_F32) + (OM ? (size_t)TT * SB * 16 * sizeof(T) : 0);
  auto kern = k_aw<T, SB, OM>;
  TTR_HIP(set_lds(kern, lds));
  // column groups: at most one round of resident work-groups over all row blocks, so no
  // partial second round idles most of the device
  int64_t cap = std::max<int64_t>(1, kMaxGroups / rb);
  const int64_t slots = resident_groups(kern, kThreads, lds);
  if (slots >= rb) cap = std::min(cap, slots / rb);
  const int64_t G = groups_for(ntiles, cap);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  if (!part_fits(a, Gu, a.m_pad * SB * 16, sizeof(T))) return hipErrorInvalidValue;
  TTR_HIP(mark_event(a.ev_begin, a.stream));
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)Gu, (unsigned)rb), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m,
                       a.n, (int)a.m_pad, (const T*)a.W, (T*)a.part, tpg, ntiles, a.seed, a.kmode, a.s);
    TTR_HIP(hipGetLastError());
  }
  TTR_HIP(mark_event(a.ev_end, a.stream));
  const int64_t total = a.m * a.s;
  hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, a.stream, (const T*)a.part,
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

template <typename T, int PPW, int NT = kThreads, typename MT = T>
static hipError_t launch_gram_t(const StreamArgs& a, double* gm) {
  constexpr int TT = tile_cols_t<T>();
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t G = groups_for(ntiles, kGramGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = (size_t)a.m_pad * (TT + gram_pad<T, PPW, MT>()) * sizeof(T);
  auto kern = k_gram<T, PPW, NT, MT>;
  TTR_HIP(set_lds(kern, lds));
  if (!part_fits(a, Gu, a.m_pad * a.m_pad, sizeof(double))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(NT), lds, a.stream, (const T*)a.A, a.m, a.n,
                     (int)a.m_pad, (double*)a.part, tpg, ntiles);
  TTR_HIP(hipGetLastError());
  const int64_t total = a.m * a.m;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, a.stream,
                     (const double*)a.part, Gu, (int)a.m_pad, (int)a.m, gm);
  return hipGetLastError();
}

// Dispatch on (dtype, S/16, rows per wave): whole aligned blocks through the FULL kernel,
// the ragged last block (or everything, when unaligned) through the guarded one.
template <typename T, int SB, int KS>
static hipError_t launch_carry_small_t(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  constexpr int VEC = 16 / (int)sizeof(T), CB = 16 * VEC;
  const int64_t nblocks = (a.n + CB - 1) / CB;
  const bool vec_ok = (reinterpret_cast<uintptr_t>(a.A) & 15) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0 &&
                      a.n % VEC == 0 && ldo % VEC == 0;
  const int64_t nfull = vec_ok ? a.n / CB : 0;
  if (nfull > 0) {
    const int64_t groups = std::max<int64_t>(1, std::min<int64_t>((nfull + kWaves - 1) / kWaves, kSmallGroups));
    hipLaunchKernelGGL((k_carry_small<T, SB, KS, true>), dim3((unsigned)groups), dim3(kThreads), 0, a.stream,
                       (const T*)a.A, a.m, a.n, (int)a.m_pad, (const T*)a.Z, (T*)out, ldo, s_out, (int64_t)0, nfull);
    TTR_HIP(hipGetLastError());
  }
  if (nfull < nblocks) {
    const int64_t rest = nblocks - nfull;
    const int64_t groups = std::max<int64_t>(1, std::min<int64_t>((rest + kWaves - 1) / kWaves, kSmallGroups));
    hipLaunchKernelGGL((k_carry_small<T, SB, KS, false>), dim3((unsigned)groups), dim3(kThreads), 0, a.stream,
                       (const T*)a.A, a.m, a.n, (int)a.m_pad, (const T*)a.Z, (T*)out, ldo, s_out, nfull, nblocks);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t carry_small_dispatch(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  const int SB = a.S / 16, KS = (int)(a.m_pad / 4);
#define TTR_C(SBv, KSv) \
  if (SB == SBv && KS == KSv) return launch_carry_small_t<T, SBv, KSv>(a, out, ldo, s_out);
#define TTR_CA(SBv) TTR_C(SBv, 4) TTR_C(SBv, 8) TTR_C(SBv, 12) TTR_C(SBv, 16)
  TTR_CA(1) TTR_CA(2) TTR_CA(3) TTR_CA(4)
#undef TTR_CA
#undef TTR_C
  return hipErrorInvalidValue;
}

// Whole aligned blocks through the FULL kernel; the ragged last block (or all blocks,
// when unaligned) in a second launch that writes its own partial after the first's.
template <typename T, int MB>
static hipError_t launch_gram_small_t(const StreamArgs& a, double* gm) {
  constexpr int VEC = 16 / (int)sizeof(T), CB = 4 * VEC * 4;
  const int64_t nblocks = (a.n + CB - 1) / CB;
  const bool vec_ok = (reinterpret_cast<uintptr_t>(a.A) & 15) == 0 && a.n % VEC == 0;
  const int64_t nfull = vec_ok ? a.n / CB : 0;
  const int64_t g1 = nfull > 0 ? std::max<int64_t>(1, std::min<int64_t>((nfull + kWaves - 1) / kWaves,
                                                                          kGramSmallGroups - 1)) : 0;
  const int64_t rest = nblocks - nfull;
  const int64_t g2 = rest > 0 ? std::max<int64_t>(1, std::min<int64_t>((rest + kWaves - 1) / kWaves,
                                                                       kGramSmallGroups - g1)) : 0;
  if (!part_fits(a, g1 + g2, a.m_pad * a.m_pad, sizeof(double))) return hipErrorInvalidValue;
  if (g1 > 0) {
    hipLaunchKernelGGL((k_gram_small<T, MB, true>), dim3((unsigned)g1), dim3(kThreads), 0, a.stream, (const T*)a.A,
                       a.m, a.n, (int)a.m_pad, (double*)a.part, (int64_t)0, nfull);
    TTR_HIP(hipGetLastError());
  }
  if (g2 > 0) {
    double* p2 = (double*)a.part + g1 * a.m_pad * a.m_pad;
    hipLaunchKernelGGL((k_gram_small<T, MB, false>), dim3((unsigned)g2), dim3(kThreads), 0, a.stream, (const T*)a.A,
                       a.m, a.n, (int)a.m_pad, p2, nfull, nblocks);
    TTR_HIP(hipGetLastError());
  }
  const int64_t total = a.m * a.m;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, a.stream,
                     (const double*)a.part, g1 + g2, (int)a.m_pad, (int)a.m, gm);
  return hipGetLastError();
}

template <int SB, int KPW>
static hipError_t launch_carry_zr_t(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  constexpr int TT = kZrTileCols;
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t G = groups_for(ntiles, kFusedZrGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = fused_zr_lds_bytes(KPW * 4 * kZrWaves, SB * 16);
  auto kern = k_fused_zr<SB, KPW, 1>;
  TTR_HIP(set_lds(kern, lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(kZrThreads), lds, a.stream, (const float*)a.A, a.m, a.n,
                     (int)a.m_pad, (const float*)a.Z, (float*)out, tpg, ntiles, ldo, s_out);
  return hipGetLastError();
}

static hipError_t carry_zr_dispatch(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  const int SB = a.S / 16;
  const int64_t mpk = fused_zr_rows(a.m_pad);
#define TTR_Z(SBv, MPKv) \
  if (SB == SBv && mpk == MPKv) return launch_carry_zr_t<SBv, MPKv / 32>(a, out, ldo, s_out);
#define TTR_ZA(SBv) TTR_Z(SBv, 576) TTR_Z(SBv, 640) TTR_Z(SBv, 704) TTR_Z(SBv, 768) TTR_Z(SBv, 832) \
  TTR_Z(SBv, 896)
  TTR_ZA(1) TTR_ZA(2) TTR_Z(2, 960) TTR_Z(2, 1024)
#undef TTR_ZA
#undef TTR_Z
  return hipErrorInvalidValue;
}

template <int SB, int KPW>
static hipError_t launch_fused_zr_t(const StreamArgs& a) {
  constexpr int TT = kZrTileCols;
  const int64_t ntiles = (a.n + TT - 1) / TT;
  const int64_t G = groups_for(ntiles, kFusedZrGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t lds = fused_zr_lds_bytes(KPW * 4 * kZrWaves, SB * 16);
  auto kern = k_fused_zr<SB, KPW, 0>;
  TTR_HIP(set_lds(kern, lds));
  if (!part_fits(a, Gu, a.m_pad * SB * 16, sizeof(float))) return hipErrorInvalidValue;
  TTR_HIP(mark_event(a.ev_begin, a.stream));
  for (int rep = 0; rep < a.reps; ++rep) {
    hipLaunchKernelGGL(kern, dim3((unsigned)Gu), dim3(kZrThreads), lds, a.stream, (const float*)a.A, a.m, a.n,
                       (int)a.m_pad, (const float*)a.Z, (float*)a.part, tpg, ntiles, (int64_t)0, 0);
    TTR_HIP(hipGetLastError());
  }
  TTR_HIP(mark_event(a.ev_end, a.stream));
  const int64_t total = a.m * a.s;
  hipLaunchKernelGGL(k_reduce<float>, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, a.stream,
                     (const float*)a.part, Gu, a.m_pad * (int64_t)(SB * 16), (int)a.m, SB * 16, a.s, a.y, a.ldy);
  return hipGetLastError();
}

static hipError_t fused_zr_dispatch(const StreamArgs& a) {
  const int SB = a.S / 16;
  const int64_t mpk = fused_zr_rows(a.m_pad);
#define TTR_Z(SBv, MPKv) \
  if (SB == SBv && mpk == MPKv) return launch_fused_zr_t<SBv, MPKv / 32>(a);
#define TTR_ZA(SBv) TTR_Z(SBv, 576) TTR_Z(SBv, 640) TTR_Z(SBv, 704) TTR_Z(SBv, 768) TTR_Z(SBv, 832) \
  TTR_Z(SBv, 896)
  TTR_ZA(1) TTR_ZA(2) TTR_Z(2, 960) TTR_Z(2, 1024)
#undef TTR_ZA
#undef TTR_Z
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t fused_dispatch(const StreamArgs& a) {
  if (sizeof(T) == 4 && a.m_pad > kFusedMaxRows) return fused_zr_dispatch(a);
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

template <typename T, bool OM = false>
static hipError_t aw_dispatch(const StreamArgs& a) {
  switch (a.S / 16) {
    case 1: return launch_aw_t<T, 1, OM>(a);
    case 2: return launch_aw_t<T, 2, OM>(a);
    case 3: return launch_aw_t<T, 3, OM>(a);
    case 4: return launch_aw_t<T, 4, OM>(a);
  }
  return hipErrorInvalidValue;
}

// Z resident in LDS for the whole launch when it takes at most this many bytes.
constexpr size_t kWideZResBytes = 64 * 1024;

template <typename T, typename TO, int SB, int OUTMODE>
static hipError_t launch_atz_wide_t(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  constexpr int TC = wide_cols_t<T>();
  const int64_t ntiles = (a.n + TC - 1) / TC;
  const int64_t G = groups_for(ntiles, kMaxGroups);
  const int64_t tpg = (ntiles + G - 1) / G;
  const int64_t Gu = (ntiles + tpg - 1) / tpg;
  const size_t zbytes = (size_t)a.m_pad * SB * 16 * sizeof(T);
  const bool zres = zbytes <= kWideZResBytes;
  const size_t lds = (size_t)wide_tile_elems(TC, SB * 16) * sizeof(T) + (zres ? zbytes : (size_t)kWideRows * SB * 16 * sizeof(T));
  auto kern = zres ? k_atz_wide<T, TO, SB, OUTMODE, true> : k_atz_wide<T, TO, SB, OUTMODE, false>;
  TTR_HIP(set_lds(kern, lds));
  // Few column tiles (a short, tall unfolding): split the rows over the grid's second
  // dimension, at least two 64-row chunks per split, into partials in a.part
  const int nchunks = (int)((a.m_pad + kWideRows - 1) / kWideRows);
  int nsplit = 1;
  if (Gu < 128 && nchunks >= 4) {
    nsplit = (int)std::min<int64_t>(nchunks / 2, (256 + Gu - 1) / Gu);
    const size_t per = (size_t)a.n * SB * 16 * sizeof(T);
    if (a.part) nsplit = (int)std::min<size_t>((size_t)nsplit, a.part_bytes / per);
    else nsplit = 1;
    if (nsplit < 2) nsplit = 1;
  }
  const int cps = (nchunks + nsplit - 1) / nsplit;
  nsplit = (nchunks + cps - 1) / cps;
  hipLaunchKernelGGL(kern, dim3((unsigned)Gu, (unsigned)nsplit), dim3(kThreads), lds, a.stream, (const T*)a.A, a.m,
                     a.n, (int)a.m_pad, (const T*)a.Z, (TO*)out, ldo, s_out, tpg, ntiles, cps, (T*)a.part);
  TTR_HIP(hipGetLastError());
  if (nsplit == 1) return hipSuccess;
  const int64_t total = (int64_t)(OUTMODE == 0 ? SB * 16 : s_out) * a.n;
  hipLaunchKernelGGL((k_atz_split_reduce<T, TO, OUTMODE>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     a.stream, (const T*)a.part, nsplit, a.n, SB * 16, (TO*)out, ldo, s_out);
  return hipGetLastError();
}

template <typename T, typename TO, int OUTMODE>
static hipError_t atz_dispatch(const StreamArgs& a, void* out, int64_t ldo, int s_out) {
  switch (a.S / 16) {
    case 1: return launch_atz_wide_t<T, TO, 1, OUTMODE>(a, out, ldo, s_out);
    case 2: return launch_atz_wide_t<T, TO, 2, OUTMODE>(a, out, ldo, s_out);
    case 3: return launch_atz_wide_t<T, TO, 3, OUTMODE>(a, out, ldo, s_out);
    case 4: return launch_atz_wide_t<T, TO, 4, OUTMODE>(a, out, ldo, s_out);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t gram_dispatch(const StreamArgs& a, double* gm) {
  const int MB = (int)(a.m_pad / 16);
  if (a.gram_f64 && sizeof(T) == 4) {  // float32 input, float64 products (any m_pad <= 256)
    if (MB > kGramBigM / 16) return hipErrorInvalidValue;
    if (MB > kGramMaxM / 16) return launch_gram_t<T, 9, kGramBigThreads, double>(a, gm);
    const int ppw = (MB * (MB + 1) / 2 + kWaves - 1) / kWaves;
    if (ppw <= 3) return launch_gram_t<T, 3, kThreads, double>(a, gm);
    return launch_gram_t<T, 9, kThreads, double>(a, gm);
  }
  if (MB == 1) return launch_gram_small_t<T, 1>(a, gm);
  if (MB == 2) return launch_gram_small_t<T, 2>(a, gm);
  if (MB == 3) return launch_gram_small_t<T, 3>(a, gm);
  if (MB == 4) return launch_gram_small_t<T, 4>(a, gm);
  if (MB > kGramMaxM / 16) {  // 128 < m_pad <= 256: 16 waves, at most 9 block pairs each
    if (MB > kGramBigM / 16) return hipErrorInvalidValue;
    return launch_gram_t<T, 9, kGramBigThreads>(a, gm);
  }
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
  hipLaunchKernelGGL(k_reduce<float>, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, st, part, groups, stride,
                     m, S, s, y, ldy);
  return hipGetLastError();
}

hipError_t launch_reduce_gram(const double* part, int64_t groups, int m_pad, int m, double* out, hipStream_t st) {
  const int64_t total = (int64_t)m * m;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)), dim3(256), 0, st, part, groups, m_pad, m,
                     out);
  return hipGetLastError();
}

hipError_t launch_fused(const StreamArgs& a) {
  if (a.dtype == TTR_F64) return fused_dispatch<double>(a);
  if (a.dtype == TTR_F32) return fused_dispatch<float>(a);
  return launch_fused_bf16(a);
}

hipError_t launch_aw(const StreamArgs& a) {
  if (a.dtype == TTR_F32 && a.split_f32) return launch_aw_split(a);
  if (a.dtype == TTR_F64) return aw_dispatch<double>(a);
  if (a.dtype == TTR_F32) return aw_dispatch<float>(a);
  return launch_aw_bf16(a);
}

hipError_t launch_atz(const StreamArgs& a, void* out, int out_dtype, int64_t ldo, int s_out, int outmode) {
  if (a.dtype == TTR_F32 && a.split_f32 && out_dtype == TTR_F32) return launch_atz_split(a, out, ldo, s_out, outmode);
  if (outmode == 1 && out_dtype == a.dtype && a.dtype != TTR_BF16 && carry_small_fits(a.m_pad, a.S)) {
    if (a.dtype == TTR_F64) return carry_small_dispatch<double>(a, out, ldo, s_out);
    return carry_small_dispatch<float>(a, out, ldo, s_out);
  }
  if (outmode == 1 && out_dtype == TTR_F32 && fused_zr_fits(a.m_pad, a.S, a.dtype))
    return carry_zr_dispatch(a, out, ldo, s_out);
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

hipError_t launch_aw_omega(const StreamArgs& a) {
  if (a.dtype == TTR_F64) return aw_dispatch<double, true>(a);
  if (a.dtype == TTR_F32) return aw_dispatch<float, true>(a);
  return launch_aw_omega_bf16(a);
}

hipError_t launch_gram_sketch(const StreamArgs& a, double* gm) {
  if (a.dtype == TTR_BF16) return launch_gram_sketch_bf16(a, gm);
  // float32 / float64: the Gram pass is bound by the matrix cores (float64 products), where
  // a fused sketch would only add to the bound; the sketch streams A again with Omega drawn
  // in the kernel (only the timing events' first launch is the Gram's)
  StreamArgs g = a;
  g.gram_f64 = a.dtype == TTR_F32;
  g.ev_begin = g.ev_end = nullptr;
  g.reps = 1;
  TTR_HIP(launch_gram(g, gm));
  StreamArgs sk = a;
  sk.ev_begin = sk.ev_end = nullptr;
  sk.reps = 1;
  return launch_aw_omega(sk);
}

hipError_t launch_omega(uint64_t seed, int k, int64_t beta0, int64_t nrows, int s, int ldo, void* out, int out_dtype,
                        hipStream_t st) {
  const int64_t total = nrows * ((ldo + 7) / 8);
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
