// Entries of the Gaussian test matrices Omega_k (Algorithm 3, step 3) on the device:
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011) keyed by (seed, k) with counter
// (beta, g, 0, 0), and the Box-Muller transform in float64.  Entry (beta, c) of Omega_k
// is element c % 4 of group g = c / 4: words 0, 1 give entries 4g, 4g + 1 (cos, sin) and
// words 2, 3 entries 4g + 2, 4g + 3.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "convert.h"

namespace ttr {

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

// u in (0, 1): the top 52 bits of a word, offset by half a step (exact in float64).
__device__ inline double unit_open(uint64_t x) { return ((double)(x >> 12) + 0.5) * 0x1p-52; }

// Four normals of group g (entries c = 4g .. 4g+3) of row beta of Omega_k.
__device__ __attribute__((always_inline)) inline void omega4(uint64_t seed, int k, int64_t beta, int g,
                                                             double (&z)[4]) {
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

}  // namespace ttr

namespace ttr {

// Rows [beta0, beta0 + rows) of Omega_k (zero beyond row n), entries c < 4 ceil(s / 4)
// (zero for c >= s), rounded once to T and written into LDS by `nthr` threads (tid =
// 0 .. nthr-1 among them): entry (b, c) goes to Om[b * rs + c * cs] (rs = pitch, cs = 1
// for a row-major tile; rs = 1, cs = pitch for a transposed one).
template <typename T>
__device__ __attribute__((always_inline)) inline void omega_tile(uint64_t seed, int k, int64_t beta0, int rows,
                                                                 int64_t n, int s, T* __restrict__ Om, int rs, int cs,
                                                                 int tid, int nthr) {
  const int g4 = (s + 3) / 4;
  for (int id = tid; id < rows * g4; id += nthr) {
    const int b = id / g4, g = id - b * g4;
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (beta0 + b < n) omega4(seed, k, beta0 + b, g, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * g + j;
      Om[b * rs + c * cs] = round_from_f64<T>(c < s ? z[j] : 0.0);
    }
  }
}

}  // namespace ttr
