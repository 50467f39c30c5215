// Entries of the Gaussian test matrices Omega_k (Algorithm 3, step 3) on the device:
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011) keyed by (seed, k) with counter
// (beta, g, 0, 0) feeds the eight entries c = 8g .. 8g+7 of row beta: word j = (c % 8) / 2
// splits into two 23-bit uniforms u (low half) and v (high half), and the Box-Muller
// transform sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v) gives entries 8g + 2j and 8g + 2j + 1.
// The transform is evaluated in float32 by a fixed sequence of correctly rounded
// operations (no fused multiply-add; the one division and the square root are taken in
// float64 and rounded to float32, which equals the correctly rounded float32 result), so
// that any implementation following the same sequence draws the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "convert.h"

namespace ttr {

// The 128-bit product of a 64-bit word and a 64-bit constant from four 32 x 32 -> 64
// products, each partial sum kept below 2^64: lo = (p2 mod 2^32) 2^32 + (p0 mod 2^32), hi = p3.
__device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  const uint64_t aL = (uint32_t)a, aH = a >> 32, bL = (uint32_t)b, bH = b >> 32;
  const uint64_t p0 = aL * bL;
  const uint64_t p1 = aH * bL + (p0 >> 32);
  const uint64_t p2 = aL * bH + (uint32_t)p1;
  *hi = aH * bH + ((p1 >> 32) + (p2 >> 32));
  *lo = (p2 << 32) | (uint32_t)p0;
}

__device__ inline void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(x[0], M0, &hi0, &lo0);
    mulhilo64(x[2], M1, &hi1, &lo1);
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = lo1; x[2] = y2; x[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// ((w >> 9) + 1/2) 2^-23 of the 32-bit word w: an exact float32 in (0, 1).
__device__ inline float uniform23(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }

// ln u for u in (0, 1): u = 2^e f, f in [sqrt 1/2, sqrt 2], atanh series of ln f to t^11.
__device__ __attribute__((always_inline)) inline float ln32(float u) {
#pragma clang fp contract(off)
  const uint32_t bits = __float_as_uint(u);
  int e = (int)(bits >> 23) - 127;
  float f = __uint_as_float((bits & 0x7FFFFFu) | 0x3F800000u);
  if (f > 0x1.6a09e6p+0f) {
    f = f * 0.5f;
    e += 1;
  }
  const float t = (float)((double)(f - 1.0f) / (double)(f + 1.0f));
  const float w = t * t;
  float p = 0x1.745d18p-4f * w + 0x1.c71c72p-4f;
  p = p * w + 0x1.24924ap-3f;
  p = p * w + 0x1.99999ap-3f;
  p = p * w + 0x1.555556p-2f;
  p = p * w + 1.0f;
  return (float)e * 0x1.62e430p-1f + (t + t) * p;
}

// (cos 2 pi v, sin 2 pi v) for v in [0, 1): quadrant of 4 v, Taylor polynomials of sin x
// (to x^13) and cos x (to x^14) on x in [0, pi/2).
__device__ __attribute__((always_inline)) inline void cossin32(float v, float* cs, float* sn) {
#pragma clang fp contract(off)
  const float y = v * 4.0f;
  const int q = (int)y;
  const float x = (y - (float)q) * 0x1.921fb6p+0f;
  const float x2 = x * x;
  float sp = 0x1.612462p-33f * x2 + -0x1.ae6456p-26f;
  sp = sp * x2 + 0x1.71de3ap-19f;
  sp = sp * x2 + -0x1.a01a02p-13f;
  sp = sp * x2 + 0x1.111112p-7f;
  sp = sp * x2 + -0x1.555556p-3f;
  sp = sp * x2 + 1.0f;
  const float s = x * sp;
  float cp = -0x1.93974ap-37f * x2 + 0x1.1eed8ep-29f;
  cp = cp * x2 + -0x1.27e4fcp-22f;
  cp = cp * x2 + 0x1.a01a02p-16f;
  cp = cp * x2 + -0x1.6c16c2p-10f;
  cp = cp * x2 + 0x1.555556p-5f;
  cp = cp * x2 + -0.5f;
  cp = cp * x2 + 1.0f;
  const float c = cp;
  *cs = q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
  *sn = q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
}

// The eight entries c = 8g .. 8g+7 of row beta of Omega_k.
__device__ __attribute__((always_inline)) inline void omega8(uint64_t seed, int k, int64_t beta, int g,
                                                             float (&z)[8]) {
#pragma clang fp contract(off)
  uint64_t x[4] = {(uint64_t)beta, (uint64_t)g, 0ull, 0ull};
  philox4x64_10(x, seed, (uint64_t)k);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float u = uniform23((uint32_t)x[j]), v = uniform23((uint32_t)(x[j] >> 32));
    const float r = (float)sqrt((double)(-2.0f * ln32(u)));
    float cs, sn;
    cossin32(v, &cs, &sn);
    z[2 * j] = r * cs;
    z[2 * j + 1] = r * sn;
  }
}

}  // namespace ttr

namespace ttr {

// Rows [beta0, beta0 + rows) of Omega_k (zero beyond row n), entries c < 8 ceil(s / 8)
// (zero for c >= s), rounded once to T and written into LDS by `nthr` threads (tid =
// 0 .. nthr-1 among them): entry (b, c) goes to Om[b * rs + c * cs] (rs = pitch, cs = 1
// for a row-major tile; rs = 1, cs = pitch for a transposed one).
template <typename T>
__device__ __attribute__((always_inline)) inline void omega_tile(uint64_t seed, int k, int64_t beta0, int rows,
                                                                 int64_t n, int s, T* __restrict__ Om, int rs, int cs,
                                                                 int tid, int nthr) {
  const int g8 = (s + 7) / 8;
  for (int id = tid; id < rows * g8; id += nthr) {
    const int b = id / g8, g = id - b * g8;
    float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (beta0 + b < n) omega8(seed, k, beta0 + b, g, z);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = 8 * g + j;
      // z is a float32: its round to nearest even into T equals that of (double)z
      Om[b * rs + c * cs] = c < s ? (T)z[j] : T(0);
    }
  }
}

}  // namespace ttr
