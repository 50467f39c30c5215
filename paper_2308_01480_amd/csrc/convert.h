// Correctly rounded narrowing of float64 values on the device (round to nearest, ties
// to even).  bfloat16 goes through float32 with round-to-odd, which makes the second
// rounding exact: a single rounding of the float64 value, with no double-rounding
// error at ties.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ttr {

template <typename TO>
__device__ inline TO round_from_f64(double x) {
  return (TO)x;
}

template <>
__device__ inline __bf16 round_from_f64<__bf16>(double x) {
  if (x != x) return __builtin_bit_cast(__bf16, (unsigned short)0x7FC0u);
  const float f = (float)x;
  uint32_t u = __float_as_uint(f);
  const double back = (double)f;
  if (back != x) {  // inexact: truncate toward zero and set the sticky bit
    if (fabs(back) > fabs(x)) u -= 1u;
    u |= 1u;
  }
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

}  // namespace ttr
