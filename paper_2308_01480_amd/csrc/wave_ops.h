// Cross-lane reductions of float64 values inside one 64-lane wavefront (DPP row
// operations, a 32-lane swizzle and lane reads): no LDS and no barriers.
#pragma once

#include <hip/hip_runtime.h>

namespace ttr {

template <int CTRL>
__device__ inline double dpp_mov(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sums over aligned lane groups; every lane of the group obtains the same bits.
__device__ inline double sum8(double v) {
  v += dpp_mov<0xB1>(v);   // lane ^ 1
  v += dpp_mov<0x4E>(v);   // lane ^ 2
  v += dpp_mov<0x141>(v);  // mirror within 8
  return v;
}
__device__ inline double sum16(double v) {
  v += dpp_mov<0xB1>(v);   // lane ^ 1
  v += dpp_mov<0x4E>(v);   // lane ^ 2
  v += dpp_mov<0x141>(v);  // mirror within 8
  v += dpp_mov<0x140>(v);  // mirror within 16
  return v;
}
__device__ inline double swz16(double v) {  // value of lane ^ 16 (within 32)
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_ds_swizzle(lo, 0x401F);
  hi = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
  return __hiloint2double(hi, lo);
}
__device__ inline double sum32(double v) {
  v = sum16(v);
  return v + swz16(v);
}
__device__ inline double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ inline double sum64(double v) {
  v = sum32(v);
  return lane_value(v, 0) + lane_value(v, 32);
}
__device__ inline double min64(double v) {
  v = fmin(v, dpp_mov<0xB1>(v));
  v = fmin(v, dpp_mov<0x4E>(v));
  v = fmin(v, dpp_mov<0x141>(v));
  v = fmin(v, dpp_mov<0x140>(v));
  v = fmin(v, swz16(v));
  return fmin(lane_value(v, 0), lane_value(v, 32));
}
__device__ inline double max64(double v) { return -min64(-v); }
}  // namespace ttr
