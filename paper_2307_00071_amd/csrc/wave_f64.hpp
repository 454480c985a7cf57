// Wave-level FP64 reductions in a fixed order, shared by the device code.
#pragma once

#include <hip/hip_runtime.h>

namespace gmm_wave {

// FP64 reductions over the 16 lanes of a DPP row (mirror, half-mirror,
// xor 2, xor 1 exchanges): every lane of the row ends with the same bits,
// as each exchange adds the same two values on both sides.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0x140>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x4E>(v);
  return v + dpp_f64<0xB1>(v);
}
__device__ __forceinline__ double row16_max(double v) {
  v = fmax(v, dpp_f64<0x140>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  return fmax(v, dpp_f64<0xB1>(v));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// The sum over a wave: the four row sums added in row order (wave-uniform).
__device__ __forceinline__ double wave_sum_f64(double v) {
  v = row16_sum(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) +
         (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// The sums of the two 32-lane halves of a wave (lanes 0-31, 32-63), each
// the two row sums added in row order (wave-uniform).
__device__ __forceinline__ double2 half_sums_f64(double v) {
  v = row16_sum(v);
  return make_double2(readlane_f64(v, 0) + readlane_f64(v, 16),
                      readlane_f64(v, 32) + readlane_f64(v, 48));
}

// The same for 32-bit integers (exact, so any order gives the same sum).
__device__ __forceinline__ int wave_sum_i32(int v) {
  v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);
  v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);
  v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
  v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

}  // namespace gmm_wave
