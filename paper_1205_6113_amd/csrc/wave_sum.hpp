// Cross-lane sums within a 64-wide wavefront (device code of the HIP sources).
#pragma once
#include <hip/hip_runtime.h>

namespace cpc {

// v from another lane through a DPP lane pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of W lanes; the total is valid in each group's first lane.
// Lane exchanges: xor 1, xor 2 (quad permutations), mirror within 8 and within 16
// (DPP), xor 16 within 32 (swizzle), lane 32 read into lane 0.
template <int W>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (W >= 2) v += dpp<0xB1>(v);
  if constexpr (W >= 4) v += dpp<0x4E>(v);
  if constexpr (W >= 8) v += dpp<0x141>(v);
  if constexpr (W >= 16) v += dpp<0x140>(v);
  if constexpr (W >= 32) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    v += __hiloint2double(hi, lo);
  }
  if constexpr (W >= 64)
    v += __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                          __builtin_amdgcn_readlane(__double2loint(v), 32));
  return v;
}

// gsum<64> of M values at once, exchange by exchange across all of them, so that the
// swizzles of the M values are in flight together instead of one value's chain
// waiting on each of its own (the same additions in the same order per value).
template <int M>
__device__ __forceinline__ void wave_sums(double (&v)[M]) {
#pragma unroll
  for (int r = 0; r < M; ++r) v[r] += dpp<0xB1>(v[r]);
#pragma unroll
  for (int r = 0; r < M; ++r) v[r] += dpp<0x4E>(v[r]);
#pragma unroll
  for (int r = 0; r < M; ++r) v[r] += dpp<0x141>(v[r]);
#pragma unroll
  for (int r = 0; r < M; ++r) v[r] += dpp<0x140>(v[r]);
  int lo[M], hi[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    lo[r] = __builtin_amdgcn_ds_swizzle(__double2loint(v[r]), 0x401F);
    hi[r] = __builtin_amdgcn_ds_swizzle(__double2hiint(v[r]), 0x401F);
  }
#pragma unroll
  for (int r = 0; r < M; ++r) v[r] += __hiloint2double(hi[r], lo[r]);
#pragma unroll
  for (int r = 0; r < M; ++r)
    v[r] += __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[r]), 32),
                             __builtin_amdgcn_readlane(__double2loint(v[r]), 32));
}

}  // namespace cpc
