// Device-side coordinate arithmetic shared by the back-projector and its
// adjoint, so both map every (voxel, view) to the same taps and weights.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdk_internal.h"

namespace fdk {

// Storage tags for 16-bit projections.
struct f16_t {
  uint16_t bits;
};
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(f16_t x) {
  return static_cast<float>(__builtin_bit_cast(_Float16, x.bits));
}
__device__ __forceinline__ float to_f32(bf16_t x) { return __uint_as_float(uint32_t(x.bits) << 16); }

// Row index and fraction of voxel kb + t on the column: v = v(kb) + t dv/dk.
// The offset tt is never negative (fvb >= 0, dv/dk > 0), so truncation is
// floor and the hardware fraction is tt - floor(tt), both exact.
__host__ __device__ __forceinline__ void voxel_row_off(float fvb, float dvk, int32_t t,
                                                       uint32_t* n, float* fr) {
  const float tt = fmaf(static_cast<float>(t), dvk, fvb);
  *n = static_cast<uint32_t>(tt);
#if defined(__HIP_DEVICE_COMPILE__)
  *fr = __builtin_amdgcn_fractf(tt);
#else
  *fr = tt - floorf(tt);
#endif
}

}  // namespace fdk
