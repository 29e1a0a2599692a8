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

// Per (column, view) quantities of Alg. 4, lines 6-10, plus the start of the
// column's v walk. u, z (hence f and W) do not depend on k (Theorems 2, 3);
// v is affine in k. Computed once per column and view in FP64 from the
// host's FP64 view geometry, then split into an integer pixel index and an
// FP32 fraction, so that the per-voxel FP32 work only ever handles small
// offsets (a few pixels) and keeps ~1e-6 pixel accuracy at 4096 pixels.
struct ColumnView {
  int32_t nu0;  // floor(u)
  float du;     // u - floor(u)
  float w;      // W_dis = f^2
  int32_t nvb;  // floor(v(kb))
  float fvb;    // v(kb) - floor(v(kb))
  float dvk;    // dv/dk = kv * f
};

__device__ __forceinline__ ColumnView column_view(const GeoConst& gc, const ViewGeo& vg, int32_t i,
                                                  int32_t j, int32_t kb) {
  const double di = static_cast<double>(i), dj = static_cast<double>(j);
  const double z = fma(vg.ci, di, fma(vg.cj, dj, vg.c0));
  const double f = 1.0 / z;
  const double a = fma(vg.ai, di, fma(vg.aj, dj, vg.a0));
  const double u = fma(gc.ku * a, f, gc.cu);
  const double v = fma(gc.kv * (static_cast<double>(kb) - gc.cz), f, gc.cv);
  const double fu = floor(u), fv = floor(v);
  ColumnView c;
  c.nu0 = static_cast<int32_t>(fu);
  c.du = static_cast<float>(u - fu);
  c.w = static_cast<float>(f * f);
  c.nvb = static_cast<int32_t>(fv);
  c.fvb = static_cast<float>(v - fv);
  c.dvk = static_cast<float>(gc.kv * f);
  return c;
}

// Row index and fraction of voxel kb + t on the column: v = v(kb) + t dv/dk.
// The offset tt is never negative (fvb >= 0, dv/dk > 0), so truncation is
// floor and the hardware fraction is tt - floor(tt), both exact.
__device__ __forceinline__ void voxel_row_off(float fvb, float dvk, int32_t t, uint32_t* n,
                                              float* fr) {
  const float tt = fmaf(static_cast<float>(t), dvk, fvb);
  *n = static_cast<uint32_t>(tt);
  *fr = __builtin_amdgcn_fractf(tt);
}

__device__ __forceinline__ void voxel_row(const ColumnView& c, int32_t t, int32_t* n, float* fr) {
  uint32_t dn;
  voxel_row_off(c.fvb, c.dvk, t, &dn, fr);
  *n = c.nvb + static_cast<int32_t>(dn);
}

}  // namespace fdk
