// Internal launch descriptors shared by the host front end (fdk_api.cpp) and
// the HIP kernels. Not part of the public ABI.
#pragma once

#include <cstdint>

#include "../../include/fdk.h"

namespace fdk {

// Views per kernel launch: the per-view constants travel in the kernel
// argument block, and each launch reads and writes the volume once.
constexpr int kMaxViewsPerLaunch = 32;

// Per-view geometry in the reduced-cost form of Alg. 4, evaluated in FP64 on
// the host from the view angle (Eq. 2 expanded):
//   z(i, j)   = ci*i + cj*j + c0                      (Eq. 3, Theorem 3)
//   a(i, j)   = ai*i + aj*j + a0   gantry coordinate across the detector
//   u         = cu + ku * a / z                        (Theorem 2)
//   v(k)      = cv + kv * (k - cz) / z                 (linear in k)
struct ViewGeo {
  double ai, aj, a0;
  double ci, cj, c0;
};

// Launch-invariant geometry.
struct GeoConst {
  int32_t nx, ny, nz, nu, nv;
  double cu, cv, cz;  // principal point (pixels) and volume centre slice
  double ku;          // D / Du
  double kv;          // D * Dz / Dv
  int32_t mirror_g;   // Nv - 1 + 2 off_v when that is an integer (Theorem 1)
};

// A run of global slices processed by one launch family.
//  mirror = 0: slices k_first + t (t < n) stored at slab slice loc_lo + t.
//  mirror = 1: pairs (k_first + t, Nz - 1 - k_first - t), t < n; the lower
//              slice at loc_lo + t, its mirror at loc_hi - t.
struct SliceRun {
  int32_t k_first, n, loc_lo, loc_hi, mirror;
};

struct ViewBatch {
  ViewGeo view[kMaxViewsPerLaunch];
  int32_t nviews;
};

// Launchers (defined in the .hip files). They return a hipError_t as int.
int launch_backproject(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                       const void* q, fdk_dtype q_dtype, int64_t view_stride,
                       float* vol, float scale, int accumulate, void* stream);
int launch_forward_project(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                           const float* vol, float* q, int64_t view_stride, float scale,
                           void* stream);
int launch_fill_zero(float* p, int64_t n, void* stream);
int launch_filter(const GeoConst& gc, double du, double dv, double sod, double sdd,
                  int32_t nrows, const float* e, void* q, fdk_dtype out_dtype,
                  fdk_filter_kind kind, void* stream);

}  // namespace fdk
