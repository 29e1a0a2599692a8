// Internal launch descriptors shared by the host front end (fdk_api.cpp) and
// the HIP kernels. Not part of the public ABI.
#pragma once

#include <cstdint>

#include "../../include/fdk.h"

namespace fdk {

// Views per kernel launch: each view's sine and cosine travel in the kernel
// argument block (16 bytes a view), and each launch reads (and for the
// back-projector writes) the volume once and sets up each brick once; the
// views of a call are split evenly over the fewest launches. Measured at
// 2048^3: the back-projector 6 % faster with 64 views a launch than with
// 32, and 3 % faster again with 96. The adjoint takes 96 only when every
// launch's views then span at most kFpWideSpanRad: one slot rotation serves
// all views of a launch, and 96 views spread over 120 degrees cost it 11 %
// at 2048^3, while launches over 68 and 90 degrees gained 3 % (512^3 from
// 512 views, 256^3 from 360). Otherwise it takes at most 64 (2 % faster than
// 32 at 2048^3, 10 % at 256^3 from 360 views).
constexpr int kMaxViewsPerLaunch = 96;
constexpr int kFpViewsPerLaunch = 64;
constexpr double kFpWideSpanRad = 1.75;  // about 100 degrees

// Per-view geometry in the reduced-cost form of Alg. 4, evaluated in FP64
// from the sine and cosine of the view angle (Eq. 2 expanded; view_geo, on
// the host and in the kernels):
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
  double dx, dy, d;   // voxel pitches in x and y, source to axis
  double ox, oy;      // volume centre column (voxels)
  int32_t mirror_g;   // Nv - 1 + 2 off_v when that is an integer (Theorem 1)
};

// ViewGeo of the view with sin(beta) = s, cos(beta) = c (Eq. 2 expanded:
// world X = Dx (i - ox), Y = -Dy (j - oy); after the rotation,
// z = d + sin(b) X + cos(b) Y and a = cos(b) X - sin(b) Y). Host and device.
constexpr ViewGeo view_geo(const GeoConst& gc, double s, double c) {
  ViewGeo v{};
  v.ci = s * gc.dx;
  v.cj = -c * gc.dy;
  v.c0 = gc.d - s * gc.dx * gc.ox + c * gc.dy * gc.oy;
  v.ai = c * gc.dx;
  v.aj = s * gc.dy;
  v.a0 = -c * gc.dx * gc.ox - s * gc.dy * gc.oy;
  return v;
}

// A run of global slices processed by one launch family.
//  mirror = 0: slices k_first + t (t < n) stored at slab slice loc_lo + t.
//  mirror = 1: pairs (k_first + t, Nz - 1 - k_first - t), t < n; the lower
//              slice at loc_lo + t, its mirror at loc_hi - t.
struct SliceRun {
  int32_t k_first, n, loc_lo, loc_hi, mirror;
};

struct ViewBatch {
  double sn[kMaxViewsPerLaunch], cs[kMaxViewsPerLaunch];  // sin and cos of each view's angle
  int32_t nviews;
};

// Bricked back-projection: a workgroup of 256 threads owns a brick of
// kBrickX x kBrickY columns and kBrickZ consecutive slices of a slice run
// (plus their mirrors for a mirrored run). In the tiled variant it stages
// the brick's detector footprint for each view, a tile of tu x tv pixels,
// into LDS, vc views at a time. tu and tv are host-side upper bounds.
constexpr int kBrickX = 16;
constexpr int kBrickY = 16;
constexpr int kBrickZ = 16;
constexpr int kBrickThreads = kBrickX * kBrickY;
constexpr int kWaveLanes = 64;
// Occupancy decides the back-projector's speed more than staging depth
// does (measured on MI355X): five 256-thread workgroups per CU, hence at
// most 27.5 KB of tiles (with the 4.5 KB of per-view brick constants, 32 KB
// a workgroup) and 102 VGPRs, with two views per stage, run 5 %
// faster than four with three views (and four with three 11 % (FP32) to
// 47 % (FP16) faster than three with four). The adjoint stages up to three
// views in 35.5 KB.
constexpr int kMaxStageViews = 3;
constexpr int kBpStageViews = 2;
constexpr int kPrefetchSlots = 6;       // tile entries a thread prefetches per stage
// Tiles too tall for the five-wave back-projector's slots (more than three
// staging passes per view) go to a four-wave instance with more slots.
constexpr int kWidePrefetchSlots = 12;
constexpr int kTileLdsBytes = 36352;    // LDS budget for the adjoint's and the four-wave tiles
constexpr int kBpTileLdsBytes = 28160;  // and for the five-wave back-projector's
constexpr int kTileEntryBytes = 16;     // (q, dq/du) of a row and of its mirror row

struct TileShape {
  int32_t tu, tv, tvp;   // tile columns, rows, and the (odd) column pitch in entries
  int32_t vc;            // views staged at once; 0 selects the direct variant
  int32_t rstep, rows;   // staging: rows advanced per pass, passes per view
  int32_t wide;          // back-projector: the four-wave instance with kWidePrefetchSlots
  int32_t nbx, nby, nseg;  // bricks along x, y and z-segments of the run
  // Adjoint: lane (tx, ty) visits its slots from (rot_a tx + rot_b (ty mod 4))
  // mod 16 on, which spreads the lanes' LDS adds over the banks.
  int32_t rot_a, rot_b;
};

// Kernel choice for a run and view batch: tiled unless the footprint tile
// exceeds the LDS or prefetch budget, or the caller asks for the direct
// variant (FDK_DIRECT).
// bz: slices per brick; entry_bytes: LDS bytes per tile entry; slots: tile
// entries a thread prefetches per stage; bp_staging: the back-projector's
// staging (lane groups per tile row) rather than the adjoint's; read_pitch:
// pad the column pitch for the mirrored back-projector's conflict-free
// entry reads.
TileShape tile_shape(const fdk_geometry* g, const GeoConst& gc, const SliceRun& run,
                     const ViewBatch& vb, int32_t bz, int32_t entry_bytes, int32_t slots,
                     bool direct, bool bp_staging = false, bool read_pitch = false);
// Plain (unmirrored) back-projection runs: 32 slices per brick, the tile
// holding (q, dq/du) of the main rows only; a prefetch slot holds one row's
// pair instead of two, so twice as many fit the same registers.
constexpr int kPlainBrickZ = 2 * kBrickZ;
constexpr int kPlainEntryBytes = 8;
constexpr int kPlainPrefetchSlots = 2 * kPrefetchSlots;

// Launchers (defined in the .hip files). They return a hipError_t as int.
int launch_backproject(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                       const TileShape& ts, const void* q, fdk_dtype q_dtype,
                       int64_t view_stride, float* vol, float scale, int accumulate,
                       void* stream);
int launch_forward_project(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                           const TileShape& ts, const float* vol, float* q, int64_t view_stride,
                           float scale, bool fixed_sums, void* stream);
int launch_fill_zero(float* p, int64_t n, void* stream);
}  // namespace fdk
