// Brick geometry shared by the back-projector and its adjoint (gfx950).
//
// A workgroup of 256 threads owns a brick of 16 x 16 (x, y) columns and 16
// consecutive slices of a slice run; for a mirrored run (Theorem 1) each
// thread also owns the 16 mirror voxels of its column.
//
// Coordinates. For each (brick, view) one lane evaluates, in FP64, the
// tile origin (the floor of the smallest u and v over the brick's corners,
// minus one pixel) and a handful of brick constants; every thread then
// derives its column's u, v(kb), W = f^2 and dv/dk in FP32 from offsets
// relative to the brick origin (Theorems 2 and 3: u and z, hence f, are
// fixed along the column; v is affine in k). All FP32 quantities are small
// offsets, which keeps coordinates accurate to a few 1e-6 pixel at 4096
// pixels. Per voxel: v = v(kb) + t dv/dk, one truncation, one fraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "geom_device.h"

namespace fdk {
namespace {

constexpr int kThreads = kBrickThreads;

template <typename T>
__device__ __forceinline__ float tap(const T* __restrict__ qs, int32_t nu, int32_t nv, int32_t a,
                                     int32_t b) {
  // Taps outside the detector read zero.
  return (static_cast<uint32_t>(a) < static_cast<uint32_t>(nu) &&
          static_cast<uint32_t>(b) < static_cast<uint32_t>(nv))
             ? to_f32(qs[static_cast<int64_t>(b) * nu + a])
             : 0.0f;
}

// Per (brick, view) constants. With tx = i - i_lo, ty = j - j_lo and
// dz = ci tx + cj ty, f = 1 / (zo + dz):
//   u    - org_u = uo + (au tx + bu ty) f
//   v(kb) - org_v = vo + (av tx + bv ty) f
// (from u = cu + ku a / z and v = cv + kv (k - cz) / z, expanded about the
// brick origin column so every FP32 term is a small offset).
struct BrickView {
  float uo, vo, au, bu, av, bv, zo, ci, cj;
  int32_t org_u, org_v;
  int32_t inside;  // the tile (columns org_u .. org_u + tu, its rows and mirror rows) is on the detector
};

// bz: slices per brick; mirror: whether the tile also holds the mirror rows
// (then `inside` requires them on the detector too). Also compiled for the
// host, where a test checks the tile bounds against every voxel's taps.
__host__ __device__ inline BrickView brick_setup(const GeoConst& gc, const ViewGeo& g, int32_t i_lo, int32_t i_hi,
                                 int32_t j_lo, int32_t j_hi, int32_t kb, int32_t tu = 0,
                                 int32_t tv = 0, int32_t bz = kBrickZ, bool mirror = true) {
  const double k0 = static_cast<double>(kb) - gc.cz;
  const double k1 = static_cast<double>(kb + bz - 1) - gc.cz;
  // u is a ratio of functions affine in (i, j) and v is affine in k at
  // fixed f: over the brick's (i, j, k) box both are extremal at corners.
  double umin = INFINITY, vmin = INFINITY;
  for (int c = 0; c < 4; ++c) {
    const double di = (c & 1) ? i_hi : i_lo, dj = (c & 2) ? j_hi : j_lo;
    const double z = fma(g.ci, di, fma(g.cj, dj, g.c0));
    const double f = 1.0 / z;
    const double a = fma(g.ai, di, fma(g.aj, dj, g.a0));
    umin = fmin(umin, fma(gc.ku * a, f, gc.cu));
    vmin = fmin(vmin, fmin(fma(gc.kv * k0, f, gc.cv), fma(gc.kv * k1, f, gc.cv)));
  }
  BrickView b;
  b.org_u = static_cast<int32_t>(floor(umin)) - 1;
  b.org_v = static_cast<int32_t>(floor(vmin)) - 1;
  const double zo = fma(g.ci, static_cast<double>(i_lo), fma(g.cj, static_cast<double>(j_lo), g.c0));
  const double fo = 1.0 / zo;
  const double ao = fma(g.ai, static_cast<double>(i_lo), fma(g.aj, static_cast<double>(j_lo), g.a0));
  const double ro = ao * fo;                 // a / z at the brick origin
  const double K = gc.kv * k0;               // v(kb) - cv = K f
  b.uo = static_cast<float>((gc.cu - b.org_u) + gc.ku * ro);
  b.vo = static_cast<float>((gc.cv - b.org_v) + K * fo);
  b.au = static_cast<float>(gc.ku * (g.ai - ro * g.ci));
  b.bu = static_cast<float>(gc.ku * (g.aj - ro * g.cj));
  b.av = static_cast<float>(-K * fo * g.ci);
  b.bv = static_cast<float>(-K * fo * g.cj);
  b.zo = static_cast<float>(zo);
  b.ci = static_cast<float>(g.ci);
  b.cj = static_cast<float>(g.cj);
  const bool cols_in = b.org_u >= 0 && b.org_u + tu < gc.nu;
  const bool rows_in = b.org_v >= 0 && b.org_v + tv <= gc.nv;
  // (mirror_g is INT32_MIN when there is no pixel-aligned mirror: only
  // mirrored runs, which have one, evaluate it.)
  const bool mirror_in =
      !mirror || (gc.mirror_g - b.org_v < gc.nv && gc.mirror_g - b.org_v - tv + 1 >= 0);
  b.inside = tu > 0 && cols_in && rows_in && mirror_in;
  return b;
}

// FP32 column quantities of one view for a thread at (tx, ty) in the brick.
struct ColumnF32 {
  uint32_t nu, nvb;  // tile column and first row (relative to the origin)
  float du, fvb;     // fractions of u and of v(kb)
  float w, dvk;      // W_dis = f^2 and dv/dk
};

// Hardware reciprocal (1 ulp) and fraction on the GPU; the host build, used
// only by the tile-bound test, takes the correctly rounded forms.
__host__ __device__ __forceinline__ float rcp_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float fract_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_fractf(x);
#else
  return x - floorf(x);
#endif
}

__host__ __device__ __forceinline__ ColumnF32 column_f32(const BrickView& b, float txf, float tyf,
                                                         float kvf) {
  const float f = rcp_f32(b.zo + fmaf(b.ci, txf, b.cj * tyf));
  const float ul = fmaf(fmaf(b.au, txf, b.bu * tyf), f, b.uo);
  const float vl = fmaf(fmaf(b.av, txf, b.bv * tyf), f, b.vo);
  ColumnF32 c;
  c.nu = static_cast<uint32_t>(ul);  // ul, vl >= 1 by the origin margin
  c.du = fract_f32(ul);
  c.nvb = static_cast<uint32_t>(vl);
  c.fvb = fract_f32(vl);
  c.w = f * f;
  c.dvk = kvf * f;
  return c;
}

// The same quantities computed per column in FP64 (direct variant: it runs
// when footprints are too large for LDS, i.e. at strong magnification,
// where brick-relative FP32 offsets would span hundreds of pixels).
// Indices are relative to the brick's tile origin, as in column_f32.
__device__ __forceinline__ ColumnF32 column_f64(const GeoConst& gc, const ViewGeo& g,
                                                const BrickView& b, int32_t i, int32_t j,
                                                int32_t kb) {
  const double di = static_cast<double>(i), dj = static_cast<double>(j);
  const double z = fma(g.ci, di, fma(g.cj, dj, g.c0));
  const double f = 1.0 / z;
  const double a = fma(g.ai, di, fma(g.aj, dj, g.a0));
  const double ul = fma(gc.ku * a, f, gc.cu) - b.org_u;  // exact: integer shift
  const double vl = fma(gc.kv * (static_cast<double>(kb) - gc.cz), f, gc.cv) - b.org_v;
  const double fu = floor(ul), fv = floor(vl);
  ColumnF32 c;
  c.nu = static_cast<uint32_t>(fu);
  c.du = static_cast<float>(ul - fu);
  c.nvb = static_cast<uint32_t>(fv);
  c.fvb = static_cast<float>(vl - fv);
  c.w = static_cast<float>(f * f);
  c.dvk = static_cast<float>(gc.kv * f);
  return c;
}

struct BrickCoords {
  int32_t i_lo, i_hi, j_lo, j_hi, i, j, t0, kb;
  float txf, tyf;
  bool owner;
};

// Brick (bx, by, z-segment) of this workgroup. Workgroups are dealt
// round-robin to the 8 XCDs, and each XCD takes a contiguous range of a
// linear order that runs over z-segments outermost and, within a segment,
// over bands of kBandRows brick rows, column by column. The workgroups an
// XCD holds at once (32 CUs x 4) then form a compact patch of bricks, about
// 16 x 8, whose detector footprints overlap from brick to brick, so that its
// L2 serves most of their taps (a row of bricks across the volume did not).
constexpr uint32_t kBandRows = 8;
__device__ __forceinline__ void brick_index(const TileShape& ts, int32_t* bx, int32_t* by,
                                            int32_t* seg) {
  const uint32_t nwg = gridDim.x;
  uint32_t lin = blockIdx.x;
  if ((nwg & 7u) == 0) lin = (lin & 7u) * (nwg >> 3) + (lin >> 3);
  const uint32_t nbx = static_cast<uint32_t>(ts.nbx), nby = static_cast<uint32_t>(ts.nby);
  const uint32_t plane = nbx * nby;
  const uint32_t sg = lin / plane, r = lin - sg * plane;
  const uint32_t band = r / (kBandRows * nbx);
  const uint32_t rows = min(kBandRows, nby - band * kBandRows);
  const uint32_t rb = r - band * kBandRows * nbx;
  *bx = static_cast<int32_t>(rb / rows);
  *by = static_cast<int32_t>(band * kBandRows + rb % rows);
  *seg = static_cast<int32_t>(sg);
}

__device__ __forceinline__ BrickCoords brick_coords(const GeoConst& gc, const SliceRun& run,
                                                    const TileShape& ts, int32_t bz = kBrickZ) {
  int32_t bx, by, seg;
  brick_index(ts, &bx, &by, &seg);
  BrickCoords bc;
  bc.i_lo = bx * kBrickX;
  bc.j_lo = by * kBrickY;
  bc.i_hi = min(bc.i_lo + kBrickX - 1, gc.nx - 1);
  bc.j_hi = min(bc.j_lo + kBrickY - 1, gc.ny - 1);
  const int32_t tx0 = threadIdx.x % kBrickX, ty0 = threadIdx.x / kBrickX;
  bc.owner = (bc.i_lo + tx0 <= bc.i_hi) && (bc.j_lo + ty0 <= bc.j_hi);
  bc.i = min(bc.i_lo + tx0, bc.i_hi);
  bc.j = min(bc.j_lo + ty0, bc.j_hi);
  bc.txf = static_cast<float>(bc.i - bc.i_lo);
  bc.tyf = static_cast<float>(bc.j - bc.j_lo);
  bc.t0 = seg * bz;
  bc.kb = run.k_first + bc.t0;
  return bc;
}

}  // namespace
}  // namespace fdk
