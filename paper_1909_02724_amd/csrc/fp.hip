// Adjoint of the back-projection (forward projection) for gfx950: every
// voxel scatters scale * W * w_tap * vol into its four taps, with exactly the
// coordinates and weights of the matching back-projection variant (same
// brick setup, brick.h; FP32 columns for the tiled variant, FP64 columns for
// the direct one), so each is the transpose of its back-projector up to
// rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "brick.h"

namespace fdk {
namespace {

// Tiled variant: per view, the brick's splats accumulate in LDS tiles with
// the back-projector's transposed layout (one more column, for the u + 1
// taps) as 32-bit fixed point, a row's and its mirror row's sums paired in
// one 64-bit word (FP32 for bricks that need it, one plane for main rows
// and one for mirror rows); the tiles are then added to the projection with
// one global atomic per non-zero pixel. Direct variant: global atomics per
// tap.

__device__ __forceinline__ void splat(float* __restrict__ qs, int32_t nu, int32_t nv, int32_t a,
                                      float du, int32_t ra, int32_t rb, float fr, float val) {
  const float wa = val * (1.0f - fr), wb = val * fr;
  const float w[4] = {wa * (1.0f - du), wa * du, wb * (1.0f - du), wb * du};
  const int32_t cols[4] = {a, a + 1, a, a + 1};
  const int32_t rows[4] = {ra, ra, rb, rb};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (static_cast<uint32_t>(cols[m]) < static_cast<uint32_t>(nu) &&
        static_cast<uint32_t>(rows[m]) < static_cast<uint32_t>(nv))
      unsafeAtomicAdd(qs + static_cast<int64_t>(rows[m]) * nu + cols[m], w[m]);
  }
}

// Slot order of a lane in the adjoint. Lanes of a wave that share a detector
// column (along the rays) would otherwise add to the same LDS or global
// address in the same instruction, which serialises; rotating each lane's
// walk over its 16 slots by (tx + 4 ty) mod 16 puts such lanes on
// different rows.
__device__ __forceinline__ uint32_t slot_rotation(const TileShape& ts) {
  const uint32_t tx = threadIdx.x % kBrickX, ty = (threadIdx.x / kBrickX) & 3u;
  return (static_cast<uint32_t>(ts.rot_a) * tx + static_cast<uint32_t>(ts.rot_b) * ty) &
         (kBrickZ - 1);
}

// Voxel values of the thread's column, scaled, in the lane's slot order:
// x[t] is slot sl = (t + rot) mod 16; xm[t] is its mirror (mirrored runs)
// or slot 16 + sl (plain runs, whose bricks hold 32 slices).
template <bool MIRROR>
__device__ __forceinline__ void load_voxels(const GeoConst& gc, const SliceRun& run,
                                            const BrickCoords& bc, const float* __restrict__ vol,
                                            float scale, uint32_t rot, float* x, float* xm) {
  const int64_t slice = static_cast<int64_t>(gc.nx) * gc.ny;
  const int64_t col = static_cast<int64_t>(bc.j) * gc.nx + bc.i;
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) {
    const int32_t sl = static_cast<int32_t>((t + rot) & (kBrickZ - 1));
    const bool in = bc.owner && (bc.t0 + sl < run.n);
    x[t] = in ? scale * vol[static_cast<int64_t>(run.loc_lo + bc.t0 + sl) * slice + col] : 0.0f;
    if (MIRROR) {
      xm[t] = in ? scale * vol[static_cast<int64_t>(run.loc_hi - bc.t0 - sl) * slice + col] : 0.0f;
    } else {
      const bool in2 = bc.owner && (bc.t0 + kBrickZ + sl < run.n);
      xm[t] = in2 ? scale * vol[static_cast<int64_t>(run.loc_lo + bc.t0 + kBrickZ + sl) * slice + col]
                  : 0.0f;
    }
  }
}

// Accumulation for the tiled adjoint. LDS float atomics are serialised on
// gfx950: about 3 clocks per active lane per CU, 194 per full wave, against
// about 4.6 for a 32-bit integer add of a full wave and 6.4 for a 64-bit one
// (measured). A brick's splats therefore accumulate as 32-bit fixed point
// with integer LDS atomics (exact and independent of order within the
// workgroup), a tap's main and mirror sums in one 64-bit add, unless the
// brick spans a wide dynamic range: more than 1 % of its non-zero voxels
// lie below 2^-13 of its largest magnitude. Such a brick accumulates in
// 64-bit fixed point (the same scale rule with 2^63, one 64-bit add per
// tap), half a unit (about 2^-63 K M) per contribution: a voxel 2^-40 of
// the largest reaches a pixel through a full-weight tap at about 2^-24 K
// relative precision, so this serves bricks whose non-zero magnitudes span
// at most 2^40 (taps with weights near zero keep the absolute bound only).
// Two kinds take FP32 atomics (float tile, planar layout) instead:
//  - a brick with a NaN or an infinity, which integers cannot carry;
//  - a wide-range brick spanning more than 2^40, or one whose launch stages
//    a single view (its 64-bit tile would not fit).
// The FP32 path is slow (a workgroup on it can take longer than the rest of
// its launch), so it is kept for what fixed point cannot represent.
// On the FP32 path each pixel's sum carries FP32 rounding relative to its
// own contributions and non-finite values reach exactly the pixels they
// touch.
//
// Fixed-point scale, per brick and view, from a bound on what one pixel can
// receive:
//  - a column adds to the pixel columns floor(u) and floor(u) + 1, so pixel
//    column p hears only from columns with floor(u) in {p - 1, p};
//  - of a column's slices in the brick (16, or 32 for a plain run), those
//    with a tap on row r have v in [r - 1, r + 1): at most
//    floor(2 / (dv/dk)) + 2 of them (one spare for the rounding of v), and
//    never more than the brick's slice count;
//  - each contribution is at most M = max over columns of max|x| * W.
// A histogram over floor(u) of the per-column slot bounds gives K, the most
// contributions any pixel can receive; S = 2^(31 - e) with 1.01 K M < 2^e
// keeps every partial sum, rounding included, inside int32. S is a power of
// two, so the scaling is exact and cannot overflow however small or large
// the values. A pixel's quantisation error is at most half a unit,
// 2^(e - 32) ~ K M 2^-31, per contribution (one unit for splats above 2^23
// units, whose FP32 value is coarser than that anyway): relative to the
// brick's largest splat, not to the pixel's own sum, which is why
// wide-range bricks take 64 bits or FP32.
constexpr int32_t kHistStride = kThreads;  // tile columns tu + 1 <= 256
constexpr int64_t kFpSplitTarget = 4096;    // workgroups below which views are split
constexpr int kFpWideRangeLog2 = 13;        // "small" voxels: below 2^-13 of the brick's max
constexpr int kFpWideRangePct = 1;          // wide-range path above 1 % small voxels
constexpr int kFp64RangeLog2 = 40;          // 64-bit fixed point up to this magnitude range

// FP32 splat (FP32 path): taps (u, n), (u + 1, n), (u, n + 1),
// (u + 1, n + 1) of a tile with column pitch tvp.
__device__ __forceinline__ void splat_f32(float* p, int32_t tvp, float val, float fr, float du) {
  // (1 - fr) first: val - val fr would carry the rounding of val fr, up to
  // 2^-25 val, into a near-zero weight.
  const float fb = val * fr, fa = val * (1.0f - fr);
  const float du0 = 1.0f - du;
  atomicAdd(p, fa * du0);
  atomicAdd(p + tvp, fa * du);
  atomicAdd(p + 1, fb * du0);
  atomicAdd(p + tvp + 1, fb * du);
}

// Fixed point of x: floor(x + 0.5) in one conversion, exact below 2^23
// units and within one unit above (where the FP32 product feeding it is
// already coarser than a unit).
__device__ __forceinline__ int32_t fixed_round(float x) {
  int32_t r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Adds the fixed-point pair (a, b) to the 64-bit word at p, a into the low
// half and b into the high half: the addend is the 64-bit integer
// b 2^32 + a (a sign-extended), so every partial sum is exactly
// (sum b) 2^32 + (sum a), and both halves decode exactly while each sum
// stays inside int32. One 64-bit LDS add serves the row and its mirror.
__device__ __forceinline__ void add_pair(uint64_t* p, float a, float b) {
  const int32_t lo = fixed_round(a), hi = fixed_round(b);
  const uint64_t word = (static_cast<uint64_t>(static_cast<uint32_t>(hi + (lo >> 31))) << 32) |
                        static_cast<uint32_t>(lo);
  atomicAdd(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(word));
}

// Adds x, rounded to the nearest integer, to the 64-bit fixed-point sum at p.
__device__ __forceinline__ void add_fixed64(uint64_t* p, float x) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p),
            static_cast<unsigned long long>(__float2ll_rn(x)));
}

template <bool MIRROR>
__device__ __forceinline__ void fp_tiled_body(GeoConst gc, SliceRun run, ViewBatch vb,
                                              TileShape ts, const float* __restrict__ vol,
                                              float* __restrict__ q, int64_t vstride,
                                              float scale, int fixed_sums) {
  extern __shared__ __attribute__((aligned(16))) int atile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  __shared__ uint32_t hist[kMaxStageViews * kHistStride];
  __shared__ uint32_t kcount[kMaxStageViews], mbits[kMaxStageViews];
  __shared__ uint32_t amax_bits, amin_bits, n_nonzero, n_small, nonfinite;
  const int32_t tid = threadIdx.x;
  constexpr int BZ = MIRROR ? kBrickZ : kPlainBrickZ;  // slices per brick
  // blockIdx.y picks this workgroup's share of the launch's views: small
  // volumes split the views over several workgroups per brick (the
  // projections take their sums through atomics either way), so the grid
  // fills the chip more than once over.
  const int32_t per = (vb.nviews + static_cast<int32_t>(gridDim.y) - 1) / static_cast<int32_t>(gridDim.y);
  const int32_t v_lo = static_cast<int32_t>(blockIdx.y) * per;
  const int32_t v_hi = min(vb.nviews, v_lo + per);
  if (v_lo >= v_hi) return;  // uniform, before any barrier
  const BrickCoords bc = brick_coords(gc, run, ts, BZ);
  if (tid == 0) {
    amax_bits = n_nonzero = n_small = nonfinite = 0u;
    amin_bits = __float_as_uint(INFINITY);
  }
  if (tid >= v_lo && tid < v_hi)
    bvs[tid] = brick_setup(gc, view_geo(gc, vb.sn[tid], vb.cs[tid]), bc.i_lo, bc.i_hi, bc.j_lo, bc.j_hi, bc.kb, 0, 0, BZ,
                           MIRROR);
  const uint32_t rot = slot_rotation(ts);
  float x[kBrickZ], xm[kBrickZ];
  load_voxels<MIRROR>(gc, run, bc, vol, scale, rot, x, xm);
  // Brick statistics: largest and smallest non-zero magnitudes, non-finite
  // values (x - x is NaN exactly for those), then how many non-zero voxels
  // are small against the largest.
  float amax = 0.0f, amin = INFINITY;
  bool bad = false;
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) {
    amax = fmaxf(amax, fmaxf(fabsf(x[t]), fabsf(xm[t])));
    amin = fminf(amin, fminf(x[t] != 0.0f ? fabsf(x[t]) : INFINITY,
                             xm[t] != 0.0f ? fabsf(xm[t]) : INFINITY));
    bad = bad || ((x[t] - x[t]) != 0.0f) || ((xm[t] - xm[t]) != 0.0f);
  }
  __syncthreads();
  atomicMax(&amax_bits, __float_as_uint(amax));  // non-negative floats order as integers
  atomicMin(&amin_bits, __float_as_uint(amin));
  if (bad) nonfinite = 1u;
  __syncthreads();
  {
    const float small = ldexpf(__uint_as_float(amax_bits), -kFpWideRangeLog2);
    uint32_t nz = 0, ns = 0;
#pragma unroll
    for (int t = 0; t < kBrickZ; ++t) {
      nz += (x[t] != 0.0f) + (xm[t] != 0.0f);
      ns += (x[t] != 0.0f && fabsf(x[t]) < small) + (xm[t] != 0.0f && fabsf(xm[t]) < small);
    }
    if (nz) atomicAdd(&n_nonzero, nz);
    if (ns) atomicAdd(&n_small, ns);
  }
  __syncthreads();
  if (amax_bits == 0u && nonfinite == 0u) return;  // an all-zero brick adds nothing (uniform)
  // Accumulation of the brick (uniform): 32-bit fixed point; 64-bit fixed
  // point for a wide-range brick whose non-zero magnitudes span at most
  // 2^kFp64RangeLog2, with half the views per stage (its entries take twice
  // the bytes); FP32 for a brick with non-finite values, a wider range, or
  // when a stage holds a single view.
  // (With fixed_sums every finite brick takes 32 bits.)
  const bool wide_range =
      !fixed_sums && 100u * n_small > static_cast<uint32_t>(kFpWideRangePct) * n_nonzero;
  const bool fixed64 = nonfinite == 0u && wide_range && ts.vc >= 2 &&
                       __uint_as_float(amax_bits) <=
                           ldexpf(__uint_as_float(amin_bits), kFp64RangeLog2);
  const bool fp32_path = nonfinite != 0u || (wide_range && !fixed64);
  const int32_t vstep = fixed64 ? ts.vc / 2 : ts.vc;

  const float kvf = static_cast<float>(gc.kv);
  const int32_t tuf = ts.tu + 1, tv = ts.tv, tvp = ts.tvp;
  const int32_t slot = tuf * tvp;
  const int32_t rstep = kThreads / tuf;
  const int32_t sr = tid / tuf, sc = tid - sr * tuf;
  for (int32_t s0 = v_lo; s0 < v_hi; s0 += vstep) {
    const int32_t nvc = min(vstep, v_hi - s0);
    // Main rows in planes [0, vc) and mirror rows in planes [vc, 2 vc), one
    // 32-bit word per pixel: all LDS banks serve the adds (interleaved
    // (main, mirror) pairs reached only half of them and conflicted 10-way).
    // (The 32-bit fixed-point path of mirrored runs uses the same bytes as
    // 64-bit (main, mirror) words instead, the 64-bit one as 16-byte
    // (main, mirror) entries, and that of plain runs as 64-bit words.)
    int* const mtile = atile + ts.vc * slot;
    for (int32_t e = tid; e < (MIRROR ? 2 : 1) * ts.vc * slot; e += kThreads) atile[e] = 0;
    if (!fp32_path) {
      for (int32_t e = tid; e < nvc * kHistStride; e += kThreads) hist[e] = 0u;
      if (tid < nvc) kcount[tid] = mbits[tid] = 0u;
    }
    __syncthreads();
    if (!fp32_path) {
      // Bounds: histogram of the columns' slot bounds over floor(u), and
      // the largest contribution.
      if (bc.owner) {
        for (int32_t sl = 0; sl < nvc; ++sl) {
          const ColumnF32 c = column_f32(bvs[s0 + sl], bc.txf, bc.tyf, kvf);
          const uint32_t nu = min(c.nu, static_cast<uint32_t>(ts.tu - 1));
          const float ks = fminf(static_cast<float>(BZ), floorf(2.0f / c.dvk) + 2.0f);
          atomicAdd(&hist[sl * kHistStride + nu], static_cast<uint32_t>(ks));
          atomicMax(&mbits[sl], __float_as_uint(amax * c.w));
        }
      }
      __syncthreads();
      if (tid < tuf) {
        for (int32_t sl = 0; sl < nvc; ++sl) {
          const uint32_t* h = hist + sl * kHistStride;
          atomicMax(&kcount[sl], (tid < ts.tu ? h[tid] : 0u) + (tid > 0 ? h[tid - 1] : 0u));
        }
      }
      __syncthreads();
    }
    if (bc.owner) {
      for (int32_t sl = 0; sl < nvc; ++sl) {
        const ColumnF32 c = column_f32(bvs[s0 + sl], bc.txf, bc.tyf, kvf);
        const uint32_t nu = min(c.nu, static_cast<uint32_t>(ts.tu - 1));
        if (!fp32_path) {
          const float km = 1.01f * static_cast<float>(kcount[sl]) * __uint_as_float(mbits[sl]);
          if (!(km > 0.0f)) continue;  // nothing reaches this view (uniform)
          int e;
          frexpf(km, &e);
          const float du0 = 1.0f - c.du;
          if (fixed64) {
            // S = 2^(63 - e), applied to W x (at most M) so that no
            // intermediate overflows.
            const int sh = 63 - e;
            if constexpr (MIRROR) {
              uint64_t* const base =
                  reinterpret_cast<uint64_t*>(atile) + 2 * (sl * slot + nu * tvp + c.nvb);
              uint64_t* const base1 = base + 2 * tvp;  // pixel column u + 1
#pragma unroll
              for (int t = 0; t < kBrickZ; ++t) {
                uint32_t dn;
                float fr;
                voxel_row_off(c.fvb, c.dvk, static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn, &fr);
                const float val = ldexpf(c.w * x[t], sh), vm = ldexpf(c.w * xm[t], sh);
                const float wa = val * (1.0f - fr), wb = val * fr;
                const float ma = vm * (1.0f - fr), mb = vm * fr;
                uint64_t* const p = base + 2 * dn;
                uint64_t* const p1 = base1 + 2 * dn;
                add_fixed64(p, wa * du0);
                add_fixed64(p + 1, ma * du0);
                add_fixed64(p1, wa * c.du);
                add_fixed64(p1 + 1, ma * c.du);
                add_fixed64(p + 2, wb * du0);
                add_fixed64(p + 3, mb * du0);
                add_fixed64(p1 + 2, wb * c.du);
                add_fixed64(p1 + 3, mb * c.du);
              }
            } else {
              uint64_t* const base = reinterpret_cast<uint64_t*>(atile) + sl * slot + nu * tvp + c.nvb;
              uint64_t* const base1 = base + tvp;
#pragma unroll
              for (int t = 0; t < kBrickZ; ++t) {
                const int32_t tt = static_cast<int32_t>((t + rot) & (kBrickZ - 1));
                uint32_t dn, dn2;
                float fr, fr2;
                voxel_row_off(c.fvb, c.dvk, tt, &dn, &fr);
                voxel_row_off(c.fvb, c.dvk, kBrickZ + tt, &dn2, &fr2);
                const float val = ldexpf(c.w * x[t], sh), v2 = ldexpf(c.w * xm[t], sh);
                const float wa = val * (1.0f - fr), wb = val * fr;
                const float a2 = v2 * (1.0f - fr2), b2 = v2 * fr2;
                add_fixed64(base + dn, wa * du0);
                add_fixed64(base1 + dn, wa * c.du);
                add_fixed64(base + dn + 1, wb * du0);
                add_fixed64(base1 + dn + 1, wb * c.du);
                add_fixed64(base + dn2, a2 * du0);
                add_fixed64(base1 + dn2, a2 * c.du);
                add_fixed64(base + dn2 + 1, b2 * du0);
                add_fixed64(base1 + dn2 + 1, b2 * c.du);
              }
            }
            continue;
          }
          const float ws = ldexpf(c.w, 31 - e);  // W S, S = 2^(31 - e)
          if constexpr (MIRROR) {
            // (main, mirror) pairs of 32-bit sums in 64-bit words.
            uint64_t* const base = reinterpret_cast<uint64_t*>(atile) + sl * slot + nu * tvp + c.nvb;
            uint64_t* const base1 = base + tvp;  // pixel column u + 1
#pragma unroll
            for (int t = 0; t < kBrickZ; ++t) {
              uint32_t dn;
              float fr;
              voxel_row_off(c.fvb, c.dvk, static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn, &fr);
              const float val = ws * x[t], vm = ws * xm[t];
              const float wa = val * (1.0f - fr), wb = val * fr;
              const float ma = vm * (1.0f - fr), mb = vm * fr;
              add_pair(base + dn, wa * du0, ma * du0);
              add_pair(base1 + dn, wa * c.du, ma * c.du);
              add_pair(base + dn + 1, wb * du0, mb * du0);
              add_pair(base1 + dn + 1, wb * c.du, mb * c.du);
            }
            continue;
          }
          int* const base = atile + sl * slot + nu * tvp + c.nvb;
          int* const base1 = base + tvp;  // pixel column u + 1
#pragma unroll
          for (int t = 0; t < kBrickZ; ++t) {
            uint32_t dn;
            float fr;
            voxel_row_off(c.fvb, c.dvk, static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn, &fr);
            const float val = ws * x[t];
            const float wa = val * (1.0f - fr), wb = val * fr;
            atomicAdd(base + dn, fixed_round(wa * du0));
            atomicAdd(base1 + dn, fixed_round(wa * c.du));
            atomicAdd(base + dn + 1, fixed_round(wb * du0));
            atomicAdd(base1 + dn + 1, fixed_round(wb * c.du));
            {
              // The brick's upper 16 slices, into the same plane.
              uint32_t dn2;
              float fr2;
              voxel_row_off(c.fvb, c.dvk,
                            kBrickZ + static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn2, &fr2);
              const float v2 = ws * xm[t];
              const float a2 = v2 * (1.0f - fr2), b2 = v2 * fr2;
              atomicAdd(base + dn2, fixed_round(a2 * du0));
              atomicAdd(base1 + dn2, fixed_round(a2 * c.du));
              atomicAdd(base + dn2 + 1, fixed_round(b2 * du0));
              atomicAdd(base1 + dn2 + 1, fixed_round(b2 * c.du));
            }
          }
        } else {
          float* const fbase = reinterpret_cast<float*>(atile) + sl * slot + nu * tvp + c.nvb;
          float* const fmbase = reinterpret_cast<float*>(mtile) + sl * slot + nu * tvp + c.nvb;
#pragma unroll
          for (int t = 0; t < kBrickZ; ++t) {
            uint32_t dn;
            float fr;
            voxel_row_off(c.fvb, c.dvk, static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn, &fr);
            splat_f32(fbase + dn, tvp, c.w * x[t], fr, c.du);
            if (MIRROR) {
              splat_f32(fmbase + dn, tvp, c.w * xm[t], fr, c.du);
            } else {
              uint32_t dn2;
              float fr2;
              voxel_row_off(c.fvb, c.dvk,
                            kBrickZ + static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn2, &fr2);
              splat_f32(fbase + dn2, tvp, c.w * xm[t], fr2, c.du);
            }
          }
        }
      }
    }
    __syncthreads();
    // Flush: entry (r, c) holds pixel (org_u + c, org_v + r) and, for
    // mirrored runs, pixel (org_u + c, G - org_v - r).
    if (sr < rstep) {
      for (int32_t sl = 0; sl < nvc; ++sl) {
        const int32_t s = s0 + sl;
        const int32_t gu = bvs[s].org_u + sc;
        if (static_cast<uint32_t>(gu) >= static_cast<uint32_t>(gc.nu)) continue;
        // Value of one fixed-point unit: 2^(e - 31), or 2^(e - 63) for the
        // 64-bit path (unused on the FP32 path).
        float inv_s = 0.0f;
        double inv_s64 = 0.0;
        if (!fp32_path) {
          int e;
          frexpf(1.01f * static_cast<float>(kcount[sl]) * __uint_as_float(mbits[sl]), &e);
          inv_s = ldexpf(1.0f, e - 31);
          inv_s64 = ldexp(1.0, e - 63);
        }
        float* qs = q + s * vstride + gu;
        for (int32_t r = sr; r < tv; r += rstep) {
          const int32_t at = sl * slot + sc * tvp + r;
          float ex, ey = 0.0f;
          if (fp32_path) {
            ex = __int_as_float(atile[at]);
            if (MIRROR) ey = __int_as_float(mtile[at]);
          } else if (fixed64) {
            const int64_t* const w = reinterpret_cast<const int64_t*>(atile);
            ex = static_cast<float>(static_cast<double>(w[MIRROR ? 2 * at : at]) * inv_s64);
            if (MIRROR) ey = static_cast<float>(static_cast<double>(w[2 * at + 1]) * inv_s64);
          } else if (MIRROR) {
            // Word = (mirror sum) 2^32 + (main sum), both int32.
            const uint64_t w = reinterpret_cast<const uint64_t*>(atile)[at];
            const int32_t lo = static_cast<int32_t>(static_cast<uint32_t>(w));
            const int32_t hi = static_cast<int32_t>((w - static_cast<uint64_t>(static_cast<int64_t>(lo))) >> 32);
            ex = static_cast<float>(lo) * inv_s;
            ey = static_cast<float>(hi) * inv_s;
          } else {
            ex = static_cast<float>(atile[at]) * inv_s;
          }
          const int32_t gr = bvs[s].org_v + r;
          if (ex != 0.0f && static_cast<uint32_t>(gr) < static_cast<uint32_t>(gc.nv))
            unsafeAtomicAdd(qs + static_cast<int64_t>(gr) * gc.nu, ex);
          if (MIRROR) {
            const int32_t gm = gc.mirror_g - gr;
            if (ey != 0.0f && static_cast<uint32_t>(gm) < static_cast<uint32_t>(gc.nv))
              unsafeAtomicAdd(qs + static_cast<int64_t>(gm) * gc.nu, ey);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <bool MIRROR>
__global__ void fp_tiled_kernel(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                                const float* __restrict__ vol, float* __restrict__ q,
                                int64_t vstride, float scale, int fixed_sums);

// Mirrored runs: six 256-thread workgroups per CU (80 VGPRs). The 64-bit
// paths' code otherwise lifts the register count past it, and five
// workgroups cost 11 % at 2048^3. (Held to 80 registers, the plain variant
// spills inside its splat loops, so it keeps its count.)
template <>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6)))
void fp_tiled_kernel<true>(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                           const float* __restrict__ vol, float* __restrict__ q, int64_t vstride,
                           float scale, int fixed_sums) {
  fp_tiled_body<true>(gc, run, vb, ts, vol, q, vstride, scale, fixed_sums);
}

template <>
__global__ __launch_bounds__(kThreads)
void fp_tiled_kernel<false>(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                            const float* __restrict__ vol, float* __restrict__ q, int64_t vstride,
                            float scale, int fixed_sums) {
  fp_tiled_body<false>(gc, run, vb, ts, vol, q, vstride, scale, fixed_sums);
}

template <bool MIRROR>
__global__ __launch_bounds__(kThreads) void fp_direct_kernel(GeoConst gc, SliceRun run,
                                                             ViewBatch vb, TileShape ts,
                                                             const float* __restrict__ vol,
                                                             float* __restrict__ q,
                                                             int64_t vstride, float scale) {
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  const int32_t tid = threadIdx.x;
  constexpr int BZ = MIRROR ? kBrickZ : kPlainBrickZ;  // slices per brick
  const BrickCoords bc = brick_coords(gc, run, ts, BZ);
  if (tid < vb.nviews)
    bvs[tid] = brick_setup(gc, view_geo(gc, vb.sn[tid], vb.cs[tid]), bc.i_lo, bc.i_hi, bc.j_lo, bc.j_hi, bc.kb, 0, 0, BZ,
                           MIRROR);
  const uint32_t rot = slot_rotation(ts);
  float x[kBrickZ], xm[kBrickZ];
  load_voxels<MIRROR>(gc, run, bc, vol, scale, rot, x, xm);
  __syncthreads();
  if (!bc.owner) return;
  for (int32_t s = 0; s < vb.nviews; ++s) {
    const ColumnF32 c = column_f64(gc, view_geo(gc, vb.sn[s], vb.cs[s]), bvs[s], bc.i, bc.j, bc.kb);
    float* qs = q + s * vstride;
    const int32_t a = bvs[s].org_u + static_cast<int32_t>(c.nu);
    const int32_t nb = bvs[s].org_v + static_cast<int32_t>(c.nvb);
#pragma unroll
    for (int t = 0; t < kBrickZ; ++t) {
      const int32_t sl = static_cast<int32_t>((t + rot) & (kBrickZ - 1));
      if (bc.t0 + sl >= run.n) continue;
      uint32_t dn;
      float fr;
      voxel_row_off(c.fvb, c.dvk, sl, &dn, &fr);
      const int32_t n = nb + static_cast<int32_t>(dn);
      splat(qs, gc.nu, gc.nv, a, c.du, n, n + 1, fr, c.w * x[t]);
      if (MIRROR) {
        const int32_t m = gc.mirror_g - n;
        splat(qs, gc.nu, gc.nv, a, c.du, m, m - 1, fr, c.w * xm[t]);
      } else if (bc.t0 + kBrickZ + sl < run.n) {
        uint32_t dn2;
        float fr2;
        voxel_row_off(c.fvb, c.dvk, kBrickZ + sl, &dn2, &fr2);
        const int32_t n2 = nb + static_cast<int32_t>(dn2);
        splat(qs, gc.nu, gc.nv, a, c.du, n2, n2 + 1, fr2, c.w * xm[t]);
      }
    }
  }
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    p[m] = 0.0f;
}

}  // namespace

int launch_forward_project(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                           const TileShape& ts, const float* vol, float* q, int64_t vstride,
                           float scale, bool fixed_sums, void* stream) {
  const uint64_t nwg = static_cast<uint64_t>(ts.nbx) * ts.nby * ts.nseg;
  const dim3 block(kThreads);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ts.vc > 0) {
    // Views split over workgroups when the bricks alone give fewer than
    // kFpSplitTarget workgroups.
    int64_t vsplit = 1;
    if (nwg < static_cast<uint64_t>(kFpSplitTarget))
      vsplit = (kFpSplitTarget + static_cast<int64_t>(nwg) - 1) / static_cast<int64_t>(nwg);
    vsplit = std::max<int64_t>(1, std::min<int64_t>(vsplit, vb.nviews));
    const dim3 grid(static_cast<uint32_t>(nwg), static_cast<uint32_t>(vsplit));
    // Adjoint tile: one more column than the back-projection tile, one
    // 32-bit word per pixel and plane (main, plus mirror for mirrored runs).
    // The host sizes the back-projection tile at 16 (mirrored) or 8 (plain)
    // bytes per entry, so at least one view's tile always fits.
    TileShape tf = ts;
    const int64_t per_view =
        static_cast<int64_t>(ts.tu + 1) * ts.tvp * sizeof(int) * (run.mirror ? 2 : 1);
    tf.vc = static_cast<int32_t>(std::min<int64_t>(kMaxStageViews, kTileLdsBytes / per_view));
    if (tf.vc < 1) return static_cast<int>(hipErrorInvalidValue);
    const size_t lds = static_cast<size_t>(tf.vc) * per_view;
    if (run.mirror)
      hipLaunchKernelGGL((fp_tiled_kernel<true>), grid, block, lds, st, gc, run, vb, tf, vol,
                         q, vstride, scale, static_cast<int>(fixed_sums));
    else
      hipLaunchKernelGGL((fp_tiled_kernel<false>), grid, block, lds, st, gc, run, vb, tf, vol,
                         q, vstride, scale, static_cast<int>(fixed_sums));
  } else {
    const dim3 grid(static_cast<uint32_t>(nwg));
    if (run.mirror)
      hipLaunchKernelGGL((fp_direct_kernel<true>), grid, block, 0, st, gc, run, vb, ts, vol, q,
                         vstride, scale);
    else
      hipLaunchKernelGGL((fp_direct_kernel<false>), grid, block, 0, st, gc, run, vb, ts, vol, q,
                         vstride, scale);
  }
  return static_cast<int>(hipGetLastError());
}

int launch_fill_zero(float* p, int64_t n, void* stream) {
  if (n <= 0) return 0;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), p, n);
  return static_cast<int>(hipGetLastError());
}

}  // namespace fdk
