// Back-projection (Alg. 2 computed as Alg. 4) and its exact adjoint for
// gfx950.
//
// Work decomposition. A workgroup of 256 threads owns a brick of 16 x 16
// (x, y) columns and 16 consecutive slices of a slice run; for a mirrored
// run (Theorem 1) each thread also owns the 16 mirror voxels of its
// column. Each thread accumulates every view of the launch in registers
// and writes each voxel once per launch; lanes run along x, so volume
// traffic is coalesced. No atomics: every voxel has one owner and a fixed
// summation order, so results are bitwise reproducible.
//
// Coordinates. For each (brick, view) one lane evaluates, in FP64, the
// tile origin (the floor of the smallest u and v over the brick's corners,
// minus one pixel) and a handful of brick constants; every thread then
// derives its column's u, v(kb), W = f^2 and dv/dk in FP32 from offsets
// relative to the brick origin (Theorems 2 and 3: u and z, hence f, are
// fixed along the column; v is affine in k). All FP32 quantities are small
// offsets, which keeps coordinates accurate to a few 1e-6 pixel at 4096
// pixels. Per voxel: v = v(kb) + t dv/dk, one truncation, one fraction.
//
// Tiled variant (the main path). Per view, the brick's detector footprint
// is staged into LDS, transposed (v fastest, odd column pitch), as entries
// holding q(u, v) and q(u+1, v) - q(u, v) for the row and for its mirror
// row G - v, mirror rows in reverse order. A voxel and its mirror then read
// the same two adjacent entries with the same weights: one address and one
// fraction serve the pair, and the u-interpolation is a single FMA on the
// staged difference. Staging uses buffer loads whose out-of-range offsets
// return zero (taps outside the detector), and the next views' loads are
// issued before the current views are computed.
//
// Direct variant (fallback when a tile exceeds the LDS budget, and the
// reference the tiled variant is tested against bit for bit): identical
// arithmetic, taps read from global memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>

#include "geom_device.h"

namespace fdk {
namespace {

constexpr int kThreads = kBrickThreads;
constexpr uint32_t kBadCol = 0x40000000u;  // pushes a buffer offset out of range
constexpr uint32_t kBadRow = 0x80000000u;
constexpr int kBufferWord3 = 0x00020000;   // raw buffer descriptor, gfx9 family

template <typename T>
__device__ __forceinline__ float tap(const T* __restrict__ qs, int32_t nu, int32_t nv, int32_t a,
                                     int32_t b) {
  // Taps outside the detector read zero.
  return (static_cast<uint32_t>(a) < static_cast<uint32_t>(nu) &&
          static_cast<uint32_t>(b) < static_cast<uint32_t>(nv))
             ? to_f32(qs[static_cast<int64_t>(b) * nu + a])
             : 0.0f;
}

// Raw buffer loads for the staging prefetch: the bits stay untouched in
// registers (no wait on the load) and are converted when the tile is written.
template <typename T>
__device__ __forceinline__ uint32_t buf_load_raw(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ uint32_t buf_load_raw<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
template <>
__device__ __forceinline__ uint32_t buf_load_raw<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
template <>
__device__ __forceinline__ uint32_t buf_load_raw<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
template <typename T>
__device__ __forceinline__ float raw_to_f32(uint32_t bits);
template <>
__device__ __forceinline__ float raw_to_f32<float>(uint32_t bits) {
  return __uint_as_float(bits);
}
template <>
__device__ __forceinline__ float raw_to_f32<f16_t>(uint32_t bits) {
  return to_f32(f16_t{static_cast<uint16_t>(bits)});
}
template <>
__device__ __forceinline__ float raw_to_f32<bf16_t>(uint32_t bits) {
  return __uint_as_float(bits << 16);
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

__device__ BrickView brick_setup(const GeoConst& gc, const ViewGeo& g, int32_t i_lo, int32_t i_hi,
                                 int32_t j_lo, int32_t j_hi, int32_t kb, int32_t tu = 0,
                                 int32_t tv = 0) {
  const double k0 = static_cast<double>(kb) - gc.cz;
  const double k1 = static_cast<double>(kb + kBrickZ - 1) - gc.cz;
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
  const bool mirror_in = gc.mirror_g - b.org_v < gc.nv && gc.mirror_g - b.org_v - tv + 1 >= 0;
  b.inside = tu > 0 && cols_in && rows_in && mirror_in;
  return b;
}

// FP32 column quantities of one view for a thread at (tx, ty) in the brick.
struct ColumnF32 {
  uint32_t nu, nvb;  // tile column and first row (relative to the origin)
  float du, fvb;     // fractions of u and of v(kb)
  float w, dvk;      // W_dis = f^2 and dv/dk
};

__device__ __forceinline__ ColumnF32 column_f32(const BrickView& b, float txf, float tyf,
                                                float kvf) {
  const float f = __builtin_amdgcn_rcpf(b.zo + fmaf(b.ci, txf, b.cj * tyf));
  const float ul = fmaf(fmaf(b.au, txf, b.bu * tyf), f, b.uo);
  const float vl = fmaf(fmaf(b.av, txf, b.bv * tyf), f, b.vo);
  ColumnF32 c;
  c.nu = static_cast<uint32_t>(ul);  // ul, vl >= 1 by the origin margin
  c.du = __builtin_amdgcn_fractf(ul);
  c.nvb = static_cast<uint32_t>(vl);
  c.fvb = __builtin_amdgcn_fractf(vl);
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

template <typename T, bool MIRROR, bool TILED>
__device__ __forceinline__ void bp_brick_body(const GeoConst& gc, const SliceRun& run,
                                              const ViewBatch& vb, const TileShape& ts,
                                              const T* __restrict__ q, int64_t vstride,
                                              float* __restrict__ vol, float scale,
                                              int accumulate, float4* tile, BrickView* bvs) {

  const int32_t tid = threadIdx.x;
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of bricks so neighbours share footprints in its L2.
  const uint32_t nwg = gridDim.x;
  uint32_t lin = blockIdx.x;
  if ((nwg & 7u) == 0) lin = (lin & 7u) * (nwg >> 3) + (lin >> 3);
  const int32_t bx = static_cast<int32_t>(lin % static_cast<uint32_t>(ts.nbx));
  lin /= static_cast<uint32_t>(ts.nbx);
  const int32_t by = static_cast<int32_t>(lin % static_cast<uint32_t>(ts.nby));
  const int32_t seg = static_cast<int32_t>(lin / static_cast<uint32_t>(ts.nby));

  const int32_t i_lo = bx * kBrickX, j_lo = by * kBrickY;
  const int32_t i_hi = min(i_lo + kBrickX - 1, gc.nx - 1);
  const int32_t j_hi = min(j_lo + kBrickY - 1, gc.ny - 1);
  const int32_t tx0 = tid % kBrickX, ty0 = tid / kBrickX;
  const bool owner = (i_lo + tx0 <= i_hi) && (j_lo + ty0 <= j_hi);
  const int32_t i = min(i_lo + tx0, i_hi), j = min(j_lo + ty0, j_hi);
  const float txf = static_cast<float>(i - i_lo), tyf = static_cast<float>(j - j_lo);
  const int32_t t0 = seg * kBrickZ;
  const int32_t kb = run.k_first + t0;
  const float kvf = static_cast<float>(gc.kv);

  if (tid < vb.nviews)
    bvs[tid] = brick_setup(gc, vb.view[tid], i_lo, i_hi, j_lo, j_hi, kb, ts.tu, ts.tv);
  __syncthreads();

  float acc[kBrickZ], accm[kBrickZ];
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) acc[t] = accm[t] = 0.0f;

  if constexpr (TILED) {
    const int32_t tu = ts.tu, tv = ts.tv, tvp = ts.tvp, rstep = ts.rstep, rows = ts.rows;
    const int32_t slot_entries = tu * tvp;
    // Staging assignment: thread -> tile column sc and rows sr + m * rstep
    // (lanes along u, so global reads are coalesced).
    const int32_t sr = tid / tu, sc = tid - sr * tu;
    const bool stager = sr < rstep;
    const uint32_t es = sizeof(T);
    const uint32_t row_es = static_cast<uint32_t>(gc.nu) * es;
    const uint32_t nrec = static_cast<uint32_t>(gc.nu) * static_cast<uint32_t>(gc.nv) * es;
    uint4 pre[kPrefetchSlots];  // raw bits of (q(u), q(u+1)) for the row and its mirror

    // Issue the loads of views [s0, s0 + nvc) into pre[]: raw (q(u), q(u+1))
    // for the row and for its mirror row. Views whose tile lies on the
    // detector skip the range checks.
    auto load_stage = [&](int32_t s0, int32_t nvc) {
      int32_t sl = 0, rr = 0;
      int32_t org_v = 0, inside = 0;
      uint32_t c0 = 0, c1 = 0, off = 0, offm = 0;
      const uint32_t step = static_cast<uint32_t>(rstep) * row_es;
#pragma unroll
      for (int m = 0; m < kPrefetchSlots; ++m) {
        if (sl < nvc) {
          // The descriptor is rebuilt per slot (scalar work): carried across
          // slots, the compiler moves it to vector registers and wraps each
          // load in a loop over lanes.
          const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
              const_cast<T*>(q + (s0 + sl) * vstride), 0, nrec, kBufferWord3);
          if (rr == 0) {  // uniform: new view
            const int32_t s = s0 + sl;
            const int32_t gu = bvs[s].org_u + sc;
            org_v = bvs[s].org_v;
            inside = __builtin_amdgcn_readfirstlane(bvs[s].inside);
            c0 = static_cast<uint32_t>(gu) < static_cast<uint32_t>(gc.nu)
                     ? static_cast<uint32_t>(gu) * es : kBadCol;
            c1 = static_cast<uint32_t>(gu + 1) < static_cast<uint32_t>(gc.nu)
                     ? static_cast<uint32_t>(gu + 1) * es : kBadCol;
            off = static_cast<uint32_t>(org_v + sr) * row_es + c0;
            offm = static_cast<uint32_t>(gc.mirror_g - org_v - sr) * row_es + c0;
          }
          // Only the offsets depend on the branch: the loads themselves are
          // issued in common code, unconditionally (uniform control flow),
          // so nothing waits for them until the tile is written. A lane with
          // no row here reads at an out-of-range offset, which returns zero
          // without a fetch. Views whose tile lies on the detector just step
          // the row offsets.
          const int32_t r = sr + rr * rstep;
          const bool on = stager && r < tv;
          uint32_t o0, o1, m0, m1;
          if (inside) {
            o0 = on ? off : kBadRow;
            o1 = o0 + es;
            m0 = on ? offm : kBadRow;
            m1 = m0 + es;
          } else {
            const int32_t gr = org_v + r, gm = gc.mirror_g - gr;
            const uint32_t ro = on && static_cast<uint32_t>(gr) < static_cast<uint32_t>(gc.nv)
                                    ? __umul24(static_cast<uint32_t>(gr), row_es) : kBadRow;
            const uint32_t rm = on && static_cast<uint32_t>(gm) < static_cast<uint32_t>(gc.nv)
                                    ? __umul24(static_cast<uint32_t>(gm), row_es) : kBadRow;
            o0 = ro + c0;
            o1 = ro + c1;
            m0 = rm + c0;
            m1 = rm + c1;
          }
          uint4 p;
          p.x = buf_load_raw<T>(rsrc, o0);
          p.y = buf_load_raw<T>(rsrc, o1);
          if (MIRROR) {
            p.z = buf_load_raw<T>(rsrc, m0);
            p.w = buf_load_raw<T>(rsrc, m1);
          }
          if (!MIRROR) p.z = p.w = 0u;
          pre[m] = p;
          off += step;
          offm -= step;
        }
        if (++rr == rows) {
          rr = 0;
          ++sl;
        }
      }
    };

    auto store_stage = [&](int32_t nvc) {
      int32_t sl = 0, rr = 0;
#pragma unroll
      for (int m = 0; m < kPrefetchSlots; ++m) {
        if (sl < nvc) {
          const int32_t r = sr + rr * rstep;
          if (stager && r < tv) {
            const float a0 = raw_to_f32<T>(pre[m].x), a1 = raw_to_f32<T>(pre[m].y);
            const float b0 = raw_to_f32<T>(pre[m].z), b1 = raw_to_f32<T>(pre[m].w);
            tile[sl * slot_entries + sc * tvp + r] = make_float4(a0, a1 - a0, b0, b1 - b0);
          }
        }
        if (++rr == rows) {
          rr = 0;
          ++sl;
        }
      }
    };

    const char* tile_bytes = reinterpret_cast<const char*>(tile);
    load_stage(0, min(ts.vc, vb.nviews));
    for (int32_t s0 = 0; s0 < vb.nviews; s0 += ts.vc) {
      const int32_t nvc = min(ts.vc, vb.nviews - s0);
      if (s0 > 0) __syncthreads();  // the previous views' tiles are consumed
      store_stage(nvc);
      __syncthreads();
      if (s0 + ts.vc < vb.nviews) load_stage(s0 + ts.vc, min(ts.vc, vb.nviews - s0 - ts.vc));
      for (int32_t sl = 0; sl < nvc; ++sl) {
        const ColumnF32 c = column_f32(bvs[s0 + sl], txf, tyf, kvf);
        const uint32_t nu = min(c.nu, static_cast<uint32_t>(tu - 1));
        // One register holds the column's tile offset, so each pair's
        // address is a single shift-and-add.
        uint32_t cbase = (static_cast<uint32_t>(sl * slot_entries) +
                          nu * static_cast<uint32_t>(tvp) + c.nvb) * kTileEntryBytes;
        asm volatile("" : "+v"(cbase));
        const char* pb = tile_bytes + cbase;
        // Reads run one voxel pair ahead of use, so LDS latency overlaps the
        // previous pair's arithmetic.
        uint32_t dn;
        float fr;
        voxel_row_off(c.fvb, c.dvk, 0, &dn, &fr);
        float4 A = reinterpret_cast<const float4*>(pb + dn * kTileEntryBytes)[0];
        float4 B = reinterpret_cast<const float4*>(pb + dn * kTileEntryBytes)[1];
#pragma unroll
        for (int t = 0; t < kBrickZ; ++t) {
          float4 An = A, Bn = B;
          uint32_t dn1 = 0;
          float fr1 = 0.0f;
          if (t + 1 < kBrickZ) {
            voxel_row_off(c.fvb, c.dvk, t + 1, &dn1, &fr1);
            const float4* p = reinterpret_cast<const float4*>(pb + dn1 * kTileEntryBytes);
            An = p[0];
            Bn = p[1];
          }
          const float ta = fmaf(c.du, A.y, A.x), tb = fmaf(c.du, B.y, B.x);
          acc[t] = fmaf(c.w, fmaf(fr, tb - ta, ta), acc[t]);
          if (MIRROR) {
            const float ma = fmaf(c.du, A.w, A.z), mb = fmaf(c.du, B.w, B.z);
            accm[t] = fmaf(c.w, fmaf(fr, mb - ma, ma), accm[t]);
          }
          A = An;
          B = Bn;
          fr = fr1;
        }
      }
    }
  } else {
    for (int32_t s = 0; s < vb.nviews; ++s) {
      const ColumnF32 c = column_f64(gc, vb.view[s], bvs[s], i, j, kb);
      const T* qs = q + s * vstride;
      const int32_t a = bvs[s].org_u + static_cast<int32_t>(c.nu);
      const int32_t nb = bvs[s].org_v + static_cast<int32_t>(c.nvb);
#pragma unroll
      for (int t = 0; t < kBrickZ; ++t) {
        uint32_t dn;
        float fr;
        voxel_row_off(c.fvb, c.dvk, t, &dn, &fr);
        const int32_t n = nb + static_cast<int32_t>(dn);
        const float q0a = tap(qs, gc.nu, gc.nv, a, n), q1a = tap(qs, gc.nu, gc.nv, a + 1, n);
        const float q0b = tap(qs, gc.nu, gc.nv, a, n + 1), q1b = tap(qs, gc.nu, gc.nv, a + 1, n + 1);
        const float ta = fmaf(c.du, q1a - q0a, q0a), tb = fmaf(c.du, q1b - q0b, q0b);
        acc[t] = fmaf(c.w, fmaf(fr, tb - ta, ta), acc[t]);
        if (MIRROR) {
          // Theorem 1: v(Nz-1-k) = G - v(k): rows G - n (weight 1 - fr) and
          // G - n - 1 (weight fr).
          const int32_t m = gc.mirror_g - n;
          const float r0a = tap(qs, gc.nu, gc.nv, a, m), r1a = tap(qs, gc.nu, gc.nv, a + 1, m);
          const float r0b = tap(qs, gc.nu, gc.nv, a, m - 1), r1b = tap(qs, gc.nu, gc.nv, a + 1, m - 1);
          const float ma = fmaf(c.du, r1a - r0a, r0a), mb = fmaf(c.du, r1b - r0b, r0b);
          accm[t] = fmaf(c.w, fmaf(fr, mb - ma, ma), accm[t]);
        }
      }
    }
  }

  if (!owner) return;
  const int64_t slice = static_cast<int64_t>(gc.nx) * gc.ny;
  const int64_t col = static_cast<int64_t>(j) * gc.nx + i;
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) {
    if (t0 + t >= run.n) break;
    float* p = vol + static_cast<int64_t>(run.loc_lo + t0 + t) * slice + col;
    *p = accumulate ? fmaf(scale, acc[t], *p) : scale * acc[t];
    if (MIRROR) {
      float* pm = vol + static_cast<int64_t>(run.loc_hi - t0 - t) * slice + col;
      *pm = accumulate ? fmaf(scale, accm[t], *pm) : scale * accm[t];
    }
  }
}

// The mirrored tiled variant runs four 256-thread workgroups per CU (four
// waves per SIMD): its LDS tiles fit 36 KB and it is held to 128 VGPRs.
template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
void bp_tiled_mirror_kernel(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                            const T* __restrict__ q, int64_t vstride, float* __restrict__ vol,
                            float scale, int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, true, true>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, tile, bvs);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void bp_tiled_plain_kernel(GeoConst gc, SliceRun run,
                                                                  ViewBatch vb, TileShape ts,
                                                                  const T* __restrict__ q,
                                                                  int64_t vstride,
                                                                  float* __restrict__ vol,
                                                                  float scale, int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, false, true>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, tile, bvs);
}

template <typename T, bool MIRROR>
__global__ __launch_bounds__(kThreads) void bp_direct_kernel(GeoConst gc, SliceRun run,
                                                             ViewBatch vb, TileShape ts,
                                                             const T* __restrict__ q,
                                                             int64_t vstride,
                                                             float* __restrict__ vol, float scale,
                                                             int accumulate) {
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, MIRROR, false>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, nullptr,
                                  bvs);
}

// ------------------------------------------------------------------------
// Adjoint (forward projection): every voxel scatters scale * W * w_tap * vol
// into its four taps, with exactly the coordinates and weights of the
// matching back-projection variant (same brick setup; FP32 columns for the
// tiled variant, FP64 columns for the direct one), so each is the transpose
// of its back-projector up to rounding.
//
// Tiled variant: per view, the brick's splats accumulate in LDS tiles with
// the back-projector's transposed layout (one more column, for the u + 1
// taps), one plane for main rows and one for mirror rows, as fixed-point
// integer atomics; the tiles are then added to the projection with one
// global atomic per non-zero pixel. Direct variant: global atomics per tap.
// ------------------------------------------------------------------------

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

struct BrickCoords {
  int32_t i_lo, i_hi, j_lo, j_hi, i, j, t0, kb;
  float txf, tyf;
  bool owner;
};

__device__ __forceinline__ BrickCoords brick_coords(const GeoConst& gc, const SliceRun& run,
                                                    const TileShape& ts) {
  const uint32_t nwg = gridDim.x;
  uint32_t lin = blockIdx.x;
  if ((nwg & 7u) == 0) lin = (lin & 7u) * (nwg >> 3) + (lin >> 3);
  const int32_t bx = static_cast<int32_t>(lin % static_cast<uint32_t>(ts.nbx));
  lin /= static_cast<uint32_t>(ts.nbx);
  const int32_t by = static_cast<int32_t>(lin % static_cast<uint32_t>(ts.nby));
  const int32_t seg = static_cast<int32_t>(lin / static_cast<uint32_t>(ts.nby));
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
  bc.t0 = seg * kBrickZ;
  bc.kb = run.k_first + bc.t0;
  return bc;
}

// Slot order of a lane in the adjoint. Lanes of a wave that share a detector
// column (along the rays) would otherwise add to the same LDS or global
// address in the same instruction, which serialises; rotating each lane's
// walk over its 16 slots by (tx + 4 ty) mod 16 puts such lanes on
// different rows.
__device__ __forceinline__ uint32_t slot_rotation() {
  const uint32_t tx = threadIdx.x % kBrickX, ty = (threadIdx.x / kBrickX) & 3u;
  return (tx + 4u * ty) & (kBrickZ - 1);
}

// Voxel values of the thread's column, scaled, in the lane's slot order:
// x[t] is slot (t + rot) mod 16.
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
    xm[t] = (MIRROR && in)
                ? scale * vol[static_cast<int64_t>(run.loc_hi - bc.t0 - sl) * slice + col]
                : 0.0f;
  }
}

// Fixed-point accumulation for the tiled adjoint. LDS float atomics are
// slow on gfx950 (about 40x an integer atomic, measured), so splats are
// accumulated as 32-bit fixed point with integer LDS atomics: exact and
// independent of order within the workgroup. The scale is chosen per brick
// and view from a bound on what one pixel can receive:
//  - a column adds to the pixel columns floor(u) and floor(u) + 1, so pixel
//    column p hears only from columns with floor(u) in {p - 1, p};
//  - of a column's 16 slots, those with a tap on row r have v in [r - 1,
//    r + 1): at most floor(2 / (dv/dk)) + 2 of them (one spare for the
//    rounding of v), and never more than 16;
//  - each contribution is at most M = max over columns of max|x| * W.
// A histogram over floor(u) of the per-column slot bounds gives K, the most
// contributions any pixel can receive, and S = 2^31 / (1.01 K M) keeps
// every partial sum, rounding included, inside int32. The quantisation step
// is then about 2^-31 of K M: the error is far below that of the FP32 sum
// for the real overlap of a brick's footprint.
constexpr int32_t kHistStride = kThreads;  // tile columns tu + 1 <= 256

template <bool MIRROR>
__global__ __launch_bounds__(kThreads) void fp_tiled_kernel(GeoConst gc, SliceRun run,
                                                            ViewBatch vb, TileShape ts,
                                                            const float* __restrict__ vol,
                                                            float* __restrict__ q,
                                                            int64_t vstride, float scale) {
  extern __shared__ int atile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  __shared__ uint32_t hist[kMaxStageViews * kHistStride];
  __shared__ uint32_t kcount[kMaxStageViews], mbits[kMaxStageViews];
  __shared__ uint32_t amax_bits;
  const int32_t tid = threadIdx.x;
  const BrickCoords bc = brick_coords(gc, run, ts);
  if (tid == 0) amax_bits = 0u;
  if (tid < vb.nviews)
    bvs[tid] = brick_setup(gc, vb.view[tid], bc.i_lo, bc.i_hi, bc.j_lo, bc.j_hi, bc.kb);
  const uint32_t rot = slot_rotation();
  float x[kBrickZ], xm[kBrickZ];
  load_voxels<MIRROR>(gc, run, bc, vol, scale, rot, x, xm);
  float amax = 0.0f;
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) amax = fmaxf(amax, fmaxf(fabsf(x[t]), fabsf(xm[t])));
  __syncthreads();
  atomicMax(&amax_bits, __float_as_uint(amax));  // non-negative floats order as integers
  __syncthreads();
  if (amax_bits == 0u) return;  // an all-zero brick adds nothing (uniform)

  const float kvf = static_cast<float>(gc.kv);
  const int32_t tuf = ts.tu + 1, tv = ts.tv, tvp = ts.tvp;
  const int32_t slot = tuf * tvp;
  const int32_t rstep = kThreads / tuf;
  const int32_t sr = tid / tuf, sc = tid - sr * tuf;
  for (int32_t s0 = 0; s0 < vb.nviews; s0 += ts.vc) {
    const int32_t nvc = min(ts.vc, vb.nviews - s0);
    // Main rows in planes [0, vc) and mirror rows in planes [vc, 2 vc), one
    // 32-bit word per pixel: all LDS banks serve the adds (interleaved
    // (main, mirror) pairs reached only half of them and conflicted 10-way).
    int* const mtile = atile + ts.vc * slot;
    for (int32_t e = tid; e < nvc * slot; e += kThreads) {
      atile[e] = 0;
      if (MIRROR) mtile[e] = 0;
    }
    for (int32_t e = tid; e < nvc * kHistStride; e += kThreads) hist[e] = 0u;
    if (tid < nvc) kcount[tid] = mbits[tid] = 0u;
    __syncthreads();
    // Bounds: histogram of the columns' slot bounds over floor(u), and the
    // largest contribution.
    if (bc.owner) {
      for (int32_t sl = 0; sl < nvc; ++sl) {
        const ColumnF32 c = column_f32(bvs[s0 + sl], bc.txf, bc.tyf, kvf);
        const uint32_t nu = min(c.nu, static_cast<uint32_t>(ts.tu - 1));
        const float ks = fminf(static_cast<float>(kBrickZ), floorf(2.0f / c.dvk) + 2.0f);
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
    if (bc.owner) {
      for (int32_t sl = 0; sl < nvc; ++sl) {
        const float km = static_cast<float>(kcount[sl]) * __uint_as_float(mbits[sl]);
        if (!(km > 0.0f)) continue;  // nothing reaches this view (uniform)
        const ColumnF32 c = column_f32(bvs[s0 + sl], bc.txf, bc.tyf, kvf);
        const uint32_t nu = min(c.nu, static_cast<uint32_t>(ts.tu - 1));
        int* const base = atile + sl * slot + nu * tvp + c.nvb;
        int* const base1 = base + tvp;  // pixel column u + 1
        int* const mbase = mtile + sl * slot + nu * tvp + c.nvb;
        int* const mbase1 = mbase + tvp;
        const float ws = c.w * (2147483648.0f / (1.01f * km));
        const float du0 = 1.0f - c.du;
#pragma unroll
        for (int t = 0; t < kBrickZ; ++t) {
          uint32_t dn;
          float fr;
          voxel_row_off(c.fvb, c.dvk, static_cast<int32_t>((t + rot) & (kBrickZ - 1)), &dn, &fr);
          const float val = ws * x[t];
          const float wa = val - val * fr, wb = val * fr;
          atomicAdd(base + dn, __float2int_rn(wa * du0));
          atomicAdd(base1 + dn, __float2int_rn(wa * c.du));
          atomicAdd(base + dn + 1, __float2int_rn(wb * du0));
          atomicAdd(base1 + dn + 1, __float2int_rn(wb * c.du));
          if (MIRROR) {
            const float vm = ws * xm[t];
            const float ma = vm - vm * fr, mb = vm * fr;
            atomicAdd(mbase + dn, __float2int_rn(ma * du0));
            atomicAdd(mbase1 + dn, __float2int_rn(ma * c.du));
            atomicAdd(mbase + dn + 1, __float2int_rn(mb * du0));
            atomicAdd(mbase1 + dn + 1, __float2int_rn(mb * c.du));
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
        const float inv_s = 1.01f * static_cast<float>(kcount[sl]) *
                            __uint_as_float(mbits[sl]) * (1.0f / 2147483648.0f);
        float* qs = q + s * vstride + gu;
        for (int32_t r = sr; r < tv; r += rstep) {
          const int32_t at = sl * slot + sc * tvp + r;
          const int32_t ex = atile[at];
          const int32_t gr = bvs[s].org_v + r;
          if (ex != 0 && static_cast<uint32_t>(gr) < static_cast<uint32_t>(gc.nv))
            unsafeAtomicAdd(qs + static_cast<int64_t>(gr) * gc.nu, static_cast<float>(ex) * inv_s);
          if (MIRROR) {
            const int32_t ey = mtile[at];
            const int32_t gm = gc.mirror_g - gr;
            if (ey != 0 && static_cast<uint32_t>(gm) < static_cast<uint32_t>(gc.nv))
              unsafeAtomicAdd(qs + static_cast<int64_t>(gm) * gc.nu,
                              static_cast<float>(ey) * inv_s);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <bool MIRROR>
__global__ __launch_bounds__(kThreads) void fp_direct_kernel(GeoConst gc, SliceRun run,
                                                             ViewBatch vb, TileShape ts,
                                                             const float* __restrict__ vol,
                                                             float* __restrict__ q,
                                                             int64_t vstride, float scale) {
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  const int32_t tid = threadIdx.x;
  const BrickCoords bc = brick_coords(gc, run, ts);
  if (tid < vb.nviews)
    bvs[tid] = brick_setup(gc, vb.view[tid], bc.i_lo, bc.i_hi, bc.j_lo, bc.j_hi, bc.kb);
  const uint32_t rot = slot_rotation();
  float x[kBrickZ], xm[kBrickZ];
  load_voxels<MIRROR>(gc, run, bc, vol, scale, rot, x, xm);
  __syncthreads();
  if (!bc.owner) return;
  for (int32_t s = 0; s < vb.nviews; ++s) {
    const ColumnF32 c = column_f64(gc, vb.view[s], bvs[s], bc.i, bc.j, bc.kb);
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
      }
    }
  }
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    p[m] = 0.0f;
}

template <typename T>
int launch_bp_t(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb, const TileShape& ts,
                const void* q, int64_t vstride, float* vol, float scale, int accumulate,
                hipStream_t st) {
  const T* qt = static_cast<const T*>(q);
  const uint64_t nwg = static_cast<uint64_t>(ts.nbx) * ts.nby * ts.nseg;
  const dim3 grid(static_cast<uint32_t>(nwg)), block(kThreads);
  if (ts.vc > 0) {
    const size_t lds = static_cast<size_t>(ts.vc) * ts.tu * ts.tvp * kTileEntryBytes;
    if (run.mirror)
      hipLaunchKernelGGL((bp_tiled_mirror_kernel<T>), grid, block, lds, st, gc, run, vb, ts,
                         qt, vstride, vol, scale, accumulate);
    else
      hipLaunchKernelGGL((bp_tiled_plain_kernel<T>), grid, block, lds, st, gc, run, vb, ts,
                         qt, vstride, vol, scale, accumulate);
  } else {
    if (run.mirror)
      hipLaunchKernelGGL((bp_direct_kernel<T, true>), grid, block, 0, st, gc, run, vb, ts,
                         qt, vstride, vol, scale, accumulate);
    else
      hipLaunchKernelGGL((bp_direct_kernel<T, false>), grid, block, 0, st, gc, run, vb, ts,
                         qt, vstride, vol, scale, accumulate);
  }
  return static_cast<int>(hipGetLastError());
}

}  // namespace

// Host-side bound of a brick's footprint (pixels) over the views of a
// launch, from derivative bounds over the whole volume: with r the x-y
// half-diagonal and zmin = d - r,
//   |du/di| <= ku Dx (|cos| + |sin| r / zmin) / zmin,
//   |du/dj| <= ku Dy (|sin| + |cos| r / zmin) / zmin,
// and v(k) - cv = kv (k - cz) / z, so over 16 slices and the brick's z
// spread dz the rows span at most kv ((16 - 1) / zmin + |k - cz| dz / zmin^2).
TileShape tile_shape(const fdk_geometry* g, const GeoConst& gc, const SliceRun& run,
                     const ViewBatch& vb) {
  TileShape ts{};
  ts.nbx = (gc.nx + kBrickX - 1) / kBrickX;
  ts.nby = (gc.ny + kBrickY - 1) / kBrickY;
  ts.nseg = (run.n + kBrickZ - 1) / kBrickZ;
  const double r = 0.5 * std::hypot((g->nx - 1) * g->dx, (g->ny - 1) * g->dy);
  const double zmin = g->sod - r, rho = r / zmin;
  const char* env = std::getenv("FDK_BP_KERNEL");
  if (env && std::strcmp(env, "direct") == 0) return ts;  // vc = 0: direct variant
  const double kmax = gc.cz + kBrickZ;
  double wu = 0.0, wv = 0.0;
  for (int32_t s = 0; s < vb.nviews; ++s) {
    // |sin| and |cos| of the view from its geometry: ci = sin Dx, cj = -cos Dy.
    const double as = std::fabs(vb.view[s].ci) / g->dx, ac = std::fabs(vb.view[s].cj) / g->dy;
    const double dui = gc.ku * g->dx * (ac + as * rho) / zmin;
    const double duj = gc.ku * g->dy * (as + ac * rho) / zmin;
    wu = std::fmax(wu, (kBrickX - 1) * dui + (kBrickY - 1) * duj);
    const double dz = (kBrickX - 1) * g->dx * as + (kBrickY - 1) * g->dy * ac;
    wv = std::fmax(wv, gc.kv * ((kBrickZ - 1) / zmin + kmax * dz / (zmin * zmin)));
  }
  // floor() of the extremes adds one pixel, the second tap one row, the
  // origin margin one pixel, FP32 column arithmetic up to one more.
  ts.tu = static_cast<int32_t>(std::ceil(wu)) + 4;
  ts.tv = static_cast<int32_t>(std::ceil(wv)) + 5;
  ts.tvp = ts.tv | 1;  // odd pitch: 16 neighbouring columns hit distinct LDS banks
  if (ts.tu + 1 > kThreads) return ts;  // staging and the adjoint's flush: a thread per column
  ts.rstep = kThreads / ts.tu;
  ts.rows = (ts.tv + ts.rstep - 1) / ts.rstep;
  const int64_t per_view = static_cast<int64_t>(ts.tu) * ts.tvp * kTileEntryBytes;
  int64_t vc = std::min<int64_t>(kMaxStageViews, kTileLdsBytes / per_view);
  vc = std::min<int64_t>(vc, kPrefetchSlots / ts.rows);
  if (const char* cap = std::getenv("FDK_BP_VC")) vc = std::min<int64_t>(vc, std::atoi(cap));
  ts.vc = static_cast<int32_t>(std::max<int64_t>(vc, 0));
  return ts;
}

int launch_backproject(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                       const TileShape& ts, const void* q, fdk_dtype q_dtype, int64_t vstride,
                       float* vol, float scale, int accumulate, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (q_dtype) {
    case FDK_F32:
      return launch_bp_t<float>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, st);
    case FDK_F16:
      return launch_bp_t<f16_t>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, st);
    case FDK_BF16:
      return launch_bp_t<bf16_t>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, st);
  }
  return static_cast<int>(hipErrorInvalidValue);
}

int launch_forward_project(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                           const TileShape& ts, const float* vol, float* q, int64_t vstride,
                           float scale, void* stream) {
  const uint64_t nwg = static_cast<uint64_t>(ts.nbx) * ts.nby * ts.nseg;
  const dim3 grid(static_cast<uint32_t>(nwg)), block(kThreads);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ts.vc > 0) {
    // Adjoint tile: one more column than the back-projection tile, float2
    // entries; it always fits where the back-projection tile does.
    TileShape tf = ts;
    const int64_t per_view = static_cast<int64_t>(ts.tu + 1) * ts.tvp * sizeof(int2);
    tf.vc = static_cast<int32_t>(std::min<int64_t>(kMaxStageViews, kTileLdsBytes / per_view));
    const size_t lds = static_cast<size_t>(tf.vc) * per_view;
    if (run.mirror)
      hipLaunchKernelGGL((fp_tiled_kernel<true>), grid, block, lds, st, gc, run, vb, tf, vol,
                         q, vstride, scale);
    else
      hipLaunchKernelGGL((fp_tiled_kernel<false>), grid, block, lds, st, gc, run, vb, tf, vol,
                         q, vstride, scale);
  } else {
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
