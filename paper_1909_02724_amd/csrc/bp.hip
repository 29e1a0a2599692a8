// Back-projection (Alg. 2 computed as Alg. 4) for gfx950.
//
// Work decomposition and coordinates: brick.h. Each thread accumulates every
// view of the launch in registers and writes each voxel once per launch;
// lanes run along x, so volume traffic is coalesced. No atomics: every voxel
// has one owner and a fixed summation order, so results are bitwise
// reproducible.
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
// Direct variant (fallback when a tile exceeds the LDS budget): the same
// arithmetic with FP64 column coordinates, taps read from global memory.
#include <hip/hip_runtime.h>

#include <cmath>

#include "brick.h"

namespace fdk {
namespace {

constexpr uint32_t kBadCol = 0x40000000u;  // pushes a buffer offset out of range
constexpr uint32_t kBadRow = 0x80000000u;
constexpr int kBufferWord3 = 0x00020000;   // raw buffer descriptor, gfx9 family
constexpr int kDppWaveShl1 = 0x130;        // DPP: lane i reads lane i + 1 of the wave

// Raw buffer load at vector offset off plus scalar (wave-uniform) offset soff.
template <typename T>
__device__ __forceinline__ uint32_t buf_load_raw(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff);
template <>
__device__ __forceinline__ uint32_t buf_load_raw<float>(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                        uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
}
template <>
__device__ __forceinline__ uint32_t buf_load_raw<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                        uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
}
template <>
__device__ __forceinline__ uint32_t buf_load_raw<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                         uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
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

template <typename T, bool MIRROR, bool TILED, bool WIDE = false>
__device__ __forceinline__ void bp_brick_body(const GeoConst& gc, const SliceRun& run,
                                              const ViewBatch& vb, const TileShape& ts,
                                              const T* __restrict__ q, int64_t vstride,
                                              float* __restrict__ vol, float scale,
                                              int accumulate, float4* tile, BrickView* bvs) {

  const int32_t tid = threadIdx.x;
  int32_t bx, by, seg;
  brick_index(ts, &bx, &by, &seg);

  const int32_t i_lo = bx * kBrickX, j_lo = by * kBrickY;
  const int32_t i_hi = min(i_lo + kBrickX - 1, gc.nx - 1);
  const int32_t j_hi = min(j_lo + kBrickY - 1, gc.ny - 1);
  // Voxel column of the thread in the brick. The mirrored tiled variant reads
  // 16-byte tile entries, which the LDS serves 16 lanes at a time: in each
  // half wave, the lanes whose quad (lane / 4) has even bit parity, then
  // those with odd parity. Each such group takes a 4 x 4 patch of columns
  // (its quads the patch's rows), so its reads span a few tile columns and,
  // with the column pitch at 7 or 9 mod 16, fall in distinct banks. A wave
  // still covers 16 x 4 columns, so the volume writes stay coalesced.
  int32_t tx0 = tid % kBrickX, ty0 = tid / kBrickX;
  if constexpr (MIRROR && TILED) {
    const int32_t lane = tid & 63, quad = (lane >> 2) & 7;
    const int32_t par = __builtin_popcount(quad) & 1;
    tx0 = 4 * (2 * (lane >> 5) + par) + (lane & 3);
    ty0 = 4 * (tid >> 6) + (quad >> 1);
  }
  const bool owner = (i_lo + tx0 <= i_hi) && (j_lo + ty0 <= j_hi);
  const int32_t i = min(i_lo + tx0, i_hi), j = min(j_lo + ty0, j_hi);
  const float txf = static_cast<float>(i - i_lo), tyf = static_cast<float>(j - j_lo);
  // Mirrored runs: 16 slices and their mirrors per thread, tile entries
  // (q, dq, qm, dqm). Plain runs: 32 slices per thread (the second 16 in the
  // registers the mirrors would use), entries (q, dq).
  constexpr int BZ = MIRROR ? kBrickZ : kPlainBrickZ;
  constexpr uint32_t kEntry = MIRROR ? kTileEntryBytes : kPlainEntryBytes;
  const int32_t t0 = seg * BZ;
  const int32_t kb = run.k_first + t0;
  const float kvf = static_cast<float>(gc.kv);

  if (tid < vb.nviews)
    bvs[tid] = brick_setup(gc, view_geo(gc, vb.sn[tid], vb.cs[tid]), i_lo, i_hi, j_lo, j_hi, kb, ts.tu, ts.tv, BZ, MIRROR);
  __syncthreads();

  float acc[kBrickZ], accm[kBrickZ];
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) acc[t] = accm[t] = 0.0f;
  // Accumulator of slice t (plain runs: t < 32); t is a constant after
  // unrolling, so this selects a register.
  auto slice_acc = [&](int t) -> float& { return t < kBrickZ ? acc[t] : accm[t - kBrickZ]; };

  if constexpr (TILED) {
    const int32_t tu = ts.tu, tv = ts.tv, tvp = ts.tvp, rstep = ts.rstep, rows = ts.rows;
    const int32_t slot_entries = tu * tvp;
    // Staging assignment: a tile row takes a group of L = 256 / rstep lanes
    // (32 or 64, never straddling a wave), lane sc of the group loading
    // pixel column org_u + sc for sc <= tu; thread -> column sc and rows
    // sr + m rstep. Each lane loads one value per row (and mirror row); the
    // next column's value, which completes the difference q(u + 1) - q(u),
    // comes from the neighbouring lane. Lanes along u: coalesced reads.
    const int32_t lanes = kBrickThreads / rstep;
    const int32_t sr = tid / lanes, sc = tid - sr * lanes;
    const bool loader = sc <= tu, stager = sc < tu;
    const uint32_t es = sizeof(T);
    const uint32_t row_es = static_cast<uint32_t>(gc.nu) * es;
    const uint32_t nrec = static_cast<uint32_t>(gc.nu) * static_cast<uint32_t>(gc.nv) * es;
    // Raw bits of q(u) for the row and (mirrored runs) its mirror row.
    constexpr int NSLOT = (MIRROR ? 1 : 2) * (WIDE ? kWidePrefetchSlots : kPrefetchSlots);
    uint2 pre[NSLOT];

    // Per-lane parts of the staging offsets, fixed for the launch: column sc
    // and first row sr relative to the tile origin, main rows downwards in
    // the buffer and mirror rows upwards. Lanes that load nothing start
    // from kBadRow, which a view's base offset and the row steps (a few MB
    // at most) keep out of range, so their loads return zero without a
    // fetch and need no select.
    const uint32_t t_main =
        loader ? static_cast<uint32_t>(sr) * row_es + static_cast<uint32_t>(sc) * es : kBadRow;
    const uint32_t t_mir =
        loader ? static_cast<uint32_t>(sc) * es - static_cast<uint32_t>(sr) * row_es : kBadRow;
    const uint32_t step = static_cast<uint32_t>(rstep) * row_es;

    // Issue the loads of views [s0, s0 + nvc) into pre[]: raw q(u) of the
    // row and of its mirror row. A thread loads rows sr + rr rstep for every
    // pass rr, also those at or beyond tv (the store drops them), so the
    // loads need no row test. Views whose tile lies on the detector skip the
    // range checks: rows past the tile may leave the detector, but their
    // offsets then fall out of the buffer's range (below zero they wrap),
    // which reads zero.
    auto load_stage = [&](int32_t s0, int32_t nvc) {
      // Uniform, but the compiler may keep it in a vector register and then
      // treat every branch on it as divergent.
      nvc = __builtin_amdgcn_readfirstlane(nvc);
      int32_t sl = 0, rr = 0;
      int32_t org_u = 0, org_v = 0, inside = 0;
      uint32_t off = 0, offm = 0;
#pragma unroll
      for (int m = 0; m < NSLOT; ++m) {
        if (sl < nvc) {
          // The descriptor is rebuilt per slot (scalar work): carried across
          // slots, the compiler moves it to vector registers and wraps each
          // load in a loop over lanes.
          const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
              const_cast<T*>(q + (s0 + sl) * vstride), 0, nrec, kBufferWord3);
          if (rr == 0) {  // uniform: new view
            const int32_t s = s0 + sl;
            org_u = __builtin_amdgcn_readfirstlane(bvs[s].org_u);
            org_v = __builtin_amdgcn_readfirstlane(bvs[s].org_v);
            inside = __builtin_amdgcn_readfirstlane(bvs[s].inside);
            off = t_main + (static_cast<uint32_t>(org_v) * row_es + static_cast<uint32_t>(org_u) * es);
            offm = t_mir + (static_cast<uint32_t>(MIRROR ? gc.mirror_g - org_v : 0) * row_es +
                            static_cast<uint32_t>(org_u) * es);
          }
          // Only the offsets depend on the branch: the loads themselves are
          // issued in common code, unconditionally (uniform control flow),
          // so nothing waits for them until the tile is written.
          uint32_t o0, m0;
          if (inside) {
            // Columns org_u .. org_u + tu are on the detector.
            const uint32_t rs = static_cast<uint32_t>(rr) * step;
            o0 = off + rs;
            m0 = offm - rs;
          } else {
            const int32_t gu = org_u + sc;
            const uint32_t c0 = loader && static_cast<uint32_t>(gu) < static_cast<uint32_t>(gc.nu)
                                    ? static_cast<uint32_t>(gu) * es : kBadCol;
            // (The uniform part is summed first: hoisted out of the stage
            // loop, per-slot lane values would be kept in spilled registers.)
            const int32_t gr = __builtin_amdgcn_readfirstlane(org_v + rr * rstep) + sr;
            const int32_t gm = MIRROR ? gc.mirror_g - gr : -1;
            const uint32_t ro = static_cast<uint32_t>(gr) < static_cast<uint32_t>(gc.nv)
                                    ? static_cast<uint32_t>(gr) * row_es : kBadRow;
            const uint32_t rm = static_cast<uint32_t>(gm) < static_cast<uint32_t>(gc.nv)
                                    ? static_cast<uint32_t>(gm) * row_es : kBadRow;
            o0 = ro + c0;
            m0 = rm + c0;
          }
          uint2 p;
          p.x = buf_load_raw<T>(rsrc, o0, 0);
          p.y = MIRROR ? buf_load_raw<T>(rsrc, m0, 0) : 0u;
          pre[m] = p;
        }
        if (++rr == rows) {
          rr = 0;
          ++sl;
        }
      }
    };

    // Tile entry (sc, sr + rr rstep) of each view. Only the last pass can
    // reach rows at or beyond tv, whose loads are discarded here. q(u + 1)
    // is the next lane's q(u) (a wave-wide shift: lane sc < tu of a group
    // always has its neighbour sc + 1 <= tu in the same group).
    const uint32_t lds_lane = static_cast<uint32_t>(sc * tvp + sr);
    const bool last_ok = stager && sr + (rows - 1) * rstep < tv;
    auto next_lane = [](float x) {
      return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kDppWaveShl1, 0xF,
                                                        0xF, false));
    };
    auto store_stage = [&](int32_t nvc) {
      nvc = __builtin_amdgcn_readfirstlane(nvc);
      int32_t sl = 0, rr = 0;
#pragma unroll
      for (int m = 0; m < NSLOT; ++m) {
        if (sl < nvc) {
          // All lanes take part in the shifts.
          const float a0 = raw_to_f32<T>(pre[m].x), a1 = next_lane(a0);
          float b0 = 0.0f, b1 = 0.0f;
          if constexpr (MIRROR) {
            b0 = raw_to_f32<T>(pre[m].y);
            b1 = next_lane(b0);
          }
          if (rr == rows - 1 ? last_ok : stager) {
            const uint32_t at = lds_lane + static_cast<uint32_t>(sl * slot_entries + rr * rstep);
            if constexpr (MIRROR) {
              tile[at] = make_float4(a0, a1 - a0, b0, b1 - b0);
            } else {
              reinterpret_cast<float2*>(tile)[at] = make_float2(a0, a1 - a0);
            }
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
                          nu * static_cast<uint32_t>(tvp) + c.nvb) * kEntry;
        asm volatile("" : "+v"(cbase));
        const char* pb = tile_bytes + cbase;
        // Reads run one voxel pair ahead of use, so LDS latency overlaps the
        // previous pair's arithmetic.
        uint32_t dn;
        float fr;
        voxel_row_off(c.fvb, c.dvk, 0, &dn, &fr);
        if constexpr (MIRROR) {
          float4 A = reinterpret_cast<const float4*>(pb + dn * kEntry)[0];
          float4 B = reinterpret_cast<const float4*>(pb + dn * kEntry)[1];
#pragma unroll
          for (int t = 0; t < kBrickZ; ++t) {
            float4 An = A, Bn = B;
            uint32_t dn1 = 0;
            float fr1 = 0.0f;
            if (t + 1 < kBrickZ) {
              voxel_row_off(c.fvb, c.dvk, t + 1, &dn1, &fr1);
              const float4* p = reinterpret_cast<const float4*>(pb + dn1 * kEntry);
              An = p[0];
              Bn = p[1];
            }
            const float ta = fmaf(c.du, A.y, A.x), tb = fmaf(c.du, B.y, B.x);
            acc[t] = fmaf(c.w, fmaf(fr, tb - ta, ta), acc[t]);
            const float ma = fmaf(c.du, A.w, A.z), mb = fmaf(c.du, B.w, B.z);
            accm[t] = fmaf(c.w, fmaf(fr, mb - ma, ma), accm[t]);
            A = An;
            B = Bn;
            fr = fr1;
          }
        } else {
          // Rows n and n + 1 are adjacent 8-byte entries: one read2.
          float2 A = reinterpret_cast<const float2*>(pb + dn * kEntry)[0];
          float2 B = reinterpret_cast<const float2*>(pb + dn * kEntry)[1];
#pragma unroll
          for (int t = 0; t < BZ; ++t) {
            float2 An = A, Bn = B;
            uint32_t dn1 = 0;
            float fr1 = 0.0f;
            if (t + 1 < BZ) {
              voxel_row_off(c.fvb, c.dvk, t + 1, &dn1, &fr1);
              const float2* p = reinterpret_cast<const float2*>(pb + dn1 * kEntry);
              An = p[0];
              Bn = p[1];
            }
            const float ta = fmaf(c.du, A.y, A.x), tb = fmaf(c.du, B.y, B.x);
            slice_acc(t) = fmaf(c.w, fmaf(fr, tb - ta, ta), slice_acc(t));
            A = An;
            B = Bn;
            fr = fr1;
          }
        }
      }
    }
  } else {
    for (int32_t s = 0; s < vb.nviews; ++s) {
      const ColumnF32 c = column_f64(gc, view_geo(gc, vb.sn[s], vb.cs[s]), bvs[s], i, j, kb);
      const T* qs = q + s * vstride;
      const int32_t a = bvs[s].org_u + static_cast<int32_t>(c.nu);
      const int32_t nb = bvs[s].org_v + static_cast<int32_t>(c.nvb);
#pragma unroll
      for (int t = 0; t < BZ; ++t) {
        uint32_t dn;
        float fr;
        voxel_row_off(c.fvb, c.dvk, t, &dn, &fr);
        const int32_t n = nb + static_cast<int32_t>(dn);
        const float q0a = tap(qs, gc.nu, gc.nv, a, n), q1a = tap(qs, gc.nu, gc.nv, a + 1, n);
        const float q0b = tap(qs, gc.nu, gc.nv, a, n + 1), q1b = tap(qs, gc.nu, gc.nv, a + 1, n + 1);
        const float ta = fmaf(c.du, q1a - q0a, q0a), tb = fmaf(c.du, q1b - q0b, q0b);
        slice_acc(t) = fmaf(c.w, fmaf(fr, tb - ta, ta), slice_acc(t));
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
  float* const lo = vol + static_cast<int64_t>(run.loc_lo + t0) * slice + col;
  float* const hi = vol + static_cast<int64_t>(run.loc_hi - t0) * slice + col;
  const int32_t nt = min(BZ, run.n - t0);  // slices of the brick in the run
  // All old values are read before the first store: interleaved, each read
  // would wait out a full memory round trip, since the compiler cannot tell
  // that a store does not alias the next read. (Written this way, with the
  // reads selected rather than guarded, the plain variant also keeps its
  // accumulators out of scratch inside the view loop.)
  float old[BZ], oldm[kBrickZ];
#pragma unroll
  for (int t = 0; t < BZ; ++t) {
    old[t] = (accumulate && t < nt) ? lo[static_cast<int64_t>(t) * slice] : 0.0f;
    if (t < kBrickZ)
      oldm[t] = (MIRROR && accumulate && t < nt) ? hi[-static_cast<int64_t>(t) * slice] : 0.0f;
  }
#pragma unroll
  for (int t = 0; t < BZ; ++t) {
    if (t < nt) {
      lo[static_cast<int64_t>(t) * slice] = fmaf(scale, slice_acc(t), old[t]);
      if (MIRROR) hi[-static_cast<int64_t>(t) * slice] = fmaf(scale, accm[t], oldm[t]);
    }
  }
}

// The tiled variants run five 256-thread workgroups per CU (five waves per
// SIMD): tiles within 27.5 KB, 102 VGPRs. Tiles that need more staging passes
// per view than their prefetch slots allow run the WIDE instances: four
// workgroups per CU, 35.5 KB, 128 VGPRs and kWidePrefetchSlots slots.
template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 5)))
void bp_tiled_mirror_kernel(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                            const T* __restrict__ q, int64_t vstride, float* __restrict__ vol,
                            float scale, int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, true, true>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, tile, bvs);
}

template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
void bp_tiled_mirror_wide_kernel(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                                 const T* __restrict__ q, int64_t vstride,
                                 float* __restrict__ vol, float scale, int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, true, true, true>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, tile,
                                     bvs);
}

template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 5)))
void bp_tiled_plain_kernel(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                           const T* __restrict__ q, int64_t vstride, float* __restrict__ vol,
                           float scale, int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, false, true>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, tile, bvs);
}

template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
void bp_tiled_plain_wide_kernel(GeoConst gc, SliceRun run, ViewBatch vb, TileShape ts,
                                const T* __restrict__ q, int64_t vstride,
                                float* __restrict__ vol, float scale, int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ BrickView bvs[kMaxViewsPerLaunch];
  bp_brick_body<T, false, true, true>(gc, run, vb, ts, q, vstride, vol, scale, accumulate, tile,
                                      bvs);
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

template <typename T>
int launch_bp_t(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb, const TileShape& ts,
                const void* q, int64_t vstride, float* vol, float scale, int accumulate,
                hipStream_t st) {
  const T* qt = static_cast<const T*>(q);
  const uint64_t nwg = static_cast<uint64_t>(ts.nbx) * ts.nby * ts.nseg;
  const dim3 grid(static_cast<uint32_t>(nwg)), block(kThreads);
  if (ts.vc > 0) {
    const size_t lds = static_cast<size_t>(ts.vc) * ts.tu * ts.tvp *
                       (run.mirror ? kTileEntryBytes : kPlainEntryBytes);
    if (run.mirror && ts.wide)
      hipLaunchKernelGGL((bp_tiled_mirror_wide_kernel<T>), grid, block, lds, st, gc, run, vb, ts,
                         qt, vstride, vol, scale, accumulate);
    else if (run.mirror)
      hipLaunchKernelGGL((bp_tiled_mirror_kernel<T>), grid, block, lds, st, gc, run, vb, ts,
                         qt, vstride, vol, scale, accumulate);
    else if (ts.wide)
      hipLaunchKernelGGL((bp_tiled_plain_wide_kernel<T>), grid, block, lds, st, gc, run, vb, ts,
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

}  // namespace fdk
