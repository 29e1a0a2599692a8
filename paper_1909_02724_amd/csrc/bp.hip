// Back-projection (Alg. 2 computed as Alg. 4) and its exact adjoint for
// gfx950.
//
// Tiled kernel (the main path). A workgroup of 256 threads owns a brick of
// 16 x 16 (x, y) columns and 16 consecutive slices of a slice run; for a
// mirrored run (Theorem 1) every thread also owns the 16 mirror voxels of
// its column. For each view the brick's detector footprint is staged into
// LDS as a tile whose rows hold, for pixel (u, v), the value q(u, v), the
// forward difference q(u+1, v) - q(u, v), and the same pair for the mirror
// row G - v. With the mirror rows stored in reverse order, a voxel and its
// mirror read the same tile offsets with the same weights, so one row
// index, one fraction and one address serve the pair; the u-interpolation
// is a single FMA on the staged difference (Theorem 2: u, hence the
// fraction du, is fixed along the column). Each thread accumulates all
// views of the launch in registers and writes every voxel once per launch;
// lanes run along x, so volume traffic is coalesced. No atomics: every
// voxel has one owner and a fixed summation order.
//
// Direct kernel (fallback when a footprint tile exceeds the LDS budget):
// the same per-column arithmetic with taps read straight from global
// memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>

#include "geom_device.h"

namespace fdk {
namespace {

constexpr int kThreads = kBrickX * kBrickY;
constexpr int kBlockX = 64;  // direct kernels: 64 x 4 columns per workgroup
constexpr int kBlockY = 4;
constexpr int kZT = 8;

template <typename T>
__device__ __forceinline__ float tap(const T* __restrict__ qs, int32_t nu, int32_t nv, int32_t a,
                                     int32_t b) {
  // Taps outside the detector read zero.
  return (static_cast<uint32_t>(a) < static_cast<uint32_t>(nu) &&
          static_cast<uint32_t>(b) < static_cast<uint32_t>(nv))
             ? to_f32(qs[static_cast<int64_t>(b) * nu + a])
             : 0.0f;
}

// ------------------------------------------------------------------------
// Tiled back-projection.
// ------------------------------------------------------------------------

// u and v(k) of column (i, j) in view g, FP64 (Eq. 2 in the Alg. 4 form).
__device__ __forceinline__ void column_uv(const GeoConst& gc, const ViewGeo& g, int32_t i,
                                          int32_t j, int32_t k, double* u, double* v,
                                          double* f) {
  const double di = static_cast<double>(i), dj = static_cast<double>(j);
  const double z = fma(g.ci, di, fma(g.cj, dj, g.c0));
  *f = 1.0 / z;
  const double a = fma(g.ai, di, fma(g.aj, dj, g.a0));
  *u = fma(gc.ku * a, *f, gc.cu);
  *v = fma(gc.kv * (static_cast<double>(k) - gc.cz), *f, gc.cv);
}

template <typename T, bool MIRROR>
__global__ __launch_bounds__(kThreads) void bp_tiled_kernel(GeoConst gc, SliceRun run,
                                                            ViewBatch vb, TileShape ts,
                                                            const T* __restrict__ q,
                                                            int64_t vstride,
                                                            float* __restrict__ vol, float scale,
                                                            int accumulate) {
  extern __shared__ float4 tile[];
  __shared__ int32_t org_u[kMaxViewsPerLaunch];
  __shared__ int32_t org_v[kMaxViewsPerLaunch];

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
  const int32_t tx = tid % kBrickX, ty = tid / kBrickX;
  const bool owner = (i_lo + tx <= i_hi) && (j_lo + ty <= j_hi);
  const int32_t i = min(i_lo + tx, i_hi), j = min(j_lo + ty, j_hi);
  const int32_t t0 = seg * kBrickZ;
  const int32_t kb = run.k_first + t0;

  // Tile origin per view: u and v are extremal at the corners of the
  // brick's (i, j, k) box (z is affine in i, j; u is a ratio of affine
  // functions; v is affine in k at fixed f), so 8 corner evaluations bound
  // every tap; one pixel of margin absorbs rounding.
  if (tid < vb.nviews * 8) {
    const int32_t s = tid >> 3, c = tid & 7;
    double u, v, f;
    column_uv(gc, vb.view[s], (c & 1) ? i_hi : i_lo, (c & 2) ? j_hi : j_lo,
              (c & 4) ? kb + kBrickZ - 1 : kb, &u, &v, &f);
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
      u = fmin(u, __shfl_xor(u, m, 8));
      v = fmin(v, __shfl_xor(v, m, 8));
    }
    if (c == 0) {
      org_u[s] = static_cast<int32_t>(floor(u)) - 1;
      org_v[s] = static_cast<int32_t>(floor(v)) - 1;
    }
  }
  __syncthreads();

  float acc[kBrickZ], accm[kBrickZ];
#pragma unroll
  for (int t = 0; t < kBrickZ; ++t) acc[t] = accm[t] = 0.0f;

  const int32_t tu = ts.tu, tv = ts.tv, tuv = ts.tu * ts.tv;
  const uint32_t row_bytes = static_cast<uint32_t>(tu) * kTileEntryBytes;
  const char* tile_bytes = reinterpret_cast<const char*>(tile);
  // Staging assignment, fixed for the kernel: thread -> tile column sc and
  // first row sr; rows advance by rstep (threads beyond rstep * tu idle).
  const int32_t rstep = kThreads / tu;
  const int32_t sr = tid / tu, sc = tid - sr * tu;
  const bool stager = sr < rstep;
  for (int32_t s0 = 0; s0 < vb.nviews; s0 += ts.vc) {
    const int32_t nvc = min(ts.vc, vb.nviews - s0);
    if (s0 > 0) __syncthreads();  // the previous views' tiles are consumed
    // Stage: entry (r, c) of view slot sl holds pixel (org_u + c, org_v + r)
    // and its u-difference; for mirrored runs also pixel (org_u + c,
    // G - org_v - r), the mirror row in reverse order.
    if (stager) {
      for (int32_t sl = 0; sl < nvc; ++sl) {
        const int32_t s = s0 + sl;
        const T* qs = q + s * vstride;
        const int32_t gu = org_u[s] + sc;
        float4* trow = tile + sl * tuv + sc;
        for (int32_t r = sr; r < tv; r += rstep) {
          const int32_t gr = org_v[s] + r;
          float4 ent;
          const float a0 = tap(qs, gc.nu, gc.nv, gu, gr), a1 = tap(qs, gc.nu, gc.nv, gu + 1, gr);
          ent.x = a0;
          ent.y = a1 - a0;
          if (MIRROR) {
            const int32_t gm = gc.mirror_g - gr;
            const float b0 = tap(qs, gc.nu, gc.nv, gu, gm), b1 = tap(qs, gc.nu, gc.nv, gu + 1, gm);
            ent.z = b0;
            ent.w = b1 - b0;
          } else {
            ent.z = ent.w = 0.0f;
          }
          trow[r * tu] = ent;
        }
      }
    }
    __syncthreads();

    for (int32_t sl = 0; sl < nvc; ++sl) {
      const int32_t s = s0 + sl;
      double u, v, f;
      column_uv(gc, vb.view[s], i, j, kb, &u, &v, &f);
      const double ul = u - org_u[s], vl = v - org_v[s];  // exact: integer shifts
      const double fu = floor(ul), fv = floor(vl);
      const int32_t nu = static_cast<int32_t>(fu), nvb = static_cast<int32_t>(fv);
      const float du = static_cast<float>(ul - fu);
      const float fvb = static_cast<float>(vl - fv);
      const float w = static_cast<float>(f * f);
      const float dvk = static_cast<float>(gc.kv * f);
      // LDS byte offsets: entry (row, col) of slot sl at
      // ((sl * tv + row) * tu + col) * 16; rows advance by row_bytes.
      const uint32_t base = (static_cast<uint32_t>(sl * tuv + nvb * tu + nu)) * kTileEntryBytes;
#pragma unroll
      for (int t = 0; t < kBrickZ; ++t) {
        uint32_t dn;
        float fr;
        voxel_row_off(fvb, dvk, t, &dn, &fr);
        const uint32_t off = __umul24(dn, row_bytes) + base;
        const float4 A = *reinterpret_cast<const float4*>(tile_bytes + off);
        const float4 B = *reinterpret_cast<const float4*>(tile_bytes + off + row_bytes);
        const float ta = fmaf(du, A.y, A.x), tb = fmaf(du, B.y, B.x);
        acc[t] = fmaf(w, fmaf(fr, tb - ta, ta), acc[t]);
        if (MIRROR) {
          const float ma = fmaf(du, A.w, A.z), mb = fmaf(du, B.w, B.z);
          accm[t] = fmaf(w, fmaf(fr, mb - ma, ma), accm[t]);
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

// ------------------------------------------------------------------------
// Direct back-projection (fallback) and the adjoint.
// ------------------------------------------------------------------------

// Alg. 3 on rows ra (weight 1 - fr) and rb (weight fr), columns a, a + 1.
template <typename T>
__device__ __forceinline__ float bilinear(const T* __restrict__ qs, int32_t nu, int32_t nv,
                                          int32_t a, float du, int32_t ra, int32_t rb, float fr) {
  const float q0a = tap(qs, nu, nv, a, ra), q1a = tap(qs, nu, nv, a + 1, ra);
  const float q0b = tap(qs, nu, nv, a, rb), q1b = tap(qs, nu, nv, a + 1, rb);
  const float ta = fmaf(du, q1a - q0a, q0a);
  const float tb = fmaf(du, q1b - q0b, q0b);
  return fmaf(fr, tb - ta, ta);
}

template <typename T, bool MIRROR>
__global__ __launch_bounds__(kBlockX* kBlockY) void bp_direct_kernel(GeoConst gc, SliceRun run,
                                                                     ViewBatch vb,
                                                                     const T* __restrict__ q,
                                                                     int64_t vstride,
                                                                     float* __restrict__ vol,
                                                                     float scale, int accumulate) {
  const int32_t i = blockIdx.x * kBlockX + threadIdx.x;
  const int32_t j = blockIdx.y * kBlockY + threadIdx.y;
  const int32_t t0 = blockIdx.z * kZT;
  if (i >= gc.nx || j >= gc.ny) return;
  const int32_t kb = run.k_first + t0;
  float acc[kZT], accm[kZT];
#pragma unroll
  for (int t = 0; t < kZT; ++t) acc[t] = accm[t] = 0.0f;

  for (int32_t s = 0; s < vb.nviews; ++s) {
    const ColumnView c = column_view(gc, vb.view[s], i, j, kb);
    const T* qs = q + s * vstride;
#pragma unroll
    for (int t = 0; t < kZT; ++t) {
      int32_t n;
      float fr;
      voxel_row(c, t, &n, &fr);
      acc[t] = fmaf(c.w, bilinear(qs, gc.nu, gc.nv, c.nu0, c.du, n, n + 1, fr), acc[t]);
      if (MIRROR) {
        // Theorem 1: v(Nz-1-k) = G - v(k), so the mirror voxel samples rows
        // G - n (weight 1 - fr) and G - 1 - n (weight fr).
        const int32_t m = gc.mirror_g - n;
        accm[t] = fmaf(c.w, bilinear(qs, gc.nu, gc.nv, c.nu0, c.du, m, m - 1, fr), accm[t]);
      }
    }
  }

  const int64_t slice = static_cast<int64_t>(gc.nx) * gc.ny;
  const int64_t col = static_cast<int64_t>(j) * gc.nx + i;
#pragma unroll
  for (int t = 0; t < kZT; ++t) {
    if (t0 + t >= run.n) break;
    float* p = vol + static_cast<int64_t>(run.loc_lo + t0 + t) * slice + col;
    *p = accumulate ? fmaf(scale, acc[t], *p) : scale * acc[t];
    if (MIRROR) {
      float* pm = vol + static_cast<int64_t>(run.loc_hi - t0 - t) * slice + col;
      *pm = accumulate ? fmaf(scale, accm[t], *pm) : scale * accm[t];
    }
  }
}

// Adjoint: every voxel scatters scale * W * w_tap * vol into its taps with
// the coordinates and weights the back-projectors sample with.
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

template <bool MIRROR>
__global__ __launch_bounds__(kBlockX* kBlockY) void fp_kernel(GeoConst gc, SliceRun run,
                                                              ViewBatch vb,
                                                              const float* __restrict__ vol,
                                                              float* __restrict__ q,
                                                              int64_t vstride, float scale) {
  const int32_t i = blockIdx.x * kBlockX + threadIdx.x;
  const int32_t j = blockIdx.y * kBlockY + threadIdx.y;
  const int32_t t0 = blockIdx.z * kZT;
  if (i >= gc.nx || j >= gc.ny) return;
  const int32_t kb = run.k_first + t0;
  const int64_t slice = static_cast<int64_t>(gc.nx) * gc.ny;
  const int64_t col = static_cast<int64_t>(j) * gc.nx + i;
  float x[kZT], xm[kZT];
#pragma unroll
  for (int t = 0; t < kZT; ++t) {
    const bool in = t0 + t < run.n;
    x[t] = in ? scale * vol[static_cast<int64_t>(run.loc_lo + t0 + t) * slice + col] : 0.0f;
    xm[t] = (MIRROR && in) ? scale * vol[static_cast<int64_t>(run.loc_hi - t0 - t) * slice + col]
                           : 0.0f;
  }
  for (int32_t s = 0; s < vb.nviews; ++s) {
    const ColumnView c = column_view(gc, vb.view[s], i, j, kb);
    float* qs = q + s * vstride;
#pragma unroll
    for (int t = 0; t < kZT; ++t) {
      if (t0 + t >= run.n) break;
      int32_t n;
      float fr;
      voxel_row(c, t, &n, &fr);
      splat(qs, gc.nu, gc.nv, c.nu0, c.du, n, n + 1, fr, c.w * x[t]);
      if (MIRROR) {
        const int32_t m = gc.mirror_g - n;
        splat(qs, gc.nu, gc.nv, c.nu0, c.du, m, m - 1, fr, c.w * xm[t]);
      }
    }
  }
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    p[m] = 0.0f;
}

dim3 column_grid(const GeoConst& gc, const SliceRun& run) {
  return dim3((gc.nx + kBlockX - 1) / kBlockX, (gc.ny + kBlockY - 1) / kBlockY,
              (run.n + kZT - 1) / kZT);
}

template <typename T>
int launch_bp_t(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb, const TileShape& ts,
                const void* q, int64_t vstride, float* vol, float scale, int accumulate,
                hipStream_t st) {
  const T* qt = static_cast<const T*>(q);
  if (ts.vc > 0) {
    const uint64_t nwg = static_cast<uint64_t>(ts.nbx) * ts.nby * ts.nseg;
    const size_t lds = static_cast<size_t>(ts.vc) * ts.tu * ts.tv * kTileEntryBytes;
    if (run.mirror)
      hipLaunchKernelGGL((bp_tiled_kernel<T, true>), dim3(static_cast<uint32_t>(nwg)),
                         dim3(kThreads), lds, st, gc, run, vb, ts, qt, vstride, vol, scale,
                         accumulate);
    else
      hipLaunchKernelGGL((bp_tiled_kernel<T, false>), dim3(static_cast<uint32_t>(nwg)),
                         dim3(kThreads), lds, st, gc, run, vb, ts, qt, vstride, vol, scale,
                         accumulate);
    return static_cast<int>(hipGetLastError());
  }
  const dim3 grid = column_grid(gc, run), block(kBlockX, kBlockY);
  if (run.mirror)
    hipLaunchKernelGGL((bp_direct_kernel<T, true>), grid, block, 0, st, gc, run, vb, qt, vstride,
                       vol, scale, accumulate);
  else
    hipLaunchKernelGGL((bp_direct_kernel<T, false>), grid, block, 0, st, gc, run, vb, qt,
                       vstride, vol, scale, accumulate);
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
  const char* env = std::getenv("FDK_BP_KERNEL");
  if (env && std::strcmp(env, "direct") == 0) return ts;  // vc = 0: direct kernel
  const double r = 0.5 * std::hypot((g->nx - 1) * g->dx, (g->ny - 1) * g->dy);
  const double zmin = g->sod - r, rho = r / zmin;
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
  // origin margin one pixel, and one more absorbs rounding.
  ts.tu = static_cast<int32_t>(std::ceil(wu)) + 3;
  ts.tv = static_cast<int32_t>(std::ceil(wv)) + 4;
  const int64_t per_view = static_cast<int64_t>(ts.tu) * ts.tv * kTileEntryBytes;
  ts.vc = static_cast<int32_t>(std::min<int64_t>(kMaxStageViews, kTileLdsBytes / per_view));
  if (ts.tu > kThreads) ts.vc = 0;  // staging maps one thread per tile column
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
                           const float* vol, float* q, int64_t vstride, float scale,
                           void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid = column_grid(gc, run), block(kBlockX, kBlockY);
  if (run.mirror)
    hipLaunchKernelGGL((fp_kernel<true>), grid, block, 0, st, gc, run, vb, vol, q, vstride, scale);
  else
    hipLaunchKernelGGL((fp_kernel<false>), grid, block, 0, st, gc, run, vb, vol, q, vstride,
                       scale);
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
