// Back-projection (Alg. 2 computed as Alg. 4) and its exact adjoint for
// gfx950. One thread owns one (x, y) column segment of ZT voxels (and, for
// mirrored runs, their ZT mirror voxels: Theorem 1), accumulates every view
// of the launch in registers and writes each voxel once per launch. Lanes
// run along x, so volume reads and writes are coalesced.
#include <hip/hip_runtime.h>

#include "geom_device.h"

namespace fdk {
namespace {

constexpr int kBlockX = 64;
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
__global__ __launch_bounds__(kBlockX* kBlockY) void bp_kernel(GeoConst gc, SliceRun run,
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
// the coordinates and weights bp_kernel samples with.
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
int launch_bp_t(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb, const void* q,
                int64_t vstride, float* vol, float scale, int accumulate, hipStream_t st) {
  const dim3 grid = column_grid(gc, run), block(kBlockX, kBlockY);
  const T* qt = static_cast<const T*>(q);
  if (run.mirror)
    hipLaunchKernelGGL((bp_kernel<T, true>), grid, block, 0, st, gc, run, vb, qt, vstride, vol,
                       scale, accumulate);
  else
    hipLaunchKernelGGL((bp_kernel<T, false>), grid, block, 0, st, gc, run, vb, qt, vstride, vol,
                       scale, accumulate);
  return static_cast<int>(hipGetLastError());
}

}  // namespace

int launch_backproject(const GeoConst& gc, const SliceRun& run, const ViewBatch& vb,
                       const void* q, fdk_dtype q_dtype, int64_t vstride, float* vol,
                       float scale, int accumulate, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (q_dtype) {
    case FDK_F32:
      return launch_bp_t<float>(gc, run, vb, q, vstride, vol, scale, accumulate, st);
    case FDK_F16:
      return launch_bp_t<f16_t>(gc, run, vb, q, vstride, vol, scale, accumulate, st);
    case FDK_BF16:
      return launch_bp_t<bf16_t>(gc, run, vb, q, vstride, vol, scale, accumulate, st);
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
