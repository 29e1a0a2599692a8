// Element-wise kernels of the iterative methods built on the matched pair
// (back-projection B and its transpose F): SIRT's inverse row and column
// sums of F and its fused residual and update steps, and MLEM's guarded
// ratio and multiplicative update. Memory-bound grid-stride loops over
// contiguous FP32 arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "ops_internal.h"

namespace fdk {
namespace {

constexpr int kEwThreads = 256;
constexpr int64_t kEwMaxBlocks = 65536;

__global__ void fill_kernel(float* __restrict__ p, int64_t n, float v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    p[m] = v;
}

// Largest value of p[0, n) per block, as non-negative float bits (sums of
// non-negative weights): out must start at 0.
__global__ void max_kernel(const float* __restrict__ p, int64_t n, uint32_t* __restrict__ out) {
  __shared__ float red[kEwThreads];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  float m = 0.0f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    m = fmaxf(m, p[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kEwThreads / 2; w > 0; w /= 2) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

// p <- 1 / max(p, floor_rel * max(p)).
__global__ void invert_kernel(float* __restrict__ p, int64_t n, const uint32_t* __restrict__ maxbits,
                              float floor_rel) {
  const float lo = floor_rel * __uint_as_float(*maxbits);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    p[m] = lo > 0.0f ? 1.0f / fmaxf(p[m], lo) : 0.0f;
}

// r <- row_inv * (p - r), r holding F x on entry.
__global__ void residual_kernel(const float* __restrict__ p, const float* __restrict__ row_inv,
                                float* __restrict__ r, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    r[m] = row_inv[m] * (p[m] - r[m]);
}

// x <- x + lambda * col_inv * b, optionally clamped at zero.
__global__ void update_kernel(float* __restrict__ x, const float* __restrict__ col_inv,
                              const float* __restrict__ b, int64_t n, float lambda, int nonneg) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride) {
    const float v = fmaf(lambda * col_inv[m], b[m], x[m]);
    x[m] = nonneg ? fmaxf(v, 0.0f) : v;
  }
}

// MLEM ratio: r <- p / max(r, floor_rel * max(r)), and 0 where that
// denominator is 0; r holds F x on entry.
__global__ void mlem_ratio_kernel(const float* __restrict__ p, float* __restrict__ r, int64_t n,
                                  const uint32_t* __restrict__ maxbits, float floor_rel) {
  const float lo = floor_rel * __uint_as_float(*maxbits);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride) {
    const float den = fmaxf(r[m], lo);
    r[m] = den > 0.0f ? p[m] / den : 0.0f;
  }
}

// MLEM update: x <- x * col_inv * b.
__global__ void mlem_update_kernel(float* __restrict__ x, const float* __restrict__ col_inv,
                                   const float* __restrict__ b, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += stride)
    x[m] = x[m] * (col_inv[m] * b[m]);
}

dim3 ew_grid(int64_t n) {
  return dim3(static_cast<uint32_t>(std::min<int64_t>((n + kEwThreads - 1) / kEwThreads, kEwMaxBlocks)));
}

}  // namespace

int launch_fill(float* p, int64_t n, float v, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_kernel, ew_grid(n), dim3(kEwThreads), 0, static_cast<hipStream_t>(stream),
                     p, n, v);
  return static_cast<int>(hipGetLastError());
}

int launch_invert_floor(float* p, int64_t n, float floor_rel, uint32_t* maxbits, void* stream) {
  if (n <= 0) return 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(kEwThreads), 0, st,
                     reinterpret_cast<float*>(maxbits), int64_t{1}, 0.0f);
  hipLaunchKernelGGL(max_kernel, ew_grid(n), dim3(kEwThreads), 0, st, p, n, maxbits);
  hipLaunchKernelGGL(invert_kernel, ew_grid(n), dim3(kEwThreads), 0, st, p, n, maxbits, floor_rel);
  return static_cast<int>(hipGetLastError());
}

int launch_sirt_residual(const float* p, const float* row_inv, float* r, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(residual_kernel, ew_grid(n), dim3(kEwThreads), 0,
                     static_cast<hipStream_t>(stream), p, row_inv, r, n);
  return static_cast<int>(hipGetLastError());
}

int launch_sirt_update(float* x, const float* col_inv, const float* b, int64_t n, float lambda,
                       int nonneg, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(update_kernel, ew_grid(n), dim3(kEwThreads), 0,
                     static_cast<hipStream_t>(stream), x, col_inv, b, n, lambda, nonneg);
  return static_cast<int>(hipGetLastError());
}

int launch_mlem_ratio(const float* p, float* r, int64_t n, float floor_rel, uint32_t* maxbits,
                      void* stream) {
  if (n <= 0) return 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(kEwThreads), 0, st,
                     reinterpret_cast<float*>(maxbits), int64_t{1}, 0.0f);
  hipLaunchKernelGGL(max_kernel, ew_grid(n), dim3(kEwThreads), 0, st, r, n, maxbits);
  hipLaunchKernelGGL(mlem_ratio_kernel, ew_grid(n), dim3(kEwThreads), 0, st, p, r, n, maxbits,
                     floor_rel);
  return static_cast<int>(hipGetLastError());
}

// Workspace of the entry points that allocate nothing: one array per GPU,
// held from the library's load until the process ends. Host code never
// uses the array's name as an address (on the host it is only a stand-in):
// the device address comes from hipGetSymbolAddress, once per device, with
// that device current.
static __device__ __align__(256) float scratch[kStaticScratchFloats];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

int static_scratch(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return static_cast<int>(e);
  if (dev < 0 || dev >= kMaxScratchDevices) return static_cast<int>(hipErrorInvalidDevice);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return static_cast<int>(e);
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<float*>(g_scratch_ptr[dev]);
  return 0;
}

int launch_mlem_update(float* x, const float* col_inv, const float* b, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(mlem_update_kernel, ew_grid(n), dim3(kEwThreads), 0,
                     static_cast<hipStream_t>(stream), x, col_inv, b, n);
  return static_cast<int>(hipGetLastError());
}

}  // namespace fdk
