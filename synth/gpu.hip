// GPU-side synthetic input generators (test and benchmark infrastructure,
// not part of the reconstruction library):
//  - synth_hash_fill: SplitMix64 counter-based values (Steele, Lea and Flood,
//    OOPSLA 2014) on the grid 2^-23 in [-1, 1), stored as FP32 / FP16 /
//    BF16 with round-to-nearest-even; the CPU oracle regenerates the same
//    values from its own implementation of the published generator.
//  - synth_phantom_project: analytic line integrals of a sum of ellipsoids
//    along the ray from the source to every detector pixel centre (FP64).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float uniform_pm1(uint64_t seed, uint64_t counter) {
  const int32_t m = static_cast<int32_t>(splitmix64(seed, counter) >> 40) - 8388608;
  return static_cast<float>(m) * 0x1p-23f;  // exact: |m| < 2^24
}

__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

__global__ void hash_fill_kernel(uint64_t seed, uint64_t counter0, int64_t n, void* out,
                                 int dtype) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < n;
       m += stride) {
    const float x = uniform_pm1(seed, counter0 + static_cast<uint64_t>(m));
    if (dtype == 0)
      static_cast<float*>(out)[m] = x;
    else if (dtype == 1)
      static_cast<uint16_t*>(out)[m] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
    else
      static_cast<uint16_t*>(out)[m] = to_bf16_rne(x);
  }
}

struct ScanGeom {
  int32_t nu, nv;
  double du, dv, cu, cv, sod, sdd;
};

// Ellipsoid record: centre (3), semi-axes (3), rotation (3x3 row-major,
// columns are the axes in world coordinates), density.
__global__ void phantom_project_kernel(ScanGeom g, const double* __restrict__ angles,
                                       int32_t nviews, const double* __restrict__ ell,
                                       int32_t nell, float* __restrict__ out) {
  const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t b = blockIdx.y;
  const int32_t s = blockIdx.z;
  if (a >= g.nu || b >= g.nv || s >= nviews) return;
  const double beta = angles[s];
  const double cb = cos(beta), sb = sin(beta);
  // Source at the gantry origin; pixel (a, b) on the plane at distance D.
  const double src[3] = {-g.sod * sb, -g.sod * cb, 0.0};
  const double xr = (a - g.cu) * g.du, yr = g.sdd - g.sod, zr = -(b - g.cv) * g.dv;
  const double pix[3] = {cb * xr + sb * yr, -sb * xr + cb * yr, zr};
  const double dir[3] = {pix[0] - src[0], pix[1] - src[1], pix[2] - src[2]};
  const double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  double acc = 0.0;
  for (int32_t n = 0; n < nell; ++n) {
    const double* e = ell + 16 * n;
    const double* R = e + 6;
    double o[3], w[3];
    const double p[3] = {src[0] - e[0], src[1] - e[1], src[2] - e[2]};
    for (int m = 0; m < 3; ++m) {
      o[m] = (R[m] * p[0] + R[3 + m] * p[1] + R[6 + m] * p[2]) / e[3 + m];
      w[m] = (R[m] * dir[0] + R[3 + m] * dir[1] + R[6 + m] * dir[2]) / e[3 + m];
    }
    const double A = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double B = o[0] * w[0] + o[1] * w[1] + o[2] * w[2];
    const double Cc = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - 1.0;
    const double disc = B * B - A * Cc;
    if (disc > 0.0) acc += e[15] * (2.0 * sqrt(disc) / A) * len;
  }
  out[(static_cast<int64_t>(s) * g.nv + b) * g.nu + a] = static_cast<float>(acc);
}

}  // namespace

extern "C" {

// out: device array of n values, dtype 0 FP32, 1 FP16, 2 BF16.
int synth_hash_fill(uint64_t seed, uint64_t counter0, int64_t n, void* out, int dtype,
                    void* stream) {
  if (n <= 0) return 0;
  if (!out || dtype < 0 || dtype > 2) return static_cast<int>(hipErrorInvalidValue);
  const int64_t blocks = (n + 255) / 256 < 262144 ? (n + 255) / 256 : 262144;
  hipLaunchKernelGGL(hash_fill_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), seed, counter0, n, out, dtype);
  return static_cast<int>(hipGetLastError());
}

// angles: device FP64 [nviews]; ell: device FP64 [nell * 16]; out: device
// FP32 (nviews, nv, nu).
int synth_phantom_project(int32_t nu, int32_t nv, double du, double dv, double off_u,
                          double off_v, double sod, double sdd, const double* angles,
                          int32_t nviews, const double* ell, int32_t nell, float* out,
                          void* stream) {
  if (nu <= 0 || nv <= 0 || nviews <= 0 || nell < 0 || !angles || !out || (nell && !ell))
    return static_cast<int>(hipErrorInvalidValue);
  ScanGeom g{nu, nv, du, dv, 0.5 * (nu - 1) + off_u, 0.5 * (nv - 1) + off_v, sod, sdd};
  dim3 grid((nu + 63) / 64, nv, nviews);
  hipLaunchKernelGGL(phantom_project_kernel, grid, dim3(64), 0, static_cast<hipStream_t>(stream),
                     g, angles, nviews, ell, nell, out);
  return static_cast<int>(hipGetLastError());
}

}  // extern "C"
