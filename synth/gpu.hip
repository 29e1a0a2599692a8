// GPU-side synthetic input generators (test and benchmark infrastructure,
// not part of the reconstruction library):
//  - synth_hash_fill: SplitMix64 counter-based values (Steele, Lea and Flood,
//    OOPSLA 2014) on the grid 2^-23 in [-1, 1), stored as FP32 / FP16 /
//    BF16 with round-to-nearest-even; the CPU oracle regenerates the same
//    values from its own implementation of the published generator.
//  - synth_phantom_project: analytic line integrals of a sum of ellipsoids
//    along the ray from the source to every detector pixel centre (FP64).
//  - synth_phantom_rows: the same on a band of detector rows, plus additive
//    Gaussian noise keyed by (seed, view, row, column): two SplitMix64 draws
//    through the Box-Muller transform (Box and Muller, 1958).
//  - synth_view_sigma: per-view noise level, a fraction of the largest
//    clean line integral on the detector row through the principal point.
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
// columns are the axes in world coordinates), density. Line integral along
// the ray from the source to the centre of pixel (a, b) of the view at
// gantry angle beta.
__device__ double ray_integral(const ScanGeom& g, double beta, double a, double b,
                               const double* __restrict__ ell, int32_t nell) {
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
  return acc;
}

__global__ void phantom_project_kernel(ScanGeom g, const double* __restrict__ angles,
                                       int32_t nviews, const double* __restrict__ ell,
                                       int32_t nell, float* __restrict__ out) {
  const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t b = blockIdx.y;
  const int32_t s = blockIdx.z;
  if (a >= g.nu || b >= g.nv || s >= nviews) return;
  out[(static_cast<int64_t>(s) * g.nv + b) * g.nu + a] =
      static_cast<float>(ray_integral(g, angles[s], a, b, ell, nell));
}

// Standard normal for pixel counter m: Box-Muller on the draws 2m and
// 2m + 1, with u1 = (top 53 bits + 1) 2^-53 in (0, 1] and u2 = (top 53
// bits) 2^-53 in [0, 1).
__device__ double normal_draw(uint64_t seed, uint64_t m) {
  const double u1 = static_cast<double>((splitmix64(seed, 2u * m) >> 11) + 1u) * 0x1p-53;
  const double u2 = static_cast<double>(splitmix64(seed, 2u * m + 1u) >> 11) * 0x1p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void phantom_rows_kernel(ScanGeom g, const double* __restrict__ angles, int32_t v0,
                                    const double* __restrict__ ell, int32_t nell,
                                    uint64_t seed, int64_t view_index0,
                                    const double* __restrict__ sigma, float* __restrict__ out,
                                    int64_t vstride) {
  const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t r = blockIdx.y;
  const int32_t s = blockIdx.z;
  if (a >= g.nu) return;
  const int32_t b = v0 + r;
  double e = ray_integral(g, angles[s], a, b, ell, nell);
  if (sigma) {
    const uint64_t m = (static_cast<uint64_t>(view_index0 + s) * g.nv + b) * g.nu + a;
    e += sigma[s] * normal_draw(seed, m);
  }
  out[s * vstride + static_cast<int64_t>(r) * g.nu + a] = static_cast<float>(e);
}

__global__ void view_sigma_kernel(ScanGeom g, const double* __restrict__ angles,
                                  const double* __restrict__ ell, int32_t nell, double rel,
                                  double* __restrict__ sigma) {
  __shared__ double red[256];
  const int32_t s = blockIdx.x;
  const double row = floor(g.cv);
  double m = 0.0;
  for (int32_t a = threadIdx.x; a < g.nu; a += blockDim.x)
    m = fmax(m, ray_integral(g, angles[s], a, row, ell, nell));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int32_t w = blockDim.x / 2; w > 0; w /= 2) {
    if (static_cast<int32_t>(threadIdx.x) < w)
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[s] = rel * red[0];
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

// Rows [v0, v0 + nrows) of views view_index0 + s (s < nviews; angles holds
// those views' angles): out[s * out_view_stride + r * nu + a] = line
// integral + sigma[s] * N(seed; view, row, column). sigma may be NULL (no
// noise). All arrays are device memory.
int synth_phantom_rows(int32_t nu, int32_t nv, double du, double dv, double off_u, double off_v,
                       double sod, double sdd, const double* angles, int32_t nviews, int32_t v0,
                       int32_t nrows, const double* ell, int32_t nell, uint64_t seed,
                       int64_t view_index0, const double* sigma, float* out,
                       int64_t out_view_stride, void* stream) {
  if (nu <= 0 || nv <= 0 || nviews < 0 || nrows < 0 || v0 < 0 || v0 + nrows > nv || nell < 0 ||
      !angles || !out || (nell && !ell) || view_index0 < 0 ||
      out_view_stride < static_cast<int64_t>(nrows) * nu)
    return static_cast<int>(hipErrorInvalidValue);
  if (nviews == 0 || nrows == 0) return 0;
  ScanGeom g{nu, nv, du, dv, 0.5 * (nu - 1) + off_u, 0.5 * (nv - 1) + off_v, sod, sdd};
  dim3 grid((nu + 63) / 64, nrows, nviews);
  hipLaunchKernelGGL(phantom_rows_kernel, grid, dim3(64), 0, static_cast<hipStream_t>(stream), g,
                     angles, v0, ell, nell, seed, view_index0, sigma, out, out_view_stride);
  return static_cast<int>(hipGetLastError());
}

// sigma[s] = rel * max over columns of the clean line integral on row
// floor(cv) of view s (cv = (nv - 1) / 2 + off_v).
int synth_view_sigma(int32_t nu, int32_t nv, double du, double dv, double off_u, double off_v,
                     double sod, double sdd, const double* angles, int32_t nviews,
                     const double* ell, int32_t nell, double rel, double* sigma, void* stream) {
  if (nu <= 0 || nv <= 0 || nviews < 0 || nell < 0 || !angles || !sigma || (nell && !ell))
    return static_cast<int>(hipErrorInvalidValue);
  if (nviews == 0) return 0;
  ScanGeom g{nu, nv, du, dv, 0.5 * (nu - 1) + off_u, 0.5 * (nv - 1) + off_v, sod, sdd};
  hipLaunchKernelGGL(view_sigma_kernel, dim3(nviews), dim3(256), 0,
                     static_cast<hipStream_t>(stream), g, angles, ell, nell, rel, sigma);
  return static_cast<int>(hipGetLastError());
}

}  // extern "C"
