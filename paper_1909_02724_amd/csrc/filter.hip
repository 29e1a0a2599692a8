// Filtering stage (Alg. 1) on gfx950: cosine weighting, then a direct linear
// convolution of every detector row with the sampled ramp kernel. One
// workgroup per row; the weighted row and the kernel taps live in LDS.
#include <hip/hip_runtime.h>

#include "geom_device.h"

namespace fdk {
namespace {

constexpr int kFilterThreads = 256;

// Ramp kernel h(n) at sample pitch tau: Ram-Lak (band-limited ramp) or
// Shepp-Logan (ramp times sinc), FDK literature forms.
__device__ double ramp_tap(int kind, int32_t n, double tau) {
  const double pi = 3.14159265358979323846;
  if (kind == FDK_RAMLAK) {
    if (n == 0) return 1.0 / (4.0 * tau * tau);
    if ((n & 1) == 0) return 0.0;
    return -1.0 / (static_cast<double>(n) * n * pi * pi * tau * tau);
  }
  return -2.0 / (pi * pi * tau * tau * (4.0 * static_cast<double>(n) * n - 1.0));
}

__device__ __forceinline__ void store_q(float* p, float x) { *p = x; }
__device__ __forceinline__ void store_q(f16_t* p, float x) {
  p->bits = __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
}
__device__ __forceinline__ void store_q(bf16_t* p, float x) {
  // Round to nearest, ties to even, on the upper 16 bits; NaN stays NaN.
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    p->bits = static_cast<uint16_t>((u >> 16) | 0x40u);
    return;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  p->bits = static_cast<uint16_t>(u >> 16);
}

template <typename OutT>
__global__ __launch_bounds__(kFilterThreads) void filter_kernel(GeoConst gc, double du, double dv,
                                                                double sdd, double tau, int kind,
                                                                const float* __restrict__ e,
                                                                OutT* __restrict__ q) {
  extern __shared__ float lds[];
  const int32_t nu = gc.nu;
  float* et = lds;       // cosine-weighted row
  float* h = lds + nu;   // tau * h(|n|), n in [0, nu)
  const int64_t row = blockIdx.x;
  const int32_t b = static_cast<int32_t>(row % gc.nv);
  const float* er = e + row * nu;
  const double bb = (b - gc.cv) * dv;
  for (int32_t a = threadIdx.x; a < nu; a += kFilterThreads) {
    const double aa = (a - gc.cu) * du;
    const double w = sdd / sqrt(sdd * sdd + aa * aa + bb * bb);
    et[a] = static_cast<float>(static_cast<double>(er[a]) * w);
    h[a] = static_cast<float>(tau * ramp_tap(kind, a, tau));
  }
  __syncthreads();
  OutT* qr = q + row * nu;
  for (int32_t a = threadIdx.x; a < nu; a += kFilterThreads) {
    float acc = 0.0f;
    for (int32_t n = 0; n < nu; ++n) {
      const int32_t d = a - n;
      acc = fmaf(h[d < 0 ? -d : d], et[n], acc);
    }
    store_q(qr + a, acc);
  }
}

template <typename OutT>
int launch_filter_t(const GeoConst& gc, double du, double dv, double sdd, double tau, int kind,
                    int32_t nrows, const float* e, void* q, hipStream_t st) {
  const size_t lds = 2 * static_cast<size_t>(gc.nu) * sizeof(float);
  hipLaunchKernelGGL(filter_kernel<OutT>, dim3(nrows), dim3(kFilterThreads), lds, st, gc, du, dv,
                     sdd, tau, kind, e, static_cast<OutT*>(q));
  return static_cast<int>(hipGetLastError());
}

}  // namespace

int launch_filter(const GeoConst& gc, double du, double dv, double sod, double sdd, int32_t nrows,
                  const float* e, void* q, fdk_dtype out_dtype, fdk_filter_kind kind,
                  void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double tau = du * sod / sdd;  // pixel pitch scaled to the rotation axis
  switch (out_dtype) {
    case FDK_F32:
      return launch_filter_t<float>(gc, du, dv, sdd, tau, kind, nrows, e, q, st);
    case FDK_F16:
      return launch_filter_t<f16_t>(gc, du, dv, sdd, tau, kind, nrows, e, q, st);
    case FDK_BF16:
      return launch_filter_t<bf16_t>(gc, du, dv, sdd, tau, kind, nrows, e, q, st);
  }
  return static_cast<int>(hipErrorInvalidValue);
}

}  // namespace fdk
