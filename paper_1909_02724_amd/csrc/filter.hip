// Filtering stage (Alg. 1) on gfx950: cosine weighting, then linear
// convolution of every detector row with the sampled ramp kernel. The
// adjoint (ADJ) runs the same convolution first and weights its output: the
// kernel is even, so the convolution matrix is symmetric, and the weighting
// is diagonal.
//
// Short rows (and rows too long for the FFT tile) use a direct convolution:
// one workgroup per row, the weighted row and the kernel taps in LDS.
//
// Longer rows use the convolution theorem (Sec. 2.2.3) with FFTs in LDS:
// rows are zero-padded to L >= 2 Nu - 1 (a power of two), so the circular
// convolution of length L equals the linear one on the Nu outputs. Two rows
// travel as the real and imaginary parts of one complex sequence: the ramp
// kernel is real and even, its spectrum H is real, and IFFT(FFT(a + i b) H) =
// (a * h) + i (b * h). Each workgroup computes H once (an FFT of the
// circularly arranged taps) and then filters several row pairs. In-place
// radix-2 decimation in time on bit-reversed input; twiddles in LDS.
#include <hip/hip_runtime.h>

#include "geom_device.h"
#include "ops_internal.h"

namespace fdk {
namespace {

constexpr int kFilterThreads = 256;
constexpr int kFftMaxLog = 13;             // L <= 8192 complex points (64 KB)
constexpr int kFftMaxL = 1 << kFftMaxLog;
constexpr int kFftPerThread = kFftMaxL / kFilterThreads;
constexpr int kFftRowPairs = 8;            // row pairs per workgroup (one H each)
constexpr int kDirectMaxNu = 256;          // below this the direct kernel is cheaper
constexpr int kDirectBlock = 128;          // taps per partial sum in the direct kernel

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

// Cosine weight of pixel (a, b): D / sqrt(D^2 + ((a - cu) du)^2 + ((b - cv) dv)^2).
__device__ __forceinline__ float cos_weight(const GeoConst& gc, double du, double dv, double sdd,
                                            int32_t a, int32_t b) {
  const double aa = (a - gc.cu) * du, bb = (b - gc.cv) * dv;
  return static_cast<float>(sdd / sqrt(sdd * sdd + aa * aa + bb * bb));
}

// Row m of a band launch: input and output row pointers and detector row.
struct BandRow {
  int64_t ein, qout;  // element offsets of the row in e and q
  int32_t b;          // detector row
};
__device__ __forceinline__ BandRow band_row(const RowBand& rb, int32_t nu, int64_t m) {
  const int64_t s = m / rb.band, r = m - s * rb.band;
  return BandRow{s * rb.e_stride + r * nu, s * rb.q_stride + r * nu,
                 static_cast<int32_t>(rb.v0 + r)};
}

template <typename OutT, bool ADJ>
__global__ __launch_bounds__(kFilterThreads) void filter_direct_kernel(
    GeoConst gc, RowBand rband, double du, double dv, double sdd, double tau, int kind,
    const float* __restrict__ e, OutT* __restrict__ q) {
  extern __shared__ float lds[];
  const int32_t nu = gc.nu;
  float* et = lds;      // cosine-weighted row
  float* h = lds + nu;  // tau * h(|n|), n in [0, nu)
  const BandRow br = band_row(rband, nu, blockIdx.x);
  const int32_t b = br.b;
  const float* er = e + br.ein;
  for (int32_t a = threadIdx.x; a < nu; a += kFilterThreads) {
    et[a] = ADJ ? er[a] : er[a] * cos_weight(gc, du, dv, sdd, a, b);
    h[a] = static_cast<float>(tau * ramp_tap(kind, a, tau));
  }
  __syncthreads();
  OutT* qr = q + br.qout;
  for (int32_t a = threadIdx.x; a < nu; a += kFilterThreads) {
    // Blocked sum: a serial FP32 sum over up to 8192 taps loses about
    // 1e-5 relative; partial sums of kDirectBlock taps keep it near 2e-7.
    float acc = 0.0f;
    for (int32_t n0 = 0; n0 < nu; n0 += kDirectBlock) {
      const int32_t n1 = min(nu, n0 + kDirectBlock);
      float part = 0.0f;
      for (int32_t n = n0; n < n1; ++n) {
        const int32_t d = a - n;
        part = fmaf(h[d < 0 ? -d : d], et[n], part);
      }
      acc += part;
    }
    store_q(qr + a, ADJ ? acc * cos_weight(gc, du, dv, sdd, a, b) : acc);
  }
}

// In-place radix-2 FFT of x[0, L) (bit-reversed input, natural output),
// forward transform exp(-2 pi i k n / L); tw[k] = exp(-2 pi i k / L), k < L/2.
__device__ void fft_inplace(float2* x, const float2* tw, int32_t logl) {
  const int32_t L = 1 << logl, halfL = L >> 1;
  for (int32_t s = 1; s <= logl; ++s) {
    const int32_t half = 1 << (s - 1);
    const int32_t tstep = L >> s;  // twiddle index stride for this stage
    for (int32_t bf = threadIdx.x; bf < halfL; bf += kFilterThreads) {
      const int32_t pos = bf & (half - 1);
      const int32_t i = ((bf >> (s - 1)) << s) + pos;
      const int32_t j = i + half;
      const float2 w = tw[pos * tstep];
      const float2 u = x[i], v = x[j];
      const float2 t = make_float2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
      x[i] = make_float2(u.x + t.x, u.y + t.y);
      x[j] = make_float2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int32_t bitrev(int32_t n, int32_t logl) {
  return static_cast<int32_t>(__builtin_bitreverse32(static_cast<uint32_t>(n)) >> (32 - logl));
}

template <typename OutT, bool ADJ>
__global__ __launch_bounds__(kFilterThreads) void filter_fft_kernel(
    GeoConst gc, RowBand rband, double du, double dv, double sdd, double tau, int kind,
    int32_t logl, int64_t nrows, const float* __restrict__ e, OutT* __restrict__ q) {
  extern __shared__ float2 flds[];
  const int32_t L = 1 << logl, nu = gc.nu;
  float2* x = flds;       // L complex points
  float2* tw = flds + L;  // L / 2 twiddles
  for (int32_t k = threadIdx.x; k < L / 2; k += kFilterThreads) {
    double sv, cv;
    sincospi(-2.0 * k / L, &sv, &cv);
    tw[k] = make_float2(static_cast<float>(cv), static_cast<float>(sv));
  }
  // Kernel spectrum: taps tau * h(n) for |n| < Nu arranged circularly.
  for (int32_t n = threadIdx.x; n < L; n += kFilterThreads) {
    const int32_t m = n < L / 2 ? n : n - L;  // signed offset
    const float hv = (m > -nu && m < nu) ? static_cast<float>(tau * ramp_tap(kind, m, tau)) : 0.0f;
    x[bitrev(n, logl)] = make_float2(hv, 0.0f);
  }
  __syncthreads();
  fft_inplace(x, tw, logl);
  float H[kFftPerThread];
#pragma unroll
  for (int m = 0; m < kFftPerThread; ++m) {
    const int32_t k = threadIdx.x + m * kFilterThreads;
    H[m] = (k < L) ? x[k].x / static_cast<float>(L) : 0.0f;  // real; 1/L of the inverse folded in
  }
  __syncthreads();

  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 2 * kFftRowPairs;  // launch rows
  for (int32_t p = 0; p < kFftRowPairs; ++p) {
    const int64_t ra = row0 + 2 * p, rb = ra + 1;
    if (ra >= nrows) break;  // uniform
    const bool has_b = rb < nrows;
    const BandRow rowa = band_row(rband, nu, ra);
    const BandRow rowb = band_row(rband, nu, has_b ? rb : ra);
    for (int32_t n = threadIdx.x; n < L; n += kFilterThreads) {
      float re = 0.0f, im = 0.0f;
      if (n < nu) {
        re = ADJ ? e[rowa.ein + n] : e[rowa.ein + n] * cos_weight(gc, du, dv, sdd, n, rowa.b);
        if (has_b)
          im = ADJ ? e[rowb.ein + n] : e[rowb.ein + n] * cos_weight(gc, du, dv, sdd, n, rowb.b);
      }
      x[bitrev(n, logl)] = make_float2(re, im);
    }
    __syncthreads();
    fft_inplace(x, tw, logl);
    // Multiply by H, conjugate, and write back bit-reversed: the forward
    // transform of the conjugate is L times the conjugated inverse.
    float2 y[kFftPerThread];
#pragma unroll
    for (int m = 0; m < kFftPerThread; ++m) {
      const int32_t k = threadIdx.x + m * kFilterThreads;
      if (k < L) {
        const float2 v = x[k];
        y[m] = make_float2(v.x * H[m], -v.y * H[m]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kFftPerThread; ++m) {
      const int32_t k = threadIdx.x + m * kFilterThreads;
      if (k < L) x[bitrev(k, logl)] = y[m];
    }
    __syncthreads();
    fft_inplace(x, tw, logl);
    for (int32_t n = threadIdx.x; n < nu; n += kFilterThreads) {
      const float2 v = x[n];
      if (ADJ) {
        store_q(q + rowa.qout + n, v.x * cos_weight(gc, du, dv, sdd, n, rowa.b));
        if (has_b) store_q(q + rowb.qout + n, -v.y * cos_weight(gc, du, dv, sdd, n, rowb.b));
      } else {
        store_q(q + rowa.qout + n, v.x);
        if (has_b) store_q(q + rowb.qout + n, -v.y);
      }
    }
    __syncthreads();
  }
}

template <typename OutT, bool ADJ>
int launch_filter_t(const GeoConst& gc, const RowBand& rb, double du, double dv, double sdd,
                    double tau, int kind, const float* e, void* q, hipStream_t st) {
  OutT* qt = static_cast<OutT*>(q);
  const int64_t nrows = static_cast<int64_t>(rb.nviews) * rb.band;
  int32_t logl = 0;
  while ((1 << logl) < 2 * gc.nu - 1) ++logl;
  if (gc.nu > kDirectMaxNu && logl <= kFftMaxLog) {
    const int32_t L = 1 << logl;
    const size_t lds = (static_cast<size_t>(L) + L / 2) * sizeof(float2);
    const uint32_t groups = static_cast<uint32_t>((nrows + 2 * kFftRowPairs - 1) / (2 * kFftRowPairs));
    if (lds > 65536) {
      hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&filter_fft_kernel<OutT, ADJ>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
      if (err != hipSuccess) return static_cast<int>(err);
    }
    hipLaunchKernelGGL((filter_fft_kernel<OutT, ADJ>), dim3(groups), dim3(kFilterThreads), lds, st, gc,
                       rb, du, dv, sdd, tau, kind, logl, nrows, e, qt);
  } else {
    const size_t lds = 2 * static_cast<size_t>(gc.nu) * sizeof(float);
    hipLaunchKernelGGL((filter_direct_kernel<OutT, ADJ>), dim3(static_cast<uint32_t>(nrows)),
                       dim3(kFilterThreads), lds, st, gc, rb, du, dv, sdd, tau, kind, e, qt);
  }
  return static_cast<int>(hipGetLastError());
}

}  // namespace

int launch_filter(const GeoConst& gc, double du, double dv, double sod, double sdd,
                  const RowBand& rb, const float* e, void* q, fdk_dtype out_dtype,
                  fdk_filter_kind kind, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double tau = du * sod / sdd;  // pixel pitch scaled to the rotation axis
  switch (out_dtype) {
    case FDK_F32:
      return launch_filter_t<float, false>(gc, rb, du, dv, sdd, tau, kind, e, q, st);
    case FDK_F16:
      return launch_filter_t<f16_t, false>(gc, rb, du, dv, sdd, tau, kind, e, q, st);
    case FDK_BF16:
      return launch_filter_t<bf16_t, false>(gc, rb, du, dv, sdd, tau, kind, e, q, st);
  }
  return static_cast<int>(hipErrorInvalidValue);
}

int launch_filter_adjoint(const GeoConst& gc, double du, double dv, double sod, double sdd,
                          const RowBand& rb, const float* q_grad, float* e_grad,
                          fdk_filter_kind kind, void* stream) {
  const double tau = du * sod / sdd;
  return launch_filter_t<float, true>(gc, rb, du, dv, sdd, tau, kind, q_grad, e_grad,
                                      static_cast<hipStream_t>(stream));
}

}  // namespace fdk
