// Filtering stage (Alg. 1) on gfx950: cosine weighting, then linear
// convolution of every detector row with the sampled ramp kernel. The
// adjoint (ADJ) runs the same convolution first and weights its output: the
// kernel is even, so the convolution matrix is symmetric, and the weighting
// is diagonal.
//
// Short rows (and rows too long for the FFT tile) use a direct convolution:
// one workgroup per row, the weighted row and the kernel taps in LDS.
//
// Longer rows use the convolution theorem (Sec. 2.2.3) on the row's first
// difference and the running sum of the kernel (an identity by summation by
// parts, detailed at the FFT path below), in FP32 transforms of a
// power-of-two length L >= 2 Nu, so the circular convolution equals the
// linear one on the Nu outputs. Two rows travel as the real and imaginary
// parts of one complex sequence. The FFTs are radix-16 Stockham passes over
// points held in registers, exchanged through LDS between passes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geom_device.h"
#include "ops_internal.h"

// Multiply-adds fuse only within one expression (the explicit fmaf calls
// and single-expression products), never across statements after
// inlining: the arithmetic is then the same in every instantiation, so the
// 16-bit outputs are exactly the FP32 output rounded.
#pragma clang fp contract(on)

namespace fdk {
namespace {

constexpr int kFilterThreads = 256;
constexpr int kFftMaxLog = 13;             // L <= 8192 complex points (132 KiB of LDS)
constexpr int64_t kFftMaxGroups = 2048;    // workgroups of an FFT launch
constexpr int kDirectMaxNu = 256;          // below this the direct kernel is cheaper
constexpr int kDirectMaxLds = 8192;        // widest row of the direct kernel (2 x 64 KB of LDS)

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
__device__ __forceinline__ double cos_weight_f64(const GeoConst& gc, double du, double dv,
                                                 double sdd, int32_t a, int32_t b) {
  const double aa = (a - gc.cu) * du, bb = (b - gc.cv) * dv;
  return sdd / sqrt(sdd * sdd + aa * aa + bb * bb);
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

// Direct convolution, one workgroup per row, in FP64 (weighted row and
// taps in LDS): like the FFT path, it keeps the output accurate on smooth
// rows, whose filtered values are small next to the terms of the sum (an
// FP32 sum misses by ~3e-5 rel-L2 on 5000-pixel phantom rows).
template <typename OutT, bool ADJ>
__global__ __launch_bounds__(kFilterThreads) void filter_direct_kernel(
    GeoConst gc, RowBand rband, double du, double dv, double sdd, double tau, int kind,
    const float* __restrict__ e, OutT* __restrict__ q) {
  extern __shared__ double dlds[];
  const int32_t nu = gc.nu;
  double* et = dlds;      // cosine-weighted row
  double* h = dlds + nu;  // tau * h(|n|), n in [0, nu)
  const BandRow br = band_row(rband, nu, blockIdx.x);
  const int32_t b = br.b;
  const float* er = e + br.ein;
  for (int32_t a = threadIdx.x; a < nu; a += kFilterThreads) {
    et[a] = ADJ ? static_cast<double>(er[a]) : er[a] * cos_weight_f64(gc, du, dv, sdd, a, b);
    h[a] = tau * ramp_tap(kind, a, tau);
  }
  __syncthreads();
  OutT* qr = q + br.qout;
  for (int32_t a = threadIdx.x; a < nu; a += kFilterThreads) {
    double acc = 0.0;
    for (int32_t n = 0; n < nu; ++n) {
      const int32_t d = a - n;
      acc = fma(h[d < 0 ? -d : d], et[n], acc);
    }
    store_q(qr + a, static_cast<float>(ADJ ? acc * cos_weight_f64(gc, du, dv, sdd, a, b) : acc));
  }
}

// Lets kernel K use more than the default 64 KB of dynamic LDS on the
// current device. Called before every launch that needs it: the attribute
// call is host-side only (no stream work), so it is also valid while the
// caller's stream is being captured into a graph.
template <auto K>
hipError_t raise_lds_limit(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(K),
                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

// ---- FFT path -------------------------------------------------------------
// Ramp filtering as a first difference followed by a convolution with the
// running sum of the kernel. With g(m) = sum of tau h(j) over -N < j <= m,
// for m in [-N, N) (so g(-N) = 0 and g(m) - g(m - 1) = tau h(m) on the
// kernel's support |m| < N), summation by parts gives, for a in [0, N),
//   q(a) = sum_{n < N} g(a - n) y(n) - c g(a - N),
// with y(n) = x(n) - x(n - 1) (x(-1) = 0) the first difference of the
// weighted row x and c = x(N - 1) its last value. Setting y(N) = -c (the
// difference to x(N) = 0) folds the last term into the sum over n <= N.
// This is the factorisation of the ramp into a derivative and a
// Hilbert-type transform: |w| over |1 - e^{-iw}| stays within a factor of
// about pi/2 of its mean, so g's spectrum G is nearly flat. That is what allows FP32 transforms. The ramp
// removes most of a smooth row's content: transformed directly, the FP32
// rounding of its large low-frequency terms spreads over all bins, which
// the ramp then amplifies (1e-6 to 2e-5 rel-L2 off the FP64 result on
// projections of ellipsoid phantoms, 512 to 4096 pixels). y carries only
// the row's variation and G weights every bin about equally, so FP32
// transforms of y stay within a few FP32 roundings of the output (about
// 1e-7). y is formed in FP32 from the row's differences and the weight's
// steps (see row_diff), never from x; g comes from an FP64 scan.
//
// Rows are zero-padded to a power of two L >= 2N: with y supported on
// [0, N] and g on [-N, N), the outputs a in [0, N) see the differences
// a - n in [-N, N), whose images a - n +- L fall outside [-N, N): the
// circular convolution of length L equals the linear one there. Two rows
// travel as the real and imaginary parts of one complex sequence: g is real,
// so IFFT(FFT(a + i b) G) = (g * a) + i (g * b). The FFTs are radix-16
// Stockham passes over points held in registers, exchanged through LDS
// between passes, with each pass's twiddles read from a table of its own
// (FP64 values rounded once); the inverse transform is the forward one of
// the conjugate. Each workgroup computes the twiddle tables and G once and
// then loops over row pairs; each pair's loads are unconditional and all in
// flight together.
using cf = float2;

template <int LOGL>
struct FftCfg {
  static constexpr int L = 1 << LOGL;
  static constexpr int TPF = L / 16;                 // threads per FFT
  static constexpr int WG = TPF > 256 ? TPF : 256;   // threads per workgroup
  static constexpr int G = WG / TPF;                 // FFTs in flight per workgroup
  static constexpr int RR = 1 << (LOGL % 4);         // first-pass radix (1: none)
  static constexpr int NP = (RR > 1 ? 1 : 0) + LOGL / 4;  // passes
  static constexpr int BUF = L + L / 16;             // padded points per FFT
  // Stride NS of pass p: the length of the sub-transforms its inputs come
  // from (1 for the first pass, then the product of the earlier radices).
  static constexpr int ns(int p) { return p == 0 ? 1 : (RR > 1 ? RR : 16) << (4 * (p - 1)); }
  // Twiddle tables: pass p > 0 reads W^(r j L / (16 NS)), r in [1, 16),
  // j < NS, at entry tw_off(p) + (r - 1) NS + j; TW entries in all.
  static constexpr int tw_off(int p) {
    int off = 0;
    for (int q = 1; q < p; ++q) off += 15 * ns(q);
    return off;
  }
  static constexpr int TW = tw_off(NP);
};

template <int LOGL, int IP>
struct PassCfg {
  using C = FftCfg<LOGL>;
  static constexpr bool kRR = C::RR > 1 && IP == 0;
  static constexpr int R = kRR ? C::RR : 16;
  static constexpr int NS = C::ns(IP);
  static constexpr int B = 16 / R;  // butterflies per thread
};

// One padding point after every 16 keeps the radix-16 scatters free of bank
// conflicts.
__device__ __forceinline__ int32_t fpad(int32_t i) { return i + (i >> 4); }

__device__ __forceinline__ cf cmul(cf a, cf b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// x W16^q with W16 = exp(-2 pi i / 16), q in [0, 8): exact rotations by
// multiples of pi/2 and pi/4 use adds only.
__device__ __forceinline__ cf rot16(cf x, int q) {
  constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
  constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
  constexpr float h = 0.70710678118654752440f;   // sqrt(1/2)
  switch (q) {
    case 0: return x;
    case 1: return make_float2(fmaf(x.x, c1, x.y * s1), fmaf(x.y, c1, -x.x * s1));
    case 2: return make_float2((x.x + x.y) * h, (x.y - x.x) * h);
    case 3: return make_float2(fmaf(x.x, s1, x.y * c1), fmaf(x.y, s1, -x.x * c1));
    case 4: return make_float2(x.y, -x.x);
    case 5: return make_float2(fmaf(x.y, c1, -x.x * s1), -fmaf(x.x, c1, x.y * s1));
    case 6: return make_float2((x.y - x.x) * h, -(x.x + x.y) * h);
    default: return make_float2(fmaf(x.y, s1, -x.x * c1), -fmaf(x.x, s1, x.y * c1));
  }
}

// In-register DFT of v[0, N), N in {2, 4, 8, 16}, natural order in and out:
// radix-2 decimation in time on the bit-reversed copy.
template <int N>
__device__ __forceinline__ void dft_reg(cf* v) {
  constexpr int LOGN = N == 2 ? 1 : N == 4 ? 2 : N == 8 ? 3 : 4;
  cf a[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < LOGN; ++b) r |= ((i >> b) & 1) << (LOGN - 1 - b);
    a[r] = v[i];
  }
#pragma unroll
  for (int h = 1; h < N; h *= 2) {
#pragma unroll
    for (int i = 0; i < N; i += 2 * h) {
#pragma unroll
      for (int p = 0; p < h; ++p) {
        const cf t = rot16(a[i + p + h], p * (16 / (2 * h)));
        const cf u = a[i + p];
        a[i + p] = make_float2(u.x + t.x, u.y + t.y);
        a[i + p + h] = make_float2(u.x - t.x, u.y - t.y);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = a[i];
}

// v[r] *= W^(r k) for r in [1, 16), read from the pass's table (NS
// entries per r; the thread's j = t mod NS picks k = j L / (16 NS)).
template <int NS>
__device__ __forceinline__ void apply_twiddles(cf* v, const cf* tab, int32_t j) {
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tab[(r - 1) * NS + j]);
}

// Input index of point (m, r) of pass IP for thread t: butterfly
// j = t + m TPF, element r, index j + r L / R.
template <int LOGL, int IP>
__device__ __forceinline__ int32_t gather_index(int32_t t, int m, int r) {
  using P = PassCfg<LOGL, IP>;
  return t + m * FftCfg<LOGL>::TPF + r * (FftCfg<LOGL>::L / P::R);
}

// Output index of result r of butterfly j in pass IP (Stockham autosort).
template <int LOGL, int IP>
__device__ __forceinline__ int32_t scatter_index(int32_t j, int r) {
  using P = PassCfg<LOGL, IP>;
  return (j / P::NS) * (P::NS * P::R) + (j % P::NS) + r * P::NS;
}

// The last pass leaves point t + j TPF in register j; the first pass takes
// point t + m TPF + r L / R0 in register m R0 + r. Both are the points
// t + i TPF, i < 16, so one transform's output feeds the next without
// crossing LDS: first-pass register m R0 + r is last-pass register
// m + r (16 / R0).
template <int LOGL>
__device__ __forceinline__ constexpr int last_of_first(int i) {
  using P = PassCfg<LOGL, 0>;
  return i / P::R + (i % P::R) * P::B;
}

// Twiddle and DFT of pass IP; v holds the gathered points. Passes with
// NS > 1 are radix 16 with one butterfly per thread (j = t), twiddle
// exponent k = (t mod NS) L / (16 NS).
template <int LOGL, int IP>
__device__ __forceinline__ void pass_compute(cf* v, int32_t t, const cf* tw) {
  using P = PassCfg<LOGL, IP>;
  if constexpr (P::NS > 1)
    apply_twiddles<P::NS>(v, tw + FftCfg<LOGL>::tw_off(IP), t % P::NS);
#pragma unroll
  for (int m = 0; m < P::B; ++m) dft_reg<P::R>(v + m * P::R);
}

template <int LOGL, int IP>
__device__ __forceinline__ void pass_scatter_lds(cf* buf, int32_t t, const cf* v) {
  using P = PassCfg<LOGL, IP>;
#pragma unroll
  for (int m = 0; m < P::B; ++m)
#pragma unroll
    for (int r = 0; r < P::R; ++r)
      buf[fpad(scatter_index<LOGL, IP>(t + m * FftCfg<LOGL>::TPF, r))] = v[m * P::R + r];
}

template <int LOGL, int IP>
__device__ __forceinline__ void pass_gather_lds(const cf* buf, int32_t t, cf* v) {
  using P = PassCfg<LOGL, IP>;
#pragma unroll
  for (int m = 0; m < P::B; ++m)
#pragma unroll
    for (int r = 0; r < P::R; ++r) v[m * P::R + r] = buf[fpad(gather_index<LOGL, IP>(t, m, r))];
}

// Passes IP..NP-1 of a transform whose points sit in v (already gathered
// for pass IP). The last pass leaves its results in v, in the order of
// scatter_index; every earlier pass crosses LDS, behind a barrier that also
// orders it after the buffer's previous reads.
template <int LOGL, int IP>
__device__ __forceinline__ void fft_rest(cf* buf, int32_t t, cf* v, const cf* tw) {
  pass_compute<LOGL, IP>(v, t, tw);
  if constexpr (IP + 1 < FftCfg<LOGL>::NP) {
    __syncthreads();
    pass_scatter_lds<LOGL, IP>(buf, t, v);
    __syncthreads();
    pass_gather_lds<LOGL, IP + 1>(buf, t, v);
    fft_rest<LOGL, IP + 1>(buf, t, v, tw);
  }
}

// Cosine weight of pixel a on a row, w(a) = D / sqrt(D^2 + ((b - cv) dv)^2 +
// ((a - cu) du)^2), in FP32: the row's share `base` comes from FP64, the
// reciprocal square root from the hardware (within 1 ulp).
struct RowWeight {
  float base;  // D^2 + ((b - cv) dv)^2
};
struct ColConst {
  float cu, du, d, mddu;  // cu, du, D, and -D du
};
__device__ __forceinline__ RowWeight row_weight(const GeoConst& gc, double dv, double sdd, int32_t b) {
  const double bb = (b - gc.cv) * dv;
  return RowWeight{static_cast<float>(fma(bb, bb, sdd * sdd))};
}
__device__ __forceinline__ float pixel_weight(RowWeight rw, const ColConst& cc, int32_t a) {
  const float x = (static_cast<float>(a) - cc.cu) * cc.du;
  return cc.d * __builtin_amdgcn_rsqf(fmaf(x, x, rw.base));
}

constexpr int kBufferWord3 = 0x00020000;  // raw buffer descriptor, gfx9 family

// Raw buffer over `bytes` bytes from p: loads beyond return zero, stores
// beyond are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes),
                                           kBufferWord3);
}
__device__ __forceinline__ float buf_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store_q(float x, __amdgpu_buffer_rsrc_t r, uint32_t off, float*) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store_q(float x, __amdgpu_buffer_rsrc_t r, uint32_t off, f16_t*) {
  f16_t h;
  store_q(&h, x);
  __builtin_amdgcn_raw_buffer_store_b16(h.bits, r, off, 0, 0);
}
__device__ __forceinline__ void buf_store_q(float x, __amdgpu_buffer_rsrc_t r, uint32_t off, bf16_t*) {
  bf16_t h;
  store_q(&h, x);
  __builtin_amdgcn_raw_buffer_store_b16(h.bits, r, off, 0, 0);
}

// First difference y(n) = x(n) - x(n - 1) of the weighted row x(a) = e(a) w(a)
// at pixel n (x(-1) = 0, and x(a) = 0 for a >= N: pixels there read as zero;
// the adjoint leaves the row unweighted), in FP32 without forming x:
// y(n) = (e(n) - e(n - 1)) w(n) + e(n - 1) dw(n),
// where the weight step dw(n) = w(n) - w(n - 1) comes from the identity
// r1 - r0 = (s0 - s1) r0^2 r1^2 / (r0 + r1) for r = s^(-1/2), with
// s0 - s1 = -du (x0 + x1) exact up to rounding. Each term then carries
// rounding relative to the row's variation, not to x itself, which is what
// the FP32 transforms of y need (see the FFT path above). The load at n - 1
// for n = 0 wraps to an out-of-range offset and reads 0.
template <bool ADJ>
__device__ __forceinline__ float row_diff(__amdgpu_buffer_rsrc_t r, RowWeight rw, const ColConst& cc,
                                          int32_t n) {
  const uint32_t off = static_cast<uint32_t>(n) * 4u;
  const float e1 = buf_load_f32(r, off), e0 = buf_load_f32(r, off - 4u);
  if (ADJ) return e1 - e0;
  const float x1 = (static_cast<float>(n) - cc.cu) * cc.du;
  const float x0 = x1 - cc.du;
  const float r1 = __builtin_amdgcn_rsqf(fmaf(x1, x1, rw.base));
  const float r0 = __builtin_amdgcn_rsqf(fmaf(x0, x0, rw.base));
  const float p = r0 * r1;
  const float dw = (x1 + x0) * cc.mddu * (p * p) * __builtin_amdgcn_rcpf(r0 + r1);
  return fmaf(e1 - e0, cc.d * r1, e0 * dw);
}

template <int LOGL, typename OutT, bool ADJ>
__global__ __launch_bounds__(FftCfg<LOGL>::WG) void filter_fft_kernel(
    GeoConst gc, RowBand rband, double du, double dv, double sdd, double tau, int kind,
    int64_t nrows, const float* __restrict__ e, OutT* __restrict__ q) {
  using C = FftCfg<LOGL>;
  constexpr int R0 = PassCfg<LOGL, 0>::R, B0 = PassCfg<LOGL, 0>::B;
  extern __shared__ cf fbuf[];
  const int32_t g = static_cast<int32_t>(threadIdx.x) / C::TPF;
  const int32_t t = static_cast<int32_t>(threadIdx.x) % C::TPF;
  cf* buf = fbuf + g * C::BUF;
  cf* tw = fbuf + C::G * C::BUF;  // twiddle tables after the FFT buffers
  const int32_t nu = gc.nu;
  const ColConst cc{static_cast<float>(gc.cu), static_cast<float>(du), static_cast<float>(sdd),
                    static_cast<float>(-sdd * du)};

  for (int32_t i = threadIdx.x; i < C::TW; i += C::WG) {
    int p = 1;
    while (p + 1 < C::NP && i >= C::tw_off(p + 1)) ++p;
    const int32_t ns = C::ns(p), rel = i - C::tw_off(p);
    const int32_t m = (rel / ns + 1) * (rel % ns) * (C::L / (16 * ns));  // < L
    double sv, cv;
    sincospi(-2.0 * static_cast<double>(m) / C::L, &sv, &cv);
    tw[i] = make_float2(static_cast<float>(cv), static_cast<float>(sv));
  }

  // g(m) for m in [-N, N), FP64, at dg[m + N]: an inclusive scan of the
  // taps over the workgroup (consecutive chunks per thread, then the chunk
  // totals), in the FFT buffers: their G (L + L/16) points of 8 bytes hold
  // the 2N + WG doubles (L >= 2N and G L / 16 = WG).
  double* dg = reinterpret_cast<double*>(fbuf);
  double* part = dg + 2 * nu;
  {
    const int32_t n2 = 2 * nu;
    const int32_t chunk = (n2 + C::WG - 1) / C::WG;
    const int32_t k0 = static_cast<int32_t>(threadIdx.x) * chunk;
    double s = 0.0;
    for (int32_t j = 0; j < chunk; ++j) {
      const int32_t k = k0 + j;
      if (k < n2) {
        if (k > 0) s += tau * ramp_tap(kind, k - nu, tau);
        dg[k] = s;
      }
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int32_t off = 1; off < C::WG; off *= 2) {
      const double p = threadIdx.x >= static_cast<uint32_t>(off) ? part[threadIdx.x - off] : 0.0;
      __syncthreads();
      part[threadIdx.x] += p;
      __syncthreads();
    }
    const double before = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0.0;
    for (int32_t j = 0; j < chunk; ++j) {
      const int32_t k = k0 + j;
      if (k < n2) dg[k] += before;
    }
    __syncthreads();
  }

  // G: FFT of g placed circularly (index m mod L). Each thread keeps
  // conj(G) / L at the points it gathers in a transform's first pass.
  cf v[16];
#pragma unroll
  for (int m = 0; m < B0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int32_t n = gather_index<LOGL, 0>(t, m, r);
      const int32_t s = n < C::L / 2 ? n : n - C::L;
      const float gv = (s >= -nu && s < nu) ? static_cast<float>(dg[s + nu]) : 0.0f;
      v[m * R0 + r] = make_float2(gv, 0.0f);
    }
  fft_rest<LOGL, 0>(buf, t, v, tw);  // its first barrier follows every read of dg
  cf gc_[16];
  {
    constexpr float inv_l = 1.0f / static_cast<float>(C::L);  // a power of two: exact
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const cf x = v[last_of_first<LOGL>(i)];
      gc_[i] = make_float2(x.x * inv_l, -x.y * inv_l);
    }
  }

  // Row pairs are wave-uniform (an FFT spans whole waves), so each row is
  // addressed through a buffer descriptor: pixels at or beyond Nu, and rows
  // past the end, read as zero and are never written.
  const int32_t gw = __builtin_amdgcn_readfirstlane(g);
  const uint32_t npairs = static_cast<uint32_t>((nrows + 1) / 2);
  const uint32_t band = static_cast<uint32_t>(rband.band);
  for (uint32_t base = blockIdx.x * C::G; base < npairs; base += gridDim.x * C::G) {
    const uint32_t pr = base + static_cast<uint32_t>(gw);
    const uint32_t ra = 2 * pr, rb = ra + 1;
    const bool has_a = pr < npairs, has_b = rb < static_cast<uint32_t>(nrows);
    const uint32_t sa = ra / band, sb = rb / band;
    const int32_t ba = rband.v0 + static_cast<int32_t>(ra - sa * band);
    const int32_t bb = rband.v0 + static_cast<int32_t>(rb - sb * band);
    const int64_t rowa_in = sa * rband.e_stride + static_cast<int64_t>(ra - sa * band) * nu;
    const int64_t rowb_in = sb * rband.e_stride + static_cast<int64_t>(rb - sb * band) * nu;
    const int64_t rowa_out = sa * rband.q_stride + static_cast<int64_t>(ra - sa * band) * nu;
    const int64_t rowb_out = sb * rband.q_stride + static_cast<int64_t>(rb - sb * band) * nu;
    const __amdgpu_buffer_rsrc_t ia = row_rsrc(e + (has_a ? rowa_in : 0), has_a ? nu * 4u : 0u);
    const __amdgpu_buffer_rsrc_t ib = row_rsrc(e + (has_b ? rowb_in : 0), has_b ? nu * 4u : 0u);
    const RowWeight wa = row_weight(gc, dv, sdd, ba), wb = row_weight(gc, dv, sdd, bb);
    // Forward transform of y over [0, N] and zeros beyond. The loads are
    // unconditional, all in flight together: pixels at or beyond N read as
    // zero, so row_diff gives 0 past N and, at N, y(N) = -x(N - 1) =
    // -c (up to rounding). Points below L/2 are those of registers
    // r < R0/2; N <= L/2 can only fall at r = R0/2 when N = L/2, on thread
    // 0's first butterfly.
#pragma unroll
    for (int m = 0; m < B0; ++m)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        float re = 0.0f, im = 0.0f;
        if (r < R0 / 2) {
          const int32_t n = gather_index<LOGL, 0>(t, m, r);
          re = row_diff<ADJ>(ia, wa, cc, n);
          im = row_diff<ADJ>(ib, wb, cc, n);
        }
        v[m * R0 + r] = make_float2(re, im);
      }
    if (nu == C::L / 2) {
      const int32_t n = gather_index<LOGL, 0>(t, 0, R0 / 2);
      v[R0 / 2] = make_float2(row_diff<ADJ>(ia, wa, cc, n), row_diff<ADJ>(ib, wb, cc, n));
    }
    fft_rest<LOGL, 0>(buf, t, v, tw);
    // Inverse: the forward transform of conj(Y G) / L, taken in registers
    // (the last pass's points are the first pass's).
    cf z[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const cf y = v[last_of_first<LOGL>(i)];
      z[i] = cmul(make_float2(y.x, -y.y), gc_[i]);
    }
    fft_rest<LOGL, 0>(buf, t, z, tw);
    // The last pass has one radix-16 butterfly per thread (j = t, NS = L/16):
    // result j is point t + j L/16, so the stores are coalesced; only the
    // lower half (j < 8) holds row pixels.
    const __amdgpu_buffer_rsrc_t oa =
        row_rsrc(q + (has_a ? rowa_out : 0), has_a ? nu * static_cast<uint32_t>(sizeof(OutT)) : 0u);
    const __amdgpu_buffer_rsrc_t ob =
        row_rsrc(q + (has_b ? rowb_out : 0), has_b ? nu * static_cast<uint32_t>(sizeof(OutT)) : 0u);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int32_t n = t + j * C::TPF;
      float ya = z[j].x, yb = -z[j].y;
      if (ADJ) {
        ya *= pixel_weight(wa, cc, n);
        yb *= pixel_weight(wb, cc, n);
      }
      // The FP32 result is rounded as such before any 16-bit store: without
      // the barrier the last operation could fuse into a mixed-precision one
      // that rounds once to 16 bits, which can differ from the FP32 output
      // rounded.
      asm volatile("" : "+v"(ya), "+v"(yb));
      const uint32_t off = static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(OutT));
      buf_store_q(ya, oa, off, static_cast<OutT*>(nullptr));
      buf_store_q(yb, ob, off, static_cast<OutT*>(nullptr));
    }
  }
}

template <int LOGL, typename OutT, bool ADJ>
int launch_fft(const GeoConst& gc, const RowBand& rb, double du, double dv, double sdd, double tau,
               int kind, int64_t nrows, const float* e, OutT* q, hipStream_t st) {
  using C = FftCfg<LOGL>;
  const size_t lds = (static_cast<size_t>(C::G) * C::BUF + C::TW) * sizeof(cf);
  auto kern = &filter_fft_kernel<LOGL, OutT, ADJ>;
  if (lds > 65536) {
    const hipError_t err = raise_lds_limit<&filter_fft_kernel<LOGL, OutT, ADJ>>(lds);
    if (err != hipSuccess) return static_cast<int>(err);
  }
  // Workgroups loop over row pairs (G is computed once per workgroup): a
  // few per CU at most.
  const int64_t npairs = (nrows + 1) / 2;
  const int64_t want = (npairs + C::G - 1) / C::G;
  const uint32_t groups = static_cast<uint32_t>(std::min<int64_t>(want, kFftMaxGroups));
  hipLaunchKernelGGL(kern, dim3(groups), dim3(C::WG), lds, st, gc, rb, du, dv, sdd, tau, kind,
                     nrows, e, q);
  return static_cast<int>(hipGetLastError());
}

template <typename OutT, bool ADJ>
int launch_filter_t(const GeoConst& gc, const RowBand& rb, double du, double dv, double sdd,
                    double tau, int kind, const float* e, void* q, hipStream_t st) {
  OutT* qt = static_cast<OutT*>(q);
  int32_t logl = 0;
  while ((1 << logl) < 2 * gc.nu - 1) ++logl;
  // Launches of whole views and fewer than 2^30 rows (row indices and pair
  // counts stay 32-bit inside the kernels).
  const int32_t per = std::max<int32_t>(1, static_cast<int32_t>((int64_t{1} << 30) / rb.band));
  for (int32_t s0 = 0; s0 < rb.nviews; s0 += per) {
    RowBand sub = rb;
    sub.nviews = std::min(per, rb.nviews - s0);
    const float* es = e + s0 * rb.e_stride;
    OutT* qs = qt + s0 * rb.q_stride;
    const int64_t nrows = static_cast<int64_t>(sub.nviews) * sub.band;
    if (nrows == 0) continue;
    int err = 0;
    if (gc.nu > kDirectMaxNu && logl <= kFftMaxLog) {
      switch (logl) {
        case 10: err = launch_fft<10, OutT, ADJ>(gc, sub, du, dv, sdd, tau, kind, nrows, es, qs, st); break;
        case 11: err = launch_fft<11, OutT, ADJ>(gc, sub, du, dv, sdd, tau, kind, nrows, es, qs, st); break;
        case 12: err = launch_fft<12, OutT, ADJ>(gc, sub, du, dv, sdd, tau, kind, nrows, es, qs, st); break;
        default: err = launch_fft<13, OutT, ADJ>(gc, sub, du, dv, sdd, tau, kind, nrows, es, qs, st); break;
      }
    } else {
      const size_t lds = 2 * static_cast<size_t>(gc.nu) * sizeof(double);
      if (lds > 65536) {
        const hipError_t e2 = raise_lds_limit<&filter_direct_kernel<OutT, ADJ>>(
            2 * static_cast<size_t>(kDirectMaxLds) * sizeof(double));
        if (e2 != hipSuccess) return static_cast<int>(e2);
      }
      hipLaunchKernelGGL((filter_direct_kernel<OutT, ADJ>), dim3(static_cast<uint32_t>(nrows)),
                         dim3(kFilterThreads), lds, st, gc, sub, du, dv, sdd, tau, kind, es, qs);
      err = static_cast<int>(hipGetLastError());
    }
    if (err) return err;
  }
  return 0;
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
