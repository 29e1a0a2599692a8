// Internal launch interfaces of the filtering stage and the SIRT helpers,
// shared by the host front end (fdk_api.cpp) and filter.hip / sirt.hip. Not
// part of the public ABI.
#pragma once

#include <cstdint>

#include "fdk_internal.h"

namespace fdk {

// Element-wise helpers of the SIRT iteration (sirt.hip).
int launch_fill(float* p, int64_t n, float v, void* stream);
// p <- 1 / max(p, floor_rel * max(p)) for non-negative p; maxbits: one
// device word of scratch.
int launch_invert_floor(float* p, int64_t n, float floor_rel, uint32_t* maxbits, void* stream);
int launch_sirt_residual(const float* p, const float* row_inv, float* r, int64_t n, void* stream);
int launch_sirt_update(float* x, const float* col_inv, const float* b, int64_t n, float lambda,
                       int nonneg, void* stream);
// MLEM: r <- p / max(r, floor_rel * max(r)) (0 where that is 0), r holding
// F x on entry (non-negative); maxbits: one device word of scratch.
int launch_mlem_ratio(const float* p, float* r, int64_t n, float floor_rel, uint32_t* maxbits,
                      void* stream);
// MLEM: x <- x * col_inv * b.
int launch_mlem_update(float* x, const float* col_inv, const float* b, int64_t n, void* stream);
// Per-GPU static workspace of the entry points that allocate nothing
// (sirt.hip): kStaticScratchFloats floats (64 MiB). static_scratch gives its
// device address on the current device (looked up once per device).
constexpr int64_t kStaticScratchFloats = int64_t{1} << 24;
int static_scratch(float** out);
// Filter rows [v0, v0 + band) of nviews views; row m of the launch is view
// m / band, detector row v0 + m % band; view strides in elements.
struct RowBand {
  int32_t nviews, v0, band;
  int64_t e_stride, q_stride;
};
int launch_filter(const GeoConst& gc, double du, double dv, double sod, double sdd,
                  const RowBand& rb, const float* e, void* q, fdk_dtype out_dtype,
                  fdk_filter_kind kind, void* stream);
// Adjoint of launch_filter (FP32): convolution first, cosine weight after.
int launch_filter_adjoint(const GeoConst& gc, double du, double dv, double sod, double sdd,
                          const RowBand& rb, const float* q_grad, float* e_grad,
                          fdk_filter_kind kind, void* stream);

}  // namespace fdk
