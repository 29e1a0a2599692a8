// Host front end of the C ABI declared in include/fdk.h: argument
// validation, per-view FP64 geometry, slab decomposition into slice runs
// and kernel dispatch on the caller's stream. Nothing here touches the HIP
// runtime until every argument has been validated.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <utility>
#include <vector>

#include "fdk_internal.h"
#include "geometry_host.h"
#include "ops_internal.h"

namespace {

using fdk::make_geo;
using fdk::make_view;

thread_local std::string g_last_error;

fdk_status fail(fdk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

fdk_status ok() {
  g_last_error.clear();
  return FDK_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// An enum argument as the integer the caller passed. C callers may pass any
// int; in C++ reading an enum object that holds a value outside its
// enumerators is undefined, so arguments are validated through their bytes.
template <class E>
int32_t raw(const E& e) {
  static_assert(sizeof(E) == sizeof(int32_t), "enums of the C ABI are int-sized");
  int32_t v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

// Largest |u - cu| or |v - cv| (pixels) allowed, so that pixel indices and
// LDS/tap offsets stay well inside int32 arithmetic.
constexpr double kMaxCoord = 4194304.0;  // 2^22

fdk_status check_geometry(const fdk_geometry* g) {
  if (!g) return fail(FDK_ERR_INVALID_ARG, "geometry pointer is NULL");
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0)
    return fail(FDK_ERR_INVALID_ARG, "volume size must be positive (got %d x %d x %d)", g->nx,
                g->ny, g->nz);
  if (g->nu <= 0 || g->nv <= 0)
    return fail(FDK_ERR_INVALID_ARG, "detector size must be positive (got %d x %d)", g->nu, g->nv);
  if ((int64_t)g->nu * g->nv > (int64_t)1 << 27)
    return fail(FDK_ERR_INVALID_ARG, "detector of %d x %d pixels is too large", g->nu, g->nv);
  if ((int64_t)g->nx * g->ny > (int64_t)1 << 30)
    return fail(FDK_ERR_INVALID_ARG, "volume slice of %d x %d voxels is too large", g->nx, g->ny);
  if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz))
    return fail(FDK_ERR_INVALID_ARG, "voxel pitch must be positive and finite");
  if (!finite_pos(g->du) || !finite_pos(g->dv))
    return fail(FDK_ERR_INVALID_ARG, "pixel pitch must be positive and finite");
  if (!std::isfinite(g->off_u) || !std::isfinite(g->off_v))
    return fail(FDK_ERR_INVALID_ARG, "principal-point offsets must be finite");
  if (!finite_pos(g->sod) || !finite_pos(g->sdd))
    return fail(FDK_ERR_INVALID_ARG, "sod and sdd must be positive and finite");
  // Table 1: the detector lies beyond the rotation axis (D > d).
  if (!(g->sdd > g->sod))
    return fail(FDK_ERR_INVALID_ARG, "sdd = %g must exceed sod = %g", g->sdd, g->sod);
  if (g->np <= 0) return fail(FDK_ERR_INVALID_ARG, "np must be positive (got %d)", g->np);
  if (!g->angles) return fail(FDK_ERR_INVALID_ARG, "angles pointer is NULL");
  // Eq. 3: z = d + sin(b) X + cos(b) Y; its minimum over the voxel centres
  // is at least d minus the half-diagonal of the x-y grid of centres.
  const double r = 0.5 * std::hypot((g->nx - 1) * g->dx, (g->ny - 1) * g->dy);
  const double zmin = g->sod - r;
  if (!(zmin > 1e-6 * g->sod))
    return fail(FDK_ERR_INVALID_ARG,
                "sod = %g does not exceed the volume's x-y half-diagonal %g: some voxel has z <= 0",
                g->sod, r);
  const double umax = std::fabs((g->nu - 1) * 0.5 + g->off_u) + g->sdd / g->du * r / zmin;
  const double vmax = std::fabs((g->nv - 1) * 0.5 + g->off_v) +
                      g->sdd * g->dz / g->dv * (0.5 * (g->nz - 1)) / zmin;
  if (!(umax < kMaxCoord) || !(vmax < kMaxCoord))
    return fail(FDK_ERR_INVALID_ARG, "geometry maps voxels too far off the detector (%g, %g px)",
                umax, vmax);
  return FDK_OK;
}

fdk_status check_views(const fdk_geometry* g, int32_t view0, int32_t nviews) {
  if (view0 < 0 || nviews < 0 || (int64_t)view0 + nviews > g->np)
    return fail(FDK_ERR_INVALID_ARG, "view range [%d, %d + %d) is outside [0, %d)", view0, view0,
                nviews, g->np);
  for (int32_t s = view0; s < view0 + nviews; ++s)
    if (!std::isfinite(g->angles[s]))
      return fail(FDK_ERR_INVALID_ARG, "angle of view %d is not finite", s);
  return FDK_OK;
}

// Views per launch: the fewest launches of at most `cap` views, split
// evenly (a short last launch would read and write the volume for few
// views).
int32_t views_per_launch(int32_t nviews, int32_t cap) {
  const int32_t n = (nviews + cap - 1) / cap;
  return n > 0 ? (nviews + n - 1) / n : cap;
}

// Views per launch of the adjoint: up to kMaxViewsPerLaunch when every
// launch's views then span at most kFpWideSpanRad of angle, else up to
// kFpViewsPerLaunch.
int32_t adjoint_views_per_launch(const double* angles, int32_t nviews) {
  const int32_t wide = views_per_launch(nviews, fdk::kMaxViewsPerLaunch);
  for (int32_t b = 0; b < nviews; b += wide) {
    const int32_t n = std::min(wide, nviews - b);
    const auto [lo, hi] = std::minmax_element(angles + b, angles + b + n);
    if (*hi - *lo > fdk::kFpWideSpanRad) return views_per_launch(nviews, fdk::kFpViewsPerLaunch);
  }
  return wide;
}

// Adjoint slot rotation: the order in which each lane visits its 16 slots.
// The tiled adjoint is bound by LDS bank conflicts among the 64 lanes of each
// atomic add, and which rotation spreads them best depends on the view
// angle (at 2048^3, 32-view batches took 201-339 ms with (tx + 4 ty) and
// 201-248 ms with the best of four rotations). For large launches the host
// scores the candidates with a model of the adds' addresses: per wave
// instruction, the most lanes that fall in one of the 64 four-byte banks,
// summed over sample bricks and views. A uniform shift of all addresses
// leaves that count unchanged, so tile origins are not needed.
constexpr int kRotCand[4][2] = {{1, 4}, {1, 5}, {3, 4}, {5, 4}};
constexpr double kRotTuneMinWork = 2147483648.0;  // voxel-view updates per launch (2^31)
constexpr double kRotSwitchRatio = 0.95;

double rotation_cost(const fdk::GeoConst& gc, const fdk::ViewGeo& v, int32_t pitch, int32_t i_lo,
                     int32_t j_lo, int32_t kb, int ra, int rb) {
  double cost = 0.0;
  int32_t base[64], rot[64];
  double fvb[64], dvk[64];
  for (int w = 0; w < 4; ++w) {
    for (int l = 0; l < 64; ++l) {
      const int tid = 64 * w + l, tx = tid % 16, ty = tid / 16;
      const double i = std::min(i_lo + tx, gc.nx - 1), j = std::min(j_lo + ty, gc.ny - 1);
      const double z = v.ci * i + v.cj * j + v.c0;
      const double u = gc.cu + gc.ku * (v.ai * i + v.aj * j + v.a0) / z;
      const double v0 = gc.cv + gc.kv * (kb - gc.cz) / z;
      const double nvb = std::floor(v0);
      base[l] = static_cast<int32_t>(std::floor(u)) * pitch + static_cast<int32_t>(nvb);
      fvb[l] = v0 - nvb;
      dvk[l] = gc.kv / z;
      rot[l] = (ra * tx + rb * (ty & 3)) & 15;
    }
    for (int t = 0; t < 16; ++t) {
      int32_t addr[64];
      for (int l = 0; l < 64; ++l)
        addr[l] = base[l] + static_cast<int32_t>(std::floor(fvb[l] + ((t + rot[l]) & 15) * dvk[l]));
      const int32_t offs[4] = {0, pitch, 1, pitch + 1};  // the four taps of a splat
      for (int32_t off : offs) {
        int hist[64] = {0}, mx = 0;
        for (int l = 0; l < 64; ++l) mx = std::max(mx, ++hist[(addr[l] + off) & 63]);
        cost += mx;
      }
    }
  }
  return cost;
}

// Picks ts->rot_a, rot_b for one adjoint launch (FDK_FP_ROT=a,b forces a
// choice: a tuning aid).
void choose_rotation(const fdk::GeoConst& gc, const fdk::SliceRun& r, const fdk::ViewBatch& vb,
                     int32_t bz, fdk::TileShape* ts) {
  if (const char* env = std::getenv("FDK_FP_ROT")) {
    int a = 1, b = 4;
    if (std::sscanf(env, "%d,%d", &a, &b) == 2) {
      ts->rot_a = a;
      ts->rot_b = b;
    }
    return;
  }
  if (ts->vc <= 0 || vb.nviews <= 0) return;  // the direct variant adds to global memory
  if (static_cast<double>(gc.nx) * gc.ny * r.n * vb.nviews < kRotTuneMinWork) return;
  static const double kFrac[5][3] = {
      {0.1, 0.15, 0.0}, {0.5, 0.5, 0.5}, {0.8, 0.25, 0.95}, {0.95, 0.95, 0.06}, {0.3, 0.7, 0.3}};
  const int32_t views[3] = {0, vb.nviews / 2, vb.nviews - 1};
  double cost0 = 0.0, best = 0.0;
  int bi = 0;
  for (int c = 0; c < 4; ++c) {
    double cost = 0.0;
    for (int32_t s : views) {
      for (const auto& f : kFrac) {
        const int32_t bx = static_cast<int32_t>(f[0] * (ts->nbx - 1));
        const int32_t by = static_cast<int32_t>(f[1] * (ts->nby - 1));
        const int32_t seg = static_cast<int32_t>(f[2] * (ts->nseg - 1));
        cost += rotation_cost(gc, fdk::view_geo(gc, vb.sn[s], vb.cs[s]), ts->tvp, bx * fdk::kBrickX, by * fdk::kBrickY,
                              r.k_first + seg * bz, kRotCand[c][0], kRotCand[c][1]);
      }
    }
    if (c == 0) cost0 = cost;
    if (c == 0 || cost < best) {
      best = cost;
      bi = c;
    }
  }
  // The model ranks close candidates unreliably: leave the default unless
  // another is clearly better.
  if (best > kRotSwitchRatio * cost0) bi = 0;
  ts->rot_a = kRotCand[bi][0];
  ts->rot_b = kRotCand[bi][1];
}

struct Slab {
  std::vector<fdk::SliceRun> runs;
};

// Split the slab's slices into mirrored pairs (Theorem 1, Alg. 4's k < Nz/2
// loop) and plain runs for slices without an in-slab mirror.
fdk_status make_slab(const fdk_geometry* g, const fdk::GeoConst& gc, int32_t z0, int32_t nzl,
                     int32_t kind, Slab* out) {
  const int32_t nz = g->nz;
  if (kind != FDK_SLAB_CONTIGUOUS && kind != FDK_SLAB_MIRROR_PAIR)
    return fail(FDK_ERR_UNSUPPORTED, "unknown slab kind %d", (int)kind);
  if (z0 < 0 || nzl <= 0) return fail(FDK_ERR_INVALID_ARG, "slab z0 = %d, nz_local = %d", z0, nzl);
  const bool can_mirror = gc.mirror_g != INT32_MIN;
  std::vector<int32_t> loc(nz, -1);  // global slice -> slab slice
  if (kind == FDK_SLAB_CONTIGUOUS) {
    if ((int64_t)z0 + nzl > nz)
      return fail(FDK_ERR_INVALID_ARG, "slab [%d, %d) exceeds Nz = %d", z0, z0 + nzl, nz);
    for (int32_t t = 0; t < nzl; ++t) loc[z0 + t] = t;
  } else {
    if (nzl % 2) return fail(FDK_ERR_INVALID_ARG, "mirror-pair slab needs an even nz_local");
    const int32_t h = nzl / 2;
    if ((int64_t)z0 + h > (int64_t)nz - z0 - h)
      return fail(FDK_ERR_INVALID_ARG, "mirror-pair halves [%d, %d) and [%d, %d) overlap", z0,
                  z0 + h, nz - z0 - h, nz - z0);
    for (int32_t t = 0; t < h; ++t) {
      loc[z0 + t] = t;
      loc[nz - z0 - h + t] = h + t;
    }
  }
  std::vector<char> done(nz, 0);
  out->runs.clear();
  // Mirrored pairs: lower slice k < Nz/2 whose mirror is also held, both
  // slab-contiguous in the directions the kernel walks.
  if (can_mirror) {
    int32_t k = 0;
    while (k < nz / 2) {
      if (loc[k] < 0 || loc[nz - 1 - k] < 0) {
        ++k;
        continue;
      }
      fdk::SliceRun r{k, 1, loc[k], loc[nz - 1 - k], 1};
      while (k + r.n < nz / 2 && loc[k + r.n] == r.loc_lo + r.n &&
             loc[nz - 1 - k - r.n] == r.loc_hi - r.n)
        ++r.n;
      for (int32_t t = 0; t < r.n; ++t) done[k + t] = done[nz - 1 - k - t] = 1;
      out->runs.push_back(r);
      k += r.n;
    }
  }
  for (int32_t k = 0; k < nz;) {
    if (loc[k] < 0 || done[k]) {
      ++k;
      continue;
    }
    fdk::SliceRun r{k, 1, loc[k], loc[k], 0};
    while (k + r.n < nz && loc[k + r.n] == r.loc_lo + r.n && !done[k + r.n]) ++r.n;
    out->runs.push_back(r);
    k += r.n;
  }
  return FDK_OK;
}

size_t dtype_size(fdk_dtype t) { return t == FDK_F32 ? 4 : 2; }

}  // namespace

extern "C" {

const char* fdk_last_error(void) { return g_last_error.c_str(); }

fdk_status fdk_projection_matrix(const fdk_geometry* g, int32_t view, double* P) {
  fdk_status st = check_geometry(g);
  if (st != FDK_OK) return st;
  if ((st = check_views(g, view, 1)) != FDK_OK) return st;
  if (!P) return fail(FDK_ERR_INVALID_ARG, "matrix pointer is NULL");
  // The kernels' own constants: z = ci i + cj j + c0, u = cu + ku a / z,
  // v = cv + kv (k - cz) / z, a = ai i + aj j + a0.
  const fdk::GeoConst gc = make_geo(g);
  const fdk::ViewGeo vg = make_view(g, g->angles[view]);
  const double zr[4] = {vg.ci, vg.cj, 0.0, vg.c0};
  const double ar[4] = {vg.ai, vg.aj, 0.0, vg.a0};
  const double kr[4] = {0.0, 0.0, 1.0, -gc.cz};
  for (int c = 0; c < 4; ++c) {
    P[c] = gc.cu * zr[c] + gc.ku * ar[c];
    P[4 + c] = gc.cv * zr[c] + gc.kv * kr[c];
    P[8 + c] = zr[c];
  }
  return ok();
}

double fdk_fdk_scale(const fdk_geometry* g) {
  if (!g || g->np <= 0 || !std::isfinite(g->sod)) return std::nan("");
  return M_PI * g->sod * g->sod / g->np;
}

fdk_status fdk_backproject(const fdk_geometry* g, int32_t view0, int32_t nviews, const void* q,
                           fdk_dtype q_dtype, float* vol, int32_t z0, int32_t nz_local,
                           fdk_slab_kind slab, float scale, uint32_t flags, void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  const int32_t qd = raw(q_dtype);
  if (qd != FDK_F32 && qd != FDK_F16 && qd != FDK_BF16)
    return fail(FDK_ERR_UNSUPPORTED, "unknown projection dtype %d", qd);
  if (!vol) return fail(FDK_ERR_INVALID_ARG, "volume pointer is NULL");
  if (nviews > 0 && !q) return fail(FDK_ERR_INVALID_ARG, "projection pointer is NULL");
  if (!std::isfinite(scale)) return fail(FDK_ERR_INVALID_ARG, "scale is not finite");
  if (flags & ~(FDK_ACCUMULATE | FDK_DIRECT))
    return fail(FDK_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  const bool acc0 = flags & FDK_ACCUMULATE;
  const bool direct = flags & FDK_DIRECT;
  const int64_t slice = (int64_t)g->nx * g->ny;
  if (nviews == 0) {
    if (!acc0) {
      if (int e = fdk::launch_fill_zero(vol, slice * nz_local, stream))
        return fail(FDK_ERR_HIP, "zero fill failed: HIP error %d", e);
    }
    return ok();
  }
  const int64_t vstride = (int64_t)g->nu * g->nv;
  fdk::ViewBatch vb;
  const int32_t per = views_per_launch(nviews, fdk::kMaxViewsPerLaunch);
  for (int32_t b = 0; b < nviews; b += per) {
    vb.nviews = std::min(per, nviews - b);
    for (int32_t s = 0; s < vb.nviews; ++s) fdk::set_view(&vb, s, g->angles[view0 + b + s]);
    const char* qb = static_cast<const char*>(q) + (size_t)b * vstride * dtype_size(q_dtype);
    for (const fdk::SliceRun& r : sl.runs) {
      const fdk::TileShape ts =
          r.mirror ? fdk::tile_shape(g, gc, r, vb, fdk::kBrickZ, fdk::kTileEntryBytes,
                                     fdk::kPrefetchSlots, direct, true, true)
                   : fdk::tile_shape(g, gc, r, vb, fdk::kPlainBrickZ, fdk::kPlainEntryBytes,
                                     fdk::kPlainPrefetchSlots, direct, true);
      if (int e = fdk::launch_backproject(gc, r, vb, ts, qb, q_dtype, vstride, vol, scale,
                                          (b > 0) || acc0, stream))
        return fail(FDK_ERR_HIP, "back-projection launch failed: HIP error %d", e);
    }
  }
  return ok();
}

fdk_status fdk_forward_project(const fdk_geometry* g, int32_t view0, int32_t nviews,
                               const float* vol, int32_t z0, int32_t nz_local,
                               fdk_slab_kind slab, float* q, float scale, uint32_t flags,
                               void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  if (!vol) return fail(FDK_ERR_INVALID_ARG, "volume pointer is NULL");
  if (nviews > 0 && !q) return fail(FDK_ERR_INVALID_ARG, "projection pointer is NULL");
  if (!std::isfinite(scale)) return fail(FDK_ERR_INVALID_ARG, "scale is not finite");
  if (flags & ~(FDK_ACCUMULATE | FDK_DIRECT | FDK_FIXED_SUMS))
    return fail(FDK_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  if (nviews == 0) return ok();
  const bool direct = flags & FDK_DIRECT;
  const bool fixed_sums = flags & FDK_FIXED_SUMS;
  const int64_t vstride = (int64_t)g->nu * g->nv;
  if (!(flags & FDK_ACCUMULATE)) {
    if (int e = fdk::launch_fill_zero(q, vstride * nviews, stream))
      return fail(FDK_ERR_HIP, "zero fill failed: HIP error %d", e);
  }
  fdk::ViewBatch vb;
  const int32_t per = adjoint_views_per_launch(g->angles + view0, nviews);
  for (int32_t b = 0; b < nviews; b += per) {
    vb.nviews = std::min(per, nviews - b);
    for (int32_t s = 0; s < vb.nviews; ++s) fdk::set_view(&vb, s, g->angles[view0 + b + s]);
    for (const fdk::SliceRun& r : sl.runs) {
      // Plain runs: 32-slice bricks and a single accumulation plane; their
      // flush has no prefetch budget to respect.
      fdk::TileShape ts =
          r.mirror ? fdk::tile_shape(g, gc, r, vb, fdk::kBrickZ, fdk::kTileEntryBytes,
                                     fdk::kPrefetchSlots, direct)
                   : fdk::tile_shape(g, gc, r, vb, fdk::kPlainBrickZ, fdk::kPlainEntryBytes,
                                     std::numeric_limits<int32_t>::max(), direct);
      choose_rotation(gc, r, vb, r.mirror ? fdk::kBrickZ : fdk::kPlainBrickZ, &ts);
      if (int e = fdk::launch_forward_project(gc, r, vb, ts, vol, q + (size_t)b * vstride,
                                              vstride, scale, fixed_sums, stream))
        return fail(FDK_ERR_HIP, "forward-projection launch failed: HIP error %d", e);
    }
  }
  return ok();
}

namespace {
// Filtering of a row band, or its adjoint (FP32 output only).
fdk_status filter_rows(const fdk_geometry* g, int32_t view0, int32_t nviews, int32_t v0,
                       int32_t nrows, const float* e, int64_t e_view_stride, void* q,
                       int64_t q_view_stride, int32_t out_dtype_raw, int32_t kind_raw,
                       bool adjoint, void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  if (out_dtype_raw != FDK_F32 && out_dtype_raw != FDK_F16 && out_dtype_raw != FDK_BF16)
    return fail(FDK_ERR_UNSUPPORTED, "unknown output dtype %d", out_dtype_raw);
  if (kind_raw != FDK_RAMLAK && kind_raw != FDK_SHEPP_LOGAN)
    return fail(FDK_ERR_UNSUPPORTED, "unknown filter kind %d", kind_raw);
  const fdk_dtype out_dtype = static_cast<fdk_dtype>(out_dtype_raw);
  const fdk_filter_kind kind = static_cast<fdk_filter_kind>(kind_raw);
  if (g->nu > 8192) return fail(FDK_ERR_UNSUPPORTED, "filter rows above 8192 pixels (Nu = %d)", g->nu);
  if (v0 < 0 || nrows < 0 || (int64_t)v0 + nrows > g->nv)
    return fail(FDK_ERR_INVALID_ARG, "row band [%d, %d + %d) is outside [0, %d)", v0, v0, nrows,
                g->nv);
  if (nviews == 0 || nrows == 0) return ok();
  const int64_t band = (int64_t)nrows * g->nu;
  if (e_view_stride < band || q_view_stride < band)
    return fail(FDK_ERR_INVALID_ARG, "view stride smaller than the band (%lld elements)",
                (long long)band);
  if (!e || !q) return fail(FDK_ERR_INVALID_ARG, "projection pointer is NULL");
  const size_t nbytes_in = (size_t)((nviews - 1) * e_view_stride + band) * 4;
  const size_t nbytes_out = (size_t)((nviews - 1) * q_view_stride + band) * dtype_size(out_dtype);
  const char* a = reinterpret_cast<const char*>(e);
  const char* b = static_cast<const char*>(q);
  if (a < b + nbytes_out && b < a + nbytes_in)
    return fail(FDK_ERR_INVALID_ARG, "filter input and output overlap");
  const fdk::GeoConst gc = make_geo(g);
  const fdk::RowBand rb{nviews, v0, nrows, e_view_stride, q_view_stride};
  const int err = adjoint ? fdk::launch_filter_adjoint(gc, g->du, g->dv, g->sod, g->sdd, rb, e,
                                                       static_cast<float*>(q), kind, stream)
                          : fdk::launch_filter(gc, g->du, g->dv, g->sod, g->sdd, rb, e, q,
                                               out_dtype, kind, stream);
  if (err) return fail(FDK_ERR_HIP, "filter launch failed: HIP error %d", err);
  return ok();
}
}  // namespace

fdk_status fdk_filter_rows(const fdk_geometry* g, int32_t view0, int32_t nviews, int32_t v0,
                           int32_t nrows, const float* e, int64_t e_view_stride, void* q,
                           int64_t q_view_stride, fdk_dtype out_dtype, fdk_filter_kind kind,
                           void* stream) {
  return filter_rows(g, view0, nviews, v0, nrows, e, e_view_stride, q, q_view_stride,
                     raw(out_dtype), raw(kind), false, stream);
}

fdk_status fdk_filter_adjoint(const fdk_geometry* g, int32_t view0, int32_t nviews,
                              const float* q_grad, float* e_grad, fdk_filter_kind kind,
                              void* stream) {
  if (!g) return fail(FDK_ERR_INVALID_ARG, "geometry pointer is NULL");
  const int64_t full = (int64_t)g->nu * g->nv;
  return filter_rows(g, view0, nviews, 0, g->nv, q_grad, full, e_grad, full, FDK_F32, raw(kind),
                     true, stream);
}

namespace {
// Voxels in the slab: nz_local * Ny * Nx (after the slab is validated).
int64_t slab_voxels(const fdk_geometry* g, int32_t nz_local) {
  return (int64_t)nz_local * g->ny * g->nx;
}
constexpr float kSirtFloor = 1e-3f;  // sums below this fraction of the largest one are raised to it
constexpr float kMlemFloor = 1e-3f;  // ratio denominators below this fraction of the largest are raised
}  // namespace

fdk_status fdk_sirt_weights(const fdk_geometry* g, int32_t view0, int32_t nviews, int32_t z0,
                            int32_t nz_local, fdk_slab_kind slab, float* row_inv, float* col_inv,
                            float* vol_tmp, void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  if (nviews <= 0) return fail(FDK_ERR_INVALID_ARG, "SIRT needs at least one view");
  if (!row_inv || !col_inv || !vol_tmp) return fail(FDK_ERR_INVALID_ARG, "SIRT buffer pointer is NULL");
  if (col_inv == vol_tmp) return fail(FDK_ERR_INVALID_ARG, "col_inv and vol_tmp must differ");
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  const int64_t nproj = (int64_t)nviews * g->nu * g->nv, nvox = slab_voxels(g, nz_local);
  int e = 0;
  // Column sums B 1 (all-ones projections, held in row_inv for now).
  if ((e = fdk::launch_fill(row_inv, nproj, 1.0f, stream)))
    return fail(FDK_ERR_HIP, "fill failed: HIP error %d", e);
  if ((st = fdk_backproject(g, view0, nviews, row_inv, FDK_F32, col_inv, z0, nz_local, slab, 1.0f,
                            0, stream)))
    return st;
  // Row sums F 1.
  if ((e = fdk::launch_fill(vol_tmp, nvox, 1.0f, stream)))
    return fail(FDK_ERR_HIP, "fill failed: HIP error %d", e);
  if ((st = fdk_forward_project(g, view0, nviews, vol_tmp, z0, nz_local, slab, row_inv, 1.0f, 0,
                                stream)))
    return st;
  // vol_tmp is free again: its first word holds each max-reduction in turn
  // (the two run in stream order, and a slab has at least one voxel).
  uint32_t* scratch = reinterpret_cast<uint32_t*>(vol_tmp);
  if ((e = fdk::launch_invert_floor(row_inv, nproj, kSirtFloor, scratch, stream)) ||
      (e = fdk::launch_invert_floor(col_inv, nvox, kSirtFloor, scratch, stream)))
    return fail(FDK_ERR_HIP, "inversion failed: HIP error %d", e);
  return ok();
}

fdk_status fdk_sirt_iteration(const fdk_geometry* g, int32_t view0, int32_t nviews, const float* p,
                              const float* row_inv, const float* col_inv, float* x, int32_t z0,
                              int32_t nz_local, fdk_slab_kind slab, float lambda, uint32_t flags,
                              float* proj_tmp, float* vol_tmp, void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  if (nviews <= 0) return fail(FDK_ERR_INVALID_ARG, "SIRT needs at least one view");
  if (!p || !row_inv || !col_inv || !x || !proj_tmp || !vol_tmp)
    return fail(FDK_ERR_INVALID_ARG, "SIRT buffer pointer is NULL");
  if (proj_tmp == p || proj_tmp == row_inv || vol_tmp == x || vol_tmp == col_inv)
    return fail(FDK_ERR_INVALID_ARG, "SIRT workspaces must not alias the inputs");
  if (!std::isfinite(lambda)) return fail(FDK_ERR_INVALID_ARG, "lambda is not finite");
  if (flags & ~FDK_NONNEG) return fail(FDK_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  const int64_t nproj = (int64_t)nviews * g->nu * g->nv, nvox = slab_voxels(g, nz_local);
  if ((st = fdk_forward_project(g, view0, nviews, x, z0, nz_local, slab, proj_tmp, 1.0f,
                                FDK_FIXED_SUMS, stream)))
    return st;
  int e = fdk::launch_sirt_residual(p, row_inv, proj_tmp, nproj, stream);
  if (e) return fail(FDK_ERR_HIP, "residual failed: HIP error %d", e);
  if ((st = fdk_backproject(g, view0, nviews, proj_tmp, FDK_F32, vol_tmp, z0, nz_local, slab, 1.0f,
                            0, stream)))
    return st;
  e = fdk::launch_sirt_update(x, col_inv, vol_tmp, nvox, lambda, (flags & FDK_NONNEG) ? 1 : 0,
                              stream);
  if (e) return fail(FDK_ERR_HIP, "update failed: HIP error %d", e);
  return ok();
}

fdk_status fdk_sirt_iteration_noalloc(const fdk_geometry* g, int32_t view0, int32_t nviews,
                                      const float* p, const float* row_inv, const float* col_inv,
                                      float* x, int32_t z0, int32_t nz_local, fdk_slab_kind slab,
                                      float lambda, uint32_t flags, void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  if (nviews <= 0) return fail(FDK_ERR_INVALID_ARG, "SIRT needs at least one view");
  if (!p || !row_inv || !col_inv || !x) return fail(FDK_ERR_INVALID_ARG, "SIRT buffer pointer is NULL");
  if (!std::isfinite(lambda)) return fail(FDK_ERR_INVALID_ARG, "lambda is not finite");
  if (flags & ~FDK_NONNEG) return fail(FDK_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  // Workspace: the projections' residual, then (256-byte aligned) the
  // slab's back-projection, both in the per-GPU static array.
  const int64_t nproj = (int64_t)nviews * g->nu * g->nv;
  const int64_t nvox = slab_voxels(g, nz_local);
  const int64_t vol_off = (nproj + 63) / 64 * 64;
  if (vol_off + nvox > fdk::kStaticScratchFloats)
    return fail(FDK_ERR_INVALID_ARG,
                "workspace of %lld projection and %lld slab values exceeds the static %lld floats",
                (long long)nproj, (long long)nvox, (long long)fdk::kStaticScratchFloats);
  float* ws = nullptr;
  if (int e = fdk::static_scratch(&ws))
    return fail(FDK_ERR_HIP, "static workspace lookup failed: HIP error %d", e);
  return fdk_sirt_iteration(g, view0, nviews, p, row_inv, col_inv, x, z0, nz_local, slab, lambda,
                            flags, ws, ws + vol_off, stream);
}

fdk_status fdk_mlem_iteration(const fdk_geometry* g, int32_t view0, int32_t nviews, const float* p,
                              const float* col_inv, float* x, int32_t z0, int32_t nz_local,
                              fdk_slab_kind slab, float* proj_tmp, float* vol_tmp, void* stream) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if ((st = check_views(g, view0, nviews))) return st;
  if (nviews <= 0) return fail(FDK_ERR_INVALID_ARG, "MLEM needs at least one view");
  if (!p || !col_inv || !x || !proj_tmp || !vol_tmp)
    return fail(FDK_ERR_INVALID_ARG, "MLEM buffer pointer is NULL");
  if (proj_tmp == p || vol_tmp == x || vol_tmp == col_inv)
    return fail(FDK_ERR_INVALID_ARG, "MLEM workspaces must not alias the inputs");
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  const int64_t nproj = (int64_t)nviews * g->nu * g->nv, nvox = slab_voxels(g, nz_local);
  if ((st = fdk_forward_project(g, view0, nviews, x, z0, nz_local, slab, proj_tmp, 1.0f,
                                FDK_FIXED_SUMS, stream)))
    return st;
  // The ratio's max-reduction word lives in vol_tmp, which the
  // back-projection overwrites only afterwards (stream order).
  int e = fdk::launch_mlem_ratio(p, proj_tmp, nproj, kMlemFloor,
                                 reinterpret_cast<uint32_t*>(vol_tmp), stream);
  if (e) return fail(FDK_ERR_HIP, "MLEM ratio failed: HIP error %d", e);
  if ((st = fdk_backproject(g, view0, nviews, proj_tmp, FDK_F32, vol_tmp, z0, nz_local, slab, 1.0f,
                            0, stream)))
    return st;
  e = fdk::launch_mlem_update(x, col_inv, vol_tmp, nvox, stream);
  if (e) return fail(FDK_ERR_HIP, "MLEM update failed: HIP error %d", e);
  return ok();
}

fdk_status fdk_slab_rows(const fdk_geometry* g, int32_t z0, int32_t nz_local, fdk_slab_kind slab,
                         int32_t band[4]) {
  fdk_status st = check_geometry(g);
  if (st) return st;
  if (!band) return fail(FDK_ERR_INVALID_ARG, "band pointer is NULL");
  const fdk::GeoConst gc = make_geo(g);
  Slab sl;
  if ((st = make_slab(g, gc, z0, nz_local, raw(slab), &sl))) return st;
  // Global slice intervals the slab holds.
  int32_t iv[2][2];
  int niv = 1;
  if (slab == FDK_SLAB_CONTIGUOUS) {
    iv[0][0] = z0;
    iv[0][1] = z0 + nz_local - 1;
  } else {
    const int32_t h = nz_local / 2;
    iv[0][0] = z0;
    iv[0][1] = z0 + h - 1;
    iv[1][0] = g->nz - z0 - h;
    iv[1][1] = g->nz - z0 - 1;
    niv = 2;
  }
  // v(k) = cv + kv (k - cz) / z is monotone in k and in 1/z, and z is affine
  // in (i, j), so each view's extremes sit at the slab's end slices and the
  // volume's corner columns. Taps reach floor(v) + 1; one spare row on each
  // side covers the kernels' FP32 rounding of v.
  int32_t lo[2], hi[2];
  for (int n = 0; n < niv; ++n) {
    double vmin = INFINITY, vmax = -INFINITY;
    for (int32_t s = 0; s < g->np; ++s) {
      const fdk::ViewGeo vg = make_view(g, g->angles[s]);
      double zmin = INFINITY, zmax = -INFINITY;
      for (int ci = 0; ci < 2; ++ci)
        for (int cj = 0; cj < 2; ++cj) {
          const double z = vg.c0 + vg.ci * (ci ? g->nx - 1 : 0) + vg.cj * (cj ? g->ny - 1 : 0);
          zmin = std::fmin(zmin, z);
          zmax = std::fmax(zmax, z);
        }
      for (int e = 0; e < 2; ++e) {
        const double dk = iv[n][e] - gc.cz;
        for (double z : {zmin, zmax}) {
          const double v = gc.cv + gc.kv * dk / z;
          vmin = std::fmin(vmin, v);
          vmax = std::fmax(vmax, v);
        }
      }
    }
    lo[n] = static_cast<int32_t>(std::max(0.0, std::floor(vmin) - 1.0));
    hi[n] = static_cast<int32_t>(std::min<double>(g->nv - 1, std::floor(vmax) + 2.0));
  }
  // Non-empty intervals in ascending order, merged where they touch.
  std::vector<std::pair<int32_t, int32_t>> rows;
  for (int n = 0; n < niv; ++n)
    if (lo[n] <= hi[n]) rows.emplace_back(lo[n], hi[n]);
  std::sort(rows.begin(), rows.end());
  if (rows.size() == 2 && rows[1].first <= rows[0].second + 1) {
    rows[0].second = std::max(rows[0].second, rows[1].second);
    rows.pop_back();
  }
  band[0] = band[1] = band[2] = band[3] = 0;
  for (size_t n = 0; n < rows.size(); ++n) {
    band[2 * n] = rows[n].first;
    band[2 * n + 1] = rows[n].second - rows[n].first + 1;
  }
  return ok();
}


fdk_status fdk_filter(const fdk_geometry* g, int32_t view0, int32_t nviews, const float* e,
                      void* q, fdk_dtype out_dtype, fdk_filter_kind kind, void* stream) {
  if (!g) return fail(FDK_ERR_INVALID_ARG, "geometry pointer is NULL");
  const int64_t full = (int64_t)g->nu * g->nv;
  return filter_rows(g, view0, nviews, 0, g->nv, e, full, q, full, raw(out_dtype), raw(kind), false,
                     stream);
}

}  // extern "C"
