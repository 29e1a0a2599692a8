// Host-side sizing of the back-projection and adjoint tiles: a bound on the
// detector footprint of one brick over the views of a launch, and the
// staging layout derived from it. Host code only (it is also built into the
// tile-bound test, which checks it against every voxel's taps).
#include <algorithm>
#include <cmath>

#include "fdk_internal.h"

namespace fdk {

// Host-side bound of a brick's footprint (pixels) over the views of a
// launch, from derivative bounds over the whole volume: with r the x-y
// half-diagonal and zmin = d - r,
//   |du/di| <= ku Dx (|cos| + |sin| r / zmin) / zmin,
//   |du/dj| <= ku Dy (|sin| + |cos| r / zmin) / zmin,
// and v(k) - cv = kv (k - cz) / z, so over the brick's bz slices and its z
// spread dz the rows span at most kv ((bz - 1) / zmin + |k - cz| dz / zmin^2).
TileShape tile_shape(const fdk_geometry* g, const GeoConst& gc, const SliceRun& run,
                     const ViewBatch& vb, int32_t bz, int32_t entry_bytes, int32_t slots,
                     bool direct, bool bp_staging, bool read_pitch) {
  TileShape ts{};
  ts.rot_a = 1;
  ts.rot_b = 4;
  ts.nbx = (gc.nx + kBrickX - 1) / kBrickX;
  ts.nby = (gc.ny + kBrickY - 1) / kBrickY;
  ts.nseg = (run.n + bz - 1) / bz;
  const double r = 0.5 * std::hypot((g->nx - 1) * g->dx, (g->ny - 1) * g->dy);
  const double zmin = g->sod - r, rho = r / zmin;
  if (direct) return ts;  // vc = 0: direct variant
  const double kmax = gc.cz + bz;
  double wu = 0.0, wv = 0.0;
  for (int32_t s = 0; s < vb.nviews; ++s) {
    const double as = std::fabs(vb.sn[s]), ac = std::fabs(vb.cs[s]);
    const double dui = gc.ku * g->dx * (ac + as * rho) / zmin;
    const double duj = gc.ku * g->dy * (as + ac * rho) / zmin;
    wu = std::fmax(wu, (kBrickX - 1) * dui + (kBrickY - 1) * duj);
    const double dz = (kBrickX - 1) * g->dx * as + (kBrickY - 1) * g->dy * ac;
    wv = std::fmax(wv, gc.kv * ((bz - 1) / zmin + kmax * dz / (zmin * zmin)));
  }
  // floor() of the extremes adds one pixel, the second tap one row, the
  // origin margin one pixel, FP32 column arithmetic up to one more.
  ts.tu = static_cast<int32_t>(std::ceil(wu)) + 4;
  ts.tv = static_cast<int32_t>(std::ceil(wv)) + 5;
  ts.tvp = ts.tv | 1;  // odd pitch: 16 neighbouring columns hit distinct LDS banks
  if (read_pitch) {
    // The back-projector's 16-byte entry reads are served 16 lanes at a
    // time over 64 four-byte banks, and those 16 lanes cover a 4 x 4 patch
    // of voxel columns: a few tile columns, rows n and n + 1. With the pitch
    // at 7 or 9 mod 16, entries nu tvp + n of two such lanes share a bank
    // only if their columns are 7 or more apart.
    while (ts.tvp % 16 != 7 && ts.tvp % 16 != 9) ts.tvp += 2;
  }
  if (bp_staging) {
    // The back-projector stages a tile row with a group of 32 or 64 lanes
    // (one wave at most): a lane per column and one more.
    if (ts.tu + 1 > kWaveLanes) return ts;
    ts.rstep = kBrickThreads / (ts.tu + 1 <= kWaveLanes / 2 ? kWaveLanes / 2 : kWaveLanes);
  } else {
    // The adjoint's flush: a thread per column.
    if (ts.tu + 1 > kBrickThreads) return ts;
    ts.rstep = kBrickThreads / ts.tu;
  }
  ts.rows = (ts.tv + ts.rstep - 1) / ts.rstep;
  const int64_t per_view = static_cast<int64_t>(ts.tu) * ts.tvp * entry_bytes;
  if (!bp_staging) {
    const int64_t vc = std::min<int64_t>({kMaxStageViews, kTileLdsBytes / per_view, slots / ts.rows});
    ts.vc = static_cast<int32_t>(std::max<int64_t>(vc, 0));
    return ts;
  }
  // Back-projector: the five-wave kernel (slots prefetch slots, 27.5 KB of
  // tiles) when it stages all kBpStageViews views per stage, else the
  // four-wave one (more slots and 35.5 KB) if that stages more.
  const int64_t vc5 = std::min<int64_t>({kBpStageViews, kBpTileLdsBytes / per_view, slots / ts.rows});
  const int64_t wide_slots = static_cast<int64_t>(slots) * kWidePrefetchSlots / kPrefetchSlots;
  const int64_t vc4 = std::min<int64_t>({kBpStageViews, kTileLdsBytes / per_view, wide_slots / ts.rows});
  ts.wide = vc5 < kBpStageViews && vc4 > vc5;
  ts.vc = static_cast<int32_t>(std::max<int64_t>(ts.wide ? vc4 : vc5, 0));
  return ts;
}

}  // namespace fdk
