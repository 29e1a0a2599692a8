// Host-side geometry shared by the front end and the tile-bound test:
// launch-invariant constants and the per-view FP64 coefficients of the
// reduced-cost mapping (Eq. 2 expanded in the form of Eq. 3 and
// Theorems 2, 3).
#pragma once

#include <cmath>
#include <cstdint>

#include "fdk_internal.h"

namespace fdk {

inline GeoConst make_geo(const fdk_geometry* g) {
  GeoConst gc;
  gc.nx = g->nx;
  gc.ny = g->ny;
  gc.nz = g->nz;
  gc.nu = g->nu;
  gc.nv = g->nv;
  gc.cu = 0.5 * (g->nu - 1) + g->off_u;
  gc.cv = 0.5 * (g->nv - 1) + g->off_v;
  gc.cz = 0.5 * (g->nz - 1);
  gc.ku = g->sdd / g->du;
  gc.kv = g->sdd * g->dz / g->dv;
  // Theorem 1 with a shifted principal point: v(Nz-1-k) = 2 cv - v(k). The
  // mirrored taps line up with whole pixels only when 2 cv is an integer.
  const double G = (g->nv - 1) + 2.0 * g->off_v;
  gc.mirror_g = (std::fabs(G - std::nearbyint(G)) <= 1e-9) ? (int32_t)std::nearbyint(G) : INT32_MIN;
  gc.dx = g->dx;
  gc.dy = g->dy;
  gc.d = g->sod;
  gc.ox = 0.5 * (g->nx - 1);
  gc.oy = 0.5 * (g->ny - 1);
  return gc;
}

// Eq. 2 expanded for one gantry angle (view_geo).
inline ViewGeo make_view(const fdk_geometry* g, double beta) {
  return view_geo(make_geo(g), std::sin(beta), std::cos(beta));
}

// Sets view s of a launch to the gantry angle beta.
inline void set_view(ViewBatch* vb, int32_t s, double beta) {
  vb->sn[s] = std::sin(beta);
  vb->cs[s] = std::cos(beta);
}

}  // namespace fdk
