// Host check of the LDS tile bounds of the tiled back-projector and its
// adjoint: for seeded random geometries, every tap of every voxel of every
// brick, computed with the kernels' own brick setup and FP32 column
// arithmetic (brick.h, built for the host), must fall inside the tile that
// the host sizing (tiles.cpp) allots. A short tile would not fault: the
// back-projector clamps the tap column and the staged rows would simply be
// the wrong ones, so only a check like this one can catch it.
//
// Usage: tile_bounds_check SEED COUNT
// Prints one line per kind of run: "<kind> geometries=.. tiled=.. direct=..
// columns=.. col_viol=.. row_viol=.. neg=.. min_col_slack=.. min_row_slack=..".
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1909_02724_amd/csrc/brick.h"
#include "../paper_1909_02724_amd/csrc/geometry_host.h"

namespace {

struct SplitMix64 {  // Steele, Lea and Flood (2014)
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uni() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  double uni(double a, double b) { return a + (b - a) * uni(); }
  int irange(int a, int b) { return a + static_cast<int>(next() % static_cast<uint64_t>(b - a + 1)); }
};

struct Stats {
  long geometries = 0, tiled = 0, direct = 0, columns = 0;
  long col_viol = 0, row_viol = 0, neg = 0;
  int min_col_slack = 1 << 30, min_row_slack = 1 << 30;
};

// One launch's worth of checks for a slice run of a geometry.
void check_run(const fdk_geometry& g, const fdk::GeoConst& gc, const fdk::SliceRun& run,
               const fdk::ViewBatch& vb, Stats* st) {
  using namespace fdk;
  const bool mirror = run.mirror != 0;
  const int32_t bz = mirror ? kBrickZ : kPlainBrickZ;
  const TileShape ts = mirror ? tile_shape(&g, gc, run, vb, bz, kTileEntryBytes, kPrefetchSlots, false,
                                           true, true)
                              : tile_shape(&g, gc, run, vb, bz, kPlainEntryBytes,
                                           kPlainPrefetchSlots, false, true);
  ++st->geometries;
  if (ts.vc <= 0) {
    ++st->direct;
    return;
  }
  ++st->tiled;
  const float kvf = static_cast<float>(gc.kv);
  for (int32_t s = 0; s < vb.nviews; ++s) {
    for (int32_t seg = 0; seg < ts.nseg; ++seg) {
      const int32_t kb = run.k_first + seg * bz;
      for (int32_t by = 0; by < ts.nby; ++by) {
        for (int32_t bx = 0; bx < ts.nbx; ++bx) {
          const int32_t i_lo = bx * kBrickX, j_lo = by * kBrickY;
          const int32_t i_hi = std::min(i_lo + kBrickX - 1, gc.nx - 1);
          const int32_t j_hi = std::min(j_lo + kBrickY - 1, gc.ny - 1);
          const BrickView b = brick_setup(gc, fdk::view_geo(gc, vb.sn[s], vb.cs[s]), i_lo, i_hi, j_lo, j_hi, kb, ts.tu,
                                          ts.tv, bz, mirror);
          // Every thread of the workgroup computes a column, owners and the
          // clamped non-owners alike, so all 256 are checked.
          for (int32_t ty = 0; ty < kBrickY; ++ty) {
            for (int32_t tx = 0; tx < kBrickX; ++tx) {
              const int32_t i = std::min(i_lo + tx, i_hi), j = std::min(j_lo + ty, j_hi);
              const float txf = static_cast<float>(i - i_lo), tyf = static_cast<float>(j - j_lo);
              // ul and vl must not be negative: the kernels convert them to
              // unsigned indices.
              const float f = rcp_f32(b.zo + fmaf(b.ci, txf, b.cj * tyf));
              const float ul = fmaf(fmaf(b.au, txf, b.bu * tyf), f, b.uo);
              const float vl = fmaf(fmaf(b.av, txf, b.bv * tyf), f, b.vo);
              if (!(ul >= 0.0f) || !(vl >= 0.0f)) {
                ++st->neg;
                continue;
              }
              const ColumnF32 c = column_f32(b, txf, tyf, kvf);
              ++st->columns;
              // Entry nu holds q(nu) and q(nu + 1): nu < tu. (The adjoint's
              // tile has tu + 1 columns for the same taps.)
              const int col_slack = ts.tu - 1 - static_cast<int>(c.nu);
              // v grows with the slot: the last voxel reads the highest row,
              // nvb + dn + 1 < tv.
              uint32_t dn = 0;
              float fr = 0.0f;
              voxel_row_off(c.fvb, c.dvk, bz - 1, &dn, &fr);
              const int row_slack = ts.tv - 1 - static_cast<int>(c.nvb + dn + 1);
              if (col_slack < 0) ++st->col_viol;
              if (row_slack < 0) ++st->row_viol;
              st->min_col_slack = std::min(st->min_col_slack, col_slack);
              st->min_row_slack = std::min(st->min_row_slack, row_slack);
            }
          }
        }
      }
    }
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 3) {
    std::fprintf(stderr, "usage: %s SEED COUNT\n", argv[0]);
    return 2;
  }
  SplitMix64 rng{std::strtoull(argv[1], nullptr, 10)};
  const long count = std::strtol(argv[2], nullptr, 10);
  Stats mir, pln;
  std::vector<double> ang(fdk::kMaxViewsPerLaunch);
  for (long n = 0; n < count; ++n) {
    fdk_geometry g{};
    g.nx = rng.irange(1, 120);
    g.ny = rng.irange(1, 120);
    g.nz = rng.irange(1, 80);
    g.dx = rng.uni(0.4, 2.0);
    g.dy = rng.uni(0.4, 2.0);
    g.dz = rng.uni(0.4, 2.0);
    g.nu = rng.irange(2, 500);
    g.nv = rng.irange(2, 500);
    // Principal point: centred, shifted by whole or half pixels (a
    // pixel-aligned mirror), or shifted by a fraction (no mirror).
    const int kind = rng.irange(0, 2);
    g.off_u = rng.uni(-4.0, 4.0);
    g.off_v = kind == 0 ? 0.0 : kind == 1 ? 0.5 * rng.irange(-8, 8) : rng.uni(-4.0, 4.0);
    const double r = 0.5 * std::hypot((g.nx - 1) * g.dx, (g.ny - 1) * g.dy);
    g.sod = std::max(r, 0.5) * rng.uni(1.05, 12.0) + 1.0;
    g.sdd = g.sod * rng.uni(1.05, 4.0);
    // Pixel pitch from a magnification of 0.3 to 3 pixels per voxel at the
    // rotation axis (the larger ones exceed the LDS budget: direct variant).
    const double mag = g.sdd / g.sod;
    g.du = mag * g.dx / rng.uni(0.3, 3.0);
    g.dv = mag * g.dz / rng.uni(0.3, 3.0);
    const int nviews = rng.irange(1, fdk::kMaxViewsPerLaunch);
    for (int s = 0; s < nviews; ++s) ang[s] = rng.uni(0.0, 6.283185307179586);
    g.np = nviews;
    g.angles = ang.data();
    const fdk::GeoConst gc = fdk::make_geo(&g);
    fdk::ViewBatch vb{};
    vb.nviews = nviews;
    for (int s = 0; s < nviews; ++s) fdk::set_view(&vb, s, ang[s]);
    // The runs the front end makes for the whole volume: mirrored pairs of
    // the lower half when the mirror is pixel-aligned (plus an odd middle
    // slice), else one plain run; and a plain run over every slice.
    if (gc.mirror_g != INT32_MIN && g.nz >= 2) {
      const fdk::SliceRun r1{0, g.nz / 2, 0, g.nz - 1, 1};
      check_run(g, gc, r1, vb, &mir);
    }
    const fdk::SliceRun r2{0, g.nz, 0, 0, 0};
    check_run(g, gc, r2, vb, &pln);
  }
  const Stats* all[2] = {&mir, &pln};
  const char* names[2] = {"mirror", "plain"};
  for (int k = 0; k < 2; ++k) {
    const Stats& s = *all[k];
    std::printf("%s geometries=%ld tiled=%ld direct=%ld columns=%ld col_viol=%ld row_viol=%ld "
                "neg=%ld min_col_slack=%d min_row_slack=%d\n",
                names[k], s.geometries, s.tiled, s.direct, s.columns, s.col_viol, s.row_viol,
                s.neg, s.min_col_slack, s.min_row_slack);
  }
  return 0;
}
