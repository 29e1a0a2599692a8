"""Seeded synthetic inputs for the FDK back-projection workloads.

This module only *generates inputs*: scan geometries, view angles, random
ellipsoid phantoms and voxel samples. It holds none of the reconstruction
arithmetic (no projection matrices, no interpolation, no filtering), so the
GPU path and the CPU oracle can both take their inputs from here without
sharing any of the method.

The paper measures on filtered projections of the Shepp-Logan phantom made
with a forward projector it does not ship (Sec. 5.1); its reported
performance does not depend on content. Seeded sums of random ellipsoids
with additive densities stand in for that phantom: the same structure
(piecewise-constant ellipsoids), the paper's problem sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace

import numpy as np

__all__ = [
    "Geom", "CONFIGS", "config", "angles", "ellipsoids", "ball",
    "sample_voxels", "random_projections", "normal_draws",
]


@dataclass(frozen=True)
class Geom:
    """Circular cone-beam scan (Table 1). All lengths share one unit.

    nx, ny, nz : voxel counts; dx, dy, dz : voxel pitch
    nu, nv     : detector pixel counts; du, dv : pixel pitch
    off_u/off_v: principal-point shift in pixels (0 in the paper)
    sod        : d, source to rotation axis; sdd : D, source to detector
    """
    nx: int
    ny: int
    nz: int
    nu: int
    nv: int
    sod: float
    sdd: float
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    du: float = 2.0
    dv: float = 2.0
    off_u: float = 0.0
    off_v: float = 0.0

    def asdict(self) -> dict:
        return asdict(self)

    def replace(self, **kw) -> "Geom":
        return replace(self, **kw)


def _cube(n: int, nuv: int, nz: int | None = None) -> Geom:
    """Cube-ish workload with d = 7.8125 N and D = 2d, detector pitch 2 and
    unit voxels: unit magnification at the axis and a 3.66 degree half cone
    angle, as in the 64^3 case with d = 500, D = 1000."""
    d = 7.8125 * n
    return Geom(nx=n, ny=n, nz=n if nz is None else nz, nu=nuv, nv=nuv, sod=d, sdd=2.0 * d)


# The five workloads. `np` views over a full circle; `B` views per batch.
CONFIGS = {
    # 64^3, 64 views, 64^2 detector: the small full-FDK case.
    "fdk64": dict(geom=_cube(64, 64), np=64, n_ell=8, seed=101, filter="ramlak",
                  dtype="f32", B=96),
    # 512^3, 512 views, 512^2 detector, Shepp-Logan filtered.
    "bp512": dict(geom=_cube(512, 512), np=512, n_ell=32, seed=102, filter="shepp-logan",
                  dtype="f32", B=96),
    # 2048^3 (32 GiB FP32 volume), 2048 views of 2048^2, launches of up to 96 views.
    "bp2048": dict(geom=_cube(2048, 2048), np=2048, n_ell=32, seed=103, filter="shepp-logan",
                   dtype="f32", B=96),
    # One GPU's slab of the 4096^3 problem: 4096 x 4096 x 256, the outermost
    # mirror pair of 128-slice slabs, 4096 views of 4096^2 in FP16, 16-view chunks.
    "slab4096": dict(geom=_cube(4096, 4096), np=4096, n_ell=64, seed=104, filter="shepp-logan",
                     dtype="f16", B=16, slab=dict(kind="mirror_pair", z0=0, nz_local=256),
                     noise=0.01, noise_seed=204),
    # Differentiable: batch of 4 volumes of 256^3, 360 views of 384^2; the
    # whole volume lies inside the field of view (192 px >= 181 half-diagonal).
    "diff256": dict(geom=Geom(nx=256, ny=256, nz=256, nu=384, nv=384, sod=2000.0, sdd=4000.0),
                    np=360, batch=4, seed=105, dtype="f32", B=96),
}


def config(name: str) -> dict:
    c = dict(CONFIGS[name])
    c["name"] = name
    return c


def angles(n_views: int, start: float = 0.0, arc: float = 2.0 * math.pi) -> np.ndarray:
    """beta_s = start + s * arc / n_views (theta = 2 pi / Np, Table 1)."""
    return start + np.arange(n_views, dtype=np.float64) * (arc / n_views)


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoids(seed: int, n: int, geom: Geom) -> np.ndarray:
    """n random ellipsoids as records of 16 doubles:
    centre (3), semi-axes (3), rotation (3x3 row-major, columns = axes), density.

    Centres U[-0.25, 0.25] and semi-axes U[0.05, 0.25] of the volume's extent
    per axis; orientation a uniformly random unit quaternion; density
    U[0.1, 1]. Densities of overlapping ellipsoids add."""
    rng = np.random.default_rng(seed)
    ext = np.array([geom.nx * geom.dx, geom.ny * geom.dy, geom.nz * geom.dz])
    out = np.zeros((n, 16))
    for m in range(n):
        out[m, 0:3] = rng.uniform(-0.25, 0.25, 3) * ext
        out[m, 3:6] = rng.uniform(0.05, 0.25, 3) * ext
        out[m, 6:15] = _quat_to_rot(rng.normal(size=4)).reshape(-1)
        out[m, 15] = rng.uniform(0.1, 1.0)
    return out


def ball(radius: float, density: float, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """One sphere as a (1, 16) ellipsoid record."""
    e = np.zeros((1, 16))
    e[0, 0:3] = centre
    e[0, 3:6] = radius
    e[0, 6:15] = np.eye(3).reshape(-1)
    e[0, 15] = density
    return e


def sample_voxels(seed: int, geom: Geom, n_random: int, slices=(), columns: int = 0,
                  z_range=None) -> np.ndarray:
    """Voxel sample (i, j, k) as an (n, 3) int64 array: whole slices `slices`,
    `columns` full z-columns at random (i, j), and `n_random` random voxels.
    `z_range` = (k0, k1) restricts the random part and the columns to
    k0 <= k < k1 (a list of such pairs is also accepted)."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in slices:
        jj, ii = np.meshgrid(np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
        parts.append(np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, k)], 1))
    ranges = [(0, geom.nz)] if z_range is None else (
        [tuple(z_range)] if np.isscalar(z_range[0]) else [tuple(r) for r in z_range])
    ks_all = np.concatenate([np.arange(a, b) for a, b in ranges])
    for _ in range(columns):
        i, j = rng.integers(0, geom.nx), rng.integers(0, geom.ny)
        parts.append(np.stack([np.full(ks_all.size, i), np.full(ks_all.size, j), ks_all], 1))
    if n_random:
        parts.append(np.stack([rng.integers(0, geom.nx, n_random),
                               rng.integers(0, geom.ny, n_random),
                               ks_all[rng.integers(0, ks_all.size, n_random)]], 1))
    if not parts:
        return np.zeros((0, 3), np.int64)
    return np.ascontiguousarray(np.concatenate(parts).astype(np.int64))


def random_projections(seed: int, n_views: int, geom: Geom, smooth: bool = False) -> np.ndarray:
    """(n_views, nv, nu) float32 projections with seeded content.
    smooth=False: i.i.d. N(0, 1) (the harshest case for coordinate errors).
    smooth=True: a few random ellipse-like blobs per view plus N(0, 0.01)."""
    rng = np.random.default_rng(seed)
    if not smooth:
        return rng.standard_normal((n_views, geom.nv, geom.nu), dtype=np.float32)
    vv, uu = np.meshgrid(np.arange(geom.nv), np.arange(geom.nu), indexing="ij")
    out = np.empty((n_views, geom.nv, geom.nu), np.float32)
    for s in range(n_views):
        img = 0.01 * rng.standard_normal((geom.nv, geom.nu))
        for _ in range(4):
            cu, cv = rng.uniform(0, geom.nu), rng.uniform(0, geom.nv)
            ru, rv = rng.uniform(0.1, 0.4) * geom.nu, rng.uniform(0.1, 0.4) * geom.nv
            r2 = ((uu - cu) / ru) ** 2 + ((vv - cv) / rv) ** 2
            img += rng.uniform(0.1, 1.0) * np.sqrt(np.clip(1.0 - r2, 0.0, None))
        out[s] = img
    return out


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def _splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) output number c + 1
    of the stream started at `seed`, for each counter c (uint64 arrays)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counters + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def normal_draws(seed: int, geom: Geom, views, rows, cols) -> np.ndarray:
    """Standard normal draws keyed (seed, view, row, column), the noise of
    the noisy-phantom workload: pixel counter m = (view Nv + row) Nu + col,
    Box-Muller (Box and Muller, 1958) on SplitMix64 draws 2m and 2m + 1 with
    u1 = (top 53 bits + 1) 2^-53 in (0, 1] and u2 = (top 53 bits) 2^-53.
    Arguments broadcast against each other."""
    v, r, c = np.broadcast_arrays(np.asarray(views, np.uint64), np.asarray(rows, np.uint64),
                                  np.asarray(cols, np.uint64))
    with np.errstate(over="ignore"):
        m = (v * np.uint64(geom.nv) + r) * np.uint64(geom.nu) + c
        x1 = _splitmix64(seed, np.uint64(2) * m)
        x2 = _splitmix64(seed, np.uint64(2) * m + np.uint64(1))
    u1 = ((x1 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (x2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
