"""Precision of the adjoint (the forward projector, the transpose of Alg. 2
computed as Alg. 4 with Alg. 3's bilinear taps) on inputs that stress how it
accumulates. The tiled adjoint sums each brick's splats in LDS as 32-bit
fixed point, with a power-of-two unit of about 2^-31 of the brick's largest
possible splat times the pixels' overlap. Bricks with more than 1 % of
their non-zero voxels below 2^-13 of their largest magnitude (wide-range
bricks) sum in 64-bit fixed point (unit about 2^-63 of the same bound) when
their non-zero magnitudes span at most 2^40, and in FP32 otherwise; bricks
holding a NaN or an infinity sum in FP32. So:

* wide-range volumes (values over eight decades inside every 16^3 brick:
  one large voxel per brick over a unit or a tiny background; log-uniform
  magnitudes with random signs), each part seeded with voxels 1e-13 of its
  largest (beyond 2^40, so all three projections below take the FP32 path).
  Against the FP64 oracle they match in rel-L2; pixel by pixel, the
  superposition of the same projector applied to the large and the small
  parts separately isolates the accumulation (all three projections use
  identical taps and weights): each pixel's discrepancy must stay below
  1e-5 of the pixel's sum of |contributions|. (Compared with the oracle
  pixel by pixel, FP32 coordinates alone move a large voxel's weight on a
  footprint edge by ~1e-6, which across eight decades exceeds 1e-5 of a
  small neighbour; the oracle comparison is therefore the rel-L2 one.)
* the same volumes with seeds 2^-36 of each part's largest: the parts
  (spanning at most 2^40) take the 64-bit path, their sum (spanning more)
  the FP32 one. The 64-bit path's error is half a unit, about 2^-63 K of
  the brick's largest possible splat, per contribution: a pixel reached
  only by tap weights near zero of the smallest voxels can hold less than
  that. So the per-pixel bound gains an absolute floor of 1e-15 of the
  largest pixel (the unit is ~1e-19 of it);
* ordinary volumes take the 32-bit path, whose error is bounded relative
  to the brick's largest splats, not each pixel's own sum: the
  superposition of two disjoint halves holds to 1e-6 of the largest pixel;
  FDK_FIXED_SUMS (every finite brick in 32 bits) holds the same bound on a
  wide-range volume;
* non-finite inputs: a NaN or an infinity reaches exactly the pixels its
  voxel touches, and every other pixel is unaffected;
* magnitudes near the bottom of the FP32 range (the power-of-two unit
  cannot overflow).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

fdk = pytest.importorskip("paper_1909_02724_amd")

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

BASE = synth.Geom(nx=70, ny=45, nz=38, nu=80, nv=56, sod=420.0, sdd=760.0, du=1.5, dv=1.5)
GEOMS = {
    "mirrored": BASE,
    "plain": BASE.replace(nz=37, off_v=0.27),
    "anisotropic": BASE.replace(dx=0.8, dy=1.1, dz=1.3, du=1.2, dv=1.7, nu=96, nv=50),
}


def announce(msg):
    print(msg, flush=True)


def rel_l2(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def fp(x, g, ang, direct=False):
    return fdk.forward_project(torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV), g,
                               ang, scale=0.9, direct=direct).double().cpu().numpy()


def split_volume(kind, g, seed, seed_level=1e-13):
    """(large part, small part) of a wide-range test volume, as float32
    arrays. Each part also carries, at 1 in 32 voxels (disjoint sets for the
    two parts), values seed_level times its largest magnitude, so that every
    brick of both parts and of their sum is wide-range."""
    rng = np.random.default_rng(seed)
    shape = (g.nz, g.ny, g.nx)
    if kind == "loguniform":
        x = (10.0 ** rng.uniform(-4.0, 4.0, shape)) * rng.choice([-1.0, 1.0], shape)
        x = x.astype(np.float32)
        big = np.abs(x) >= 1.0
        large, small = np.where(big, x, 0).astype(np.float32), np.where(big, 0, x).astype(np.float32)
    else:
        background = 1.0 if kind == "spike" else 1e-4
        small = np.full(shape, background, np.float32)
        large = np.zeros(shape, np.float32)
        # One voxel of 1e4 per 16^3 block of the volume (the kernels' bricks
        # are 16 x 16 columns of 16 or 32 slices), at a seeded place inside it.
        for k0 in range(0, g.nz, 16):
            for j0 in range(0, g.ny, 16):
                for i0 in range(0, g.nx, 16):
                    k = min(k0 + rng.integers(16), g.nz - 1)
                    j = min(j0 + rng.integers(16), g.ny - 1)
                    i = min(i0 + rng.integers(16), g.nx - 1)
                    large[k, j, i] = 1e4
                    small[k, j, i] = 0.0
    # Seed voxels on a lattice (1 in 32 for each part, disjoint), so that
    # even the volume's partial edge bricks hold more than 1 % of them.
    kk, jj, ii = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    lattice = (ii + 7 * jj + 13 * kk) % 32
    seeds_l, seeds_s = lattice == 0, lattice == 16
    sign = rng.choice([-1.0, 1.0], shape)
    large = np.where(seeds_l & (large == 0), seed_level * np.abs(large).max() * sign, large)
    small = np.where(seeds_s, seed_level * np.abs(small).max() * sign, small)
    return large.astype(np.float32), small.astype(np.float32)


@pytest.mark.parametrize("path", ["tiled", "direct", "tiled64"])
@pytest.mark.parametrize("kind", ["spike", "tiny_background", "loguniform"])
@pytest.mark.parametrize("name", list(GEOMS))
def test_adjoint_high_dynamic_range(name, kind, path):
    """tiled: seeds 1e-13 of each part's largest, FP32 path; tiled64: seeds
    2^-36 of it, the parts on the 64-bit path; direct: global FP32 atomics."""
    g = GEOMS[name]
    ang = synth.angles(37, start=0.2)
    direct = path == "direct"
    large, small = split_volume(kind, g, seed=31,
                                seed_level=2.0 ** -36 if path == "tiled64" else 1e-13)
    x = large + small
    announce(f"adjoint HDR {name} {kind} {path}")
    f_x = fp(x, g, ang, direct)
    ref = oracle.forward_project(g, ang, x.astype(np.float64), scale=0.9)
    err = rel_l2(f_x, ref)
    f_l, f_s = fp(large, g, ang, direct), fp(small, g, ang, direct)
    f_al, f_as = fp(np.abs(large), g, ang, direct), fp(np.abs(small), g, ang, direct)
    bound = 1e-5 * (f_al + f_as)
    if path == "tiled64":
        bound = bound + 1e-15 * float(np.max(f_al + f_as))
    excess = np.abs(f_x - f_l - f_s) - bound
    worst = float(np.max(np.abs(f_x - f_l - f_s) / np.maximum(f_al + f_as, 1e-300)))
    announce(f"  rel-L2 vs oracle {err:.3e}; superposition: worst |F x - F x_l - F x_s| / "
             f"F|x| = {worst:.3e}, pixels over 1e-5: {int(np.sum(excess > 0))}")
    assert err <= 1e-5
    assert np.all(excess <= 0.0)


@pytest.mark.parametrize("name", list(GEOMS))
def test_adjoint_fixed_point_bound(name):
    """Ordinary volumes (U(0.5, 1.5), no wide-range brick) take the 32-bit
    fixed-point tile: exact integer sums of splats rounded to a unit of
    about 2^-31 of the brick's largest splat times the overlap. Splitting the
    volume into two disjoint random halves changes each brick's scale, so
    the superposition measures the rounding: bounded by 1e-6 of the largest
    pixel, and the rel-L2 against the oracle by 1e-5."""
    g = GEOMS[name]
    ang = synth.angles(37, start=0.2)
    rng = np.random.default_rng(77)
    x = rng.uniform(0.5, 1.5, (g.nz, g.ny, g.nx)).astype(np.float32)
    half = rng.uniform(0.0, 1.0, x.shape) < 0.5
    xa, xb = np.where(half, x, 0).astype(np.float32), np.where(half, 0, x).astype(np.float32)
    f_x, f_a, f_b = fp(x, g, ang), fp(xa, g, ang), fp(xb, g, ang)
    ref = oracle.forward_project(g, ang, x.astype(np.float64), scale=0.9)
    err = rel_l2(f_x, ref)
    sup = float(np.max(np.abs(f_x - f_a - f_b)) / np.max(np.abs(f_x)))
    announce(f"adjoint fixed point {name}: rel-L2 vs oracle {err:.3e}; "
             f"max |F x - F x_a - F x_b| / max F x = {sup:.3e}")
    assert err <= 1e-5
    assert sup <= 1e-6


@pytest.mark.parametrize("name", ["mirrored", "plain"])
def test_adjoint_fixed_sums_flag(name):
    """FDK_FIXED_SUMS: a wide-range volume summed in 32-bit fixed point
    everywhere matches the default (64-bit) projection to 1e-6 of the
    largest pixel and the oracle in rel-L2; an ordinary volume gives the
    default's result (both take the 32-bit path) up to the order of the
    workgroups' FP32 atomics."""
    g = GEOMS[name]
    ang = synth.angles(37, start=0.2)
    large, small = split_volume("loguniform", g, seed=13, seed_level=2.0 ** -36)
    x = large + small
    xt = torch.from_numpy(x).to(DEV)
    fast = fdk.forward_project(xt, g, ang, scale=0.9, fixed_sums=True).double().cpu().numpy()
    dflt = fp(x, g, ang)
    ref = oracle.forward_project(g, ang, x.astype(np.float64), scale=0.9)
    sup = float(np.max(np.abs(fast - dflt)) / np.max(np.abs(dflt)))
    err = rel_l2(fast, ref)
    xo = np.random.default_rng(4).uniform(0.5, 1.5, x.shape).astype(np.float32)
    fo = fdk.forward_project(torch.from_numpy(xo).to(DEV), g, ang, fixed_sums=True).double().cpu().numpy()
    do = fdk.forward_project(torch.from_numpy(xo).to(DEV), g, ang).double().cpu().numpy()
    ordinary = float(np.max(np.abs(fo - do)) / np.max(np.abs(do)))
    announce(f"fixed sums {name}: wide-range vs default {sup:.3e} of max, rel-L2 vs oracle "
             f"{err:.3e}; ordinary vs default {ordinary:.3e}")
    assert sup <= 1e-6
    assert err <= 1e-5
    assert ordinary <= 1e-6


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf], ids=["nan", "inf", "-inf"])
@pytest.mark.parametrize("direct", [False, True], ids=["tiled", "direct"])
@pytest.mark.parametrize("name", ["mirrored", "plain"])
def test_adjoint_nonfinite_voxel_reaches_its_footprint_only(name, direct, bad):
    g = GEOMS[name]
    ang = synth.angles(13, start=0.4)
    x = np.random.default_rng(5).uniform(0.5, 1.5, (g.nz, g.ny, g.nx)).astype(np.float32)
    vox = (g.nz // 3, g.ny // 2 + 3, g.nx // 2 - 5)
    imp = np.zeros((g.nz, g.ny, g.nx))
    imp[vox] = 1.0
    touched = oracle.forward_project(g, ang, imp, scale=1.0) > 0
    clean = fp(x, g, ang, direct)
    xb = x.copy()
    xb[vox] = bad
    got = fp(xb, g, ang, direct)
    xz = x.copy()
    xz[vox] = 0.0
    rest = fp(xz, g, ang, direct)
    announce(f"adjoint {name} {'direct' if direct else 'tiled'} voxel {bad}: "
             f"{int(touched.sum())} touched pixels, {int(np.sum(~np.isfinite(got)))} non-finite")
    assert touched.any()
    assert np.all(~np.isfinite(got[touched]))
    assert np.all(np.isfinite(got[~touched]))
    scale = np.maximum(np.abs(clean[~touched]), 1e-30)
    assert np.max(np.abs(got[~touched] - rest[~touched]) / scale) <= 1e-5


@pytest.mark.parametrize("direct", [False, True], ids=["tiled", "direct"])
def test_adjoint_tiny_magnitudes(direct):
    g = GEOMS["mirrored"]
    ang = synth.angles(21, start=0.3)
    x = (1e-25 * np.random.default_rng(9).standard_normal((g.nz, g.ny, g.nx))).astype(np.float32)
    got = fp(x, g, ang, direct)
    ref = oracle.forward_project(g, ang, x.astype(np.float64), scale=0.9)
    err = rel_l2(got, ref)
    announce(f"adjoint at 1e-25 {'direct' if direct else 'tiled'}: rel-L2 {err:.3e}")
    assert np.all(np.isfinite(got))
    assert err <= 1e-5
