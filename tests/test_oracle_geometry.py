"""Pins for the oracle's geometry (Eq. 2 and Eq. 3, Theorems 1-3) and its
ray model. Each check compares the literal matrix product with something
derived separately: the closed form of z (Eq. 3), hand-derived closed forms
for u and v, the pinhole magnification D/d, and the source/pixel positions
the phantom projector uses."""
import math

import numpy as np
import pytest

import synth

GEOMS = [
    synth.Geom(nx=12, ny=10, nz=8, nu=20, nv=14, sod=60.0, sdd=110.0,
               dx=1.0, dy=1.3, dz=0.8, du=1.7, dv=1.1),
    synth.Geom(nx=9, ny=9, nz=7, nu=16, nv=11, sod=45.0, sdd=80.0,
               dx=0.9, dy=0.9, dz=1.2, du=2.0, dv=2.0, off_u=0.75, off_v=-1.25),
]
BETAS = [0.0, 0.3, 1.1, math.pi / 2, 2.5, math.pi, 4.0, 5.9]


def closed_forms(g, beta, i, j, k):
    """Hand expansion of Eq. (2): z (Eq. 3), u and v."""
    cx, cy, cz = (g.nx - 1) / 2, (g.ny - 1) / 2, (g.nz - 1) / 2
    cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
    X, Y, Z = g.dx * (i - cx), -g.dy * (j - cy), -g.dz * (k - cz)
    z = g.sod + math.sin(beta) * (i - cx) * g.dx - math.cos(beta) * (j - cy) * g.dy
    a = math.cos(beta) * X - math.sin(beta) * Y
    u = g.sdd * a / (g.du * z) + cu
    v = g.sdd * (-Z) / (g.dv * z) + cv
    return u, v, z


def project(P, i, j, k):
    x, y, z = P @ np.array([i, j, k, 1.0])
    return x / z, y / z, z


@pytest.mark.parametrize("g", GEOMS)
def test_z_matches_eq3_and_closed_forms(orc, g):
    rng = np.random.default_rng(0)
    for beta in BETAS:
        P = orc.projection_matrix(g, beta)
        for _ in range(20):
            i, j, k = rng.uniform(-2, g.nx + 1), rng.uniform(-2, g.ny + 1), rng.uniform(-2, g.nz + 1)
            u, v, z = project(P, i, j, k)
            uc, vc, zc = closed_forms(g, beta, i, j, k)
            assert z == pytest.approx(zc, rel=1e-13, abs=1e-11)
            assert u == pytest.approx(uc, rel=1e-12, abs=1e-10)
            assert v == pytest.approx(vc, rel=1e-12, abs=1e-10)


@pytest.mark.parametrize("g", GEOMS)
def test_theorems_2_and_3_u_z_constant_on_column(orc, g):
    for beta in BETAS:
        P = orc.projection_matrix(g, beta)
        assert P[0, 2] == 0.0 and P[2, 2] == 0.0
        for i, j in [(0, 0), (3, 7), (g.nx - 1, g.ny - 1)]:
            us, zs = zip(*[(project(P, i, j, k)[0], project(P, i, j, k)[2]) for k in range(g.nz)])
            assert np.ptp(us) < 1e-11 and np.ptp(zs) < 1e-11


@pytest.mark.parametrize("g", GEOMS)
def test_theorem_1_mirror(orc, g):
    cv2 = (g.nv - 1) + 2 * g.off_v
    for beta in BETAS:
        P = orc.projection_matrix(g, beta)
        for i, j in [(0, 0), (4, 2), (g.nx - 1, 5)]:
            for k in range(g.nz):
                ua, va, _ = project(P, i, j, k)
                ub, vb, _ = project(P, i, j, g.nz - 1 - k)
                assert ua == pytest.approx(ub, abs=1e-11)
                assert va + vb == pytest.approx(cv2, abs=1e-11)


@pytest.mark.parametrize("g", GEOMS)
def test_isocentre_maps_to_principal_point(orc, g):
    for beta in BETAS:
        P = orc.projection_matrix(g, beta)
        u, v, z = project(P, (g.nx - 1) / 2, (g.ny - 1) / 2, (g.nz - 1) / 2)
        assert u == pytest.approx((g.nu - 1) / 2 + g.off_u, abs=1e-12)
        assert v == pytest.approx((g.nv - 1) / 2 + g.off_v, abs=1e-12)
        assert z == pytest.approx(g.sod, rel=1e-14)


def test_magnification_is_D_over_d(orc):
    """A step of one voxel along x at the axis plane (beta = 0) moves u by
    Dx * D / (d * Du) pixels: the pinhole magnification of the scan."""
    g = GEOMS[0]
    P = orc.projection_matrix(g, 0.0)
    c = ((g.nx - 1) / 2, (g.ny - 1) / 2, (g.nz - 1) / 2)
    u0 = project(P, *c)[0]
    u1 = project(P, c[0] + 1, c[1], c[2])[0]
    assert u1 - u0 == pytest.approx(g.dx * g.sdd / (g.sod * g.du), rel=1e-12)
    # k upwards in index is downwards in world Z (M0 negates k), v grows with k.
    v1 = project(P, c[0], c[1], c[2] + 1)[1]
    assert v1 - project(P, *c)[1] == pytest.approx(g.dz * g.sdd / (g.sod * g.dv), rel=1e-12)


@pytest.mark.parametrize("g", GEOMS)
def test_rays_of_phantom_projector_agree_with_P(orc, g):
    """Every point on the ray from the source to pixel (u, v) projects to
    (u, v) through P, and the source itself has z = 0."""
    M0 = orc.m0(g)
    M0inv = np.linalg.inv(M0)
    rng = np.random.default_rng(1)
    for beta in BETAS:
        P = orc.projection_matrix(g, beta)
        for _ in range(10):
            u, v = rng.uniform(-1, g.nu), rng.uniform(-1, g.nv)
            src, pix = orc.source_pixel(g, beta, u, v)
            s_idx = M0inv @ np.append(src, 1.0)
            assert (P @ s_idx)[2] == pytest.approx(0.0, abs=1e-9)
            for t in (0.3, 0.5, 0.8, 1.0):
                w = M0inv @ np.append(src + t * (pix - src), 1.0)
                uu, vv, z = project(P, *w[:3])
                assert uu == pytest.approx(u, abs=1e-9)
                assert vv == pytest.approx(v, abs=1e-9)
                assert z == pytest.approx(t * g.sdd, rel=1e-12)


def test_quarter_turn_geometry(orc):
    """beta + pi/2 for voxel (i, j, k) equals beta for voxel (j, N-1-i, k)
    when Nx = Ny and Dx = Dy: rotating the gantry by a quarter turn is
    rotating the object the other way."""
    g = GEOMS[1]
    for beta in BETAS:
        P = orc.projection_matrix(g, beta)
        Pq = orc.projection_matrix(g, beta + math.pi / 2)
        for (i, j, k) in [(0, 0, 0), (2, 5, 3), (8, 1, 6)]:
            a = project(Pq, i, j, k)
            b = project(P, j, g.nx - 1 - i, k)
            assert np.allclose(a, b, atol=1e-10)
