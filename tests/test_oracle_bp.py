"""Pins for the oracle's back-projection (Alg. 2 with Alg. 3) and its
adjoint. Independent checks: the separately written Alg. 4, the closed
form of a constant projection (Eq. 3), hand-computable impulse responses,
invariants (linearity, view order, quarter-turn, mirror, view chunks), a
brute-force transpose and the dot-product identity."""
import math

import numpy as np
import pytest

import synth

G = synth.Geom(nx=11, ny=9, nz=8, nu=19, nv=13, sod=40.0, sdd=75.0,
               dx=1.0, dy=1.0, dz=1.0, du=1.6, dv=1.4)
G_ODD = G.replace(nz=7)
G_OFF = G.replace(off_u=0.6, off_v=-0.35)


def rnd_q(g, n_views, seed=0):
    return np.random.default_rng(seed).standard_normal((n_views, g.nv, g.nu))


@pytest.mark.parametrize("g", [G, G_ODD, G_OFF])
def test_alg2_equals_alg4(orc, g):
    ang = synth.angles(7, start=0.2)
    q = rnd_q(g, 7)
    a2 = orc.backproject(g, ang, q, scale=1.7)
    a4 = orc.backproject_alg4(g, ang, q, scale=1.7)
    assert np.abs(a2 - a4).max() <= 1e-12 * np.abs(a2).max()


def test_constant_projection_closed_form(orc):
    """Q = c everywhere: where all four taps lie inside the detector,
    V = scale * c * sum_s 1/z_s^2 with z from Eq. (3)."""
    g = G.replace(nu=64, nv=64)  # wide detector: every tap inside
    ang = synth.angles(5, start=0.4)
    c, scale = 0.75, 2.5
    q = np.full((5, g.nv, g.nu), c)
    V = orc.backproject(g, ang, q, scale=scale)
    cx, cy = (g.nx - 1) / 2, (g.ny - 1) / 2
    for (i, j, k) in [(0, 0, 0), (5, 4, 3), (10, 8, 7), (3, 6, 1)]:
        ref = sum(1.0 / (g.sod + math.sin(b) * (i - cx) * g.dx - math.cos(b) * (j - cy) * g.dy) ** 2
                  for b in ang)
        assert V[k, j, i] == pytest.approx(scale * c * ref, rel=1e-13)


def test_impulse_response_is_bilinear_hat(orc):
    """A single unit pixel Q[s0][b0][a0] = 1 gives each voxel
    scale * W * hat(u - a0) * hat(v - b0), hat(t) = max(0, 1 - |t|).
    The detector is not square, so swapped u/v axes fail."""
    g = G
    ang = synth.angles(3, start=0.1)
    for (s0, b0, a0) in [(0, 6, 9), (2, 2, 4), (1, 10, 14), (1, 3, 11)]:
        q = np.zeros((3, g.nv, g.nu))
        q[s0, b0, a0] = 1.0
        V = orc.backproject(g, ang, q, scale=3.0)
        P = orc.projection_matrix(g, ang[s0])
        expect = np.zeros_like(V)
        for k in range(g.nz):
            for j in range(g.ny):
                for i in range(g.nx):
                    x, y, z = P @ np.array([i, j, k, 1.0])
                    u, v = x / z, y / z
                    expect[k, j, i] = 3.0 / z ** 2 * max(0, 1 - abs(u - a0)) * max(0, 1 - abs(v - b0))
        assert np.abs(V - expect).max() <= 1e-14 * max(1.0, np.abs(expect).max())
        assert np.abs(expect).max() > 0


def test_outside_detector_reads_zero(orc):
    """A voxel projecting between -1 and 0 in u takes only the in-detector
    tap (weight du), the reading of zero extension with floor."""
    g = G.replace(nu=13, nv=9)
    ang = np.array([0.0])
    P = orc.projection_matrix(g, 0.0)
    q = np.ones((1, g.nv, g.nu))
    V = orc.backproject(g, ang, q)
    hit = 0
    for k in range(g.nz):
        for j in range(g.ny):
            for i in range(g.nx):
                x, y, z = P @ np.array([i, j, k, 1.0])
                u, v = x / z, y / z
                wu = np.interp(u, [-1, 0, g.nu - 1, g.nu], [0, 1, 1, 0])
                wv = np.interp(v, [-1, 0, g.nv - 1, g.nv], [0, 1, 1, 0])
                assert V[k, j, i] == pytest.approx(wu * wv / z ** 2, rel=1e-13, abs=1e-18)
                hit += (wu < 1) or (wv < 1)
    assert hit > 0  # the geometry does put some voxels over the border


def test_linearity_and_view_order_and_chunks(orc):
    g = G_OFF
    ang = synth.angles(6, start=0.3)
    q1, q2 = rnd_q(g, 6, 1), rnd_q(g, 6, 2)
    b1, b2 = orc.backproject(g, ang, q1), orc.backproject(g, ang, q2)
    b12 = orc.backproject(g, ang, 2.5 * q1 - q2)
    assert np.allclose(b12, 2.5 * b1 - b2, rtol=0, atol=1e-12 * np.abs(b12).max())
    perm = np.array([3, 0, 5, 1, 4, 2])
    bp = orc.backproject(g, ang[perm], q1[perm])
    assert np.allclose(bp, b1, rtol=0, atol=1e-12 * np.abs(b1).max())
    ba = orc.backproject(g, ang[:2], q1[:2])
    bb = orc.backproject(g, ang[2:], q1[2:])
    assert np.allclose(ba + bb, b1, rtol=0, atol=1e-12 * np.abs(b1).max())


def test_quarter_turn_rotates_volume(orc):
    """Angles + pi/2 with the same projections give V'(i, j, k) = V(j, N-1-i, k)."""
    g = G.replace(nx=9, ny=9)
    ang = synth.angles(5, start=0.25)
    q = rnd_q(g, 5, 3)
    V = orc.backproject(g, ang, q)
    Vq = orc.backproject(g, ang + math.pi / 2, q)
    N = g.nx
    for k in range(g.nz):
        for j in range(g.ny):
            for i in range(g.nx):
                assert Vq[k, j, i] == pytest.approx(V[k, N - 1 - i, j], rel=1e-9, abs=1e-12)


def test_mirror_flip_in_v_flips_volume_in_k(orc):
    """Theorem 1: flipping every projection in v flips the volume in k."""
    g = G
    ang = synth.angles(4, start=0.7)
    q = rnd_q(g, 4, 4)
    V = orc.backproject(g, ang, q)
    Vf = orc.backproject(g, ang, q[:, ::-1, :])
    assert np.allclose(Vf, V[::-1], rtol=0, atol=1e-12 * np.abs(V).max())


def test_sampled_voxels_match_full_volume(orc):
    g = G_OFF
    ang = synth.angles(4)
    q = rnd_q(g, 4, 5)
    V = orc.backproject(g, ang, q, scale=0.5)
    vox = synth.sample_voxels(7, g, 50, slices=(2,), columns=2)
    vals = orc.backproject(g, ang, q, scale=0.5, voxels=vox)
    assert np.array_equal(vals, V[vox[:, 2], vox[:, 1], vox[:, 0]])


@pytest.mark.parametrize("rnd", [None, "f16", "bf16"])
def test_generated_taps_equal_explicit_array(orc, rnd):
    g = G
    ang = synth.angles(3)
    n = 3 * g.nv * g.nu
    q = orc.hash_values(99, np.arange(n, dtype=np.uint64), rnd=rnd).reshape(3, g.nv, g.nu)
    a = orc.backproject(g, ang, q)
    b = orc.backproject(g, ang, seed=99, rnd=rnd)
    assert np.array_equal(a, b)


def test_adjoint_dot_product(orc):
    g = G_OFF
    ang = synth.angles(5, start=0.1)
    rng = np.random.default_rng(8)
    q = rng.standard_normal((5, g.nv, g.nu))
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    lhs = np.vdot(orc.backproject(g, ang, q, scale=1.3), x)
    rhs = np.vdot(q, orc.forward_project(g, ang, x, scale=1.3))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_adjoint_is_brute_force_transpose(orc):
    """Build the back-projection matrix column by column from unit
    projections and the forward-projection matrix from unit volumes:
    one is the transpose of the other."""
    g = synth.Geom(nx=4, ny=3, nz=5, nu=6, nv=5, sod=12.0, sdd=20.0, du=1.3, dv=1.1)
    ang = synth.angles(3, start=0.5)
    nq, nvx = 3 * g.nv * g.nu, g.nz * g.ny * g.nx
    A = np.zeros((nvx, nq))
    for c in range(nq):
        e = np.zeros(nq)
        e[c] = 1.0
        A[:, c] = orc.backproject(g, ang, e.reshape(3, g.nv, g.nu)).ravel()
    B = np.zeros((nq, nvx))
    for c in range(nvx):
        e = np.zeros(nvx)
        e[c] = 1.0
        B[:, c] = orc.forward_project(g, ang, e.reshape(g.nz, g.ny, g.nx)).ravel()
    assert np.abs(A).max() > 0
    assert np.abs(A.T - B).max() <= 1e-15
