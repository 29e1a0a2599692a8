"""Pins for the oracle's phantom projector, filtering stage (Alg. 1), full
FDK and the input generator. Independent checks: sphere chords, axis
conventions, FFT convolution (numpy), textbook frequency responses of the
Ram-Lak and Shepp-Logan kernels, the cosine weight as the cosine of the ray
angle, a reconstructed uniform ball, numpy/torch rounding and the published
SplitMix64 known answers."""
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def sphere(R, rho, c=(0.0, 0.0, 0.0)):
    return synth.ball(R, rho, c)


def test_sphere_chords(orc):
    e = sphere(3.0, 0.7, (1.0, -2.0, 0.5))
    src = np.array([-20.0, -2.0, 0.5])
    assert orc.ray_integral(src, np.array([1.0, 0, 0]), e) == pytest.approx(2 * 3.0 * 0.7, rel=1e-14)
    for p in (0.0, 1.0, 2.5, 2.99):
        s = np.array([-20.0, -2.0 + p, 0.5])
        # direction length must not matter
        assert orc.ray_integral(s, np.array([7.0, 0, 0]), e) == pytest.approx(
            2 * math.sqrt(9 - p * p) * 0.7, rel=1e-12)
    assert orc.ray_integral(np.array([-20.0, 1.01, 0.5]), np.array([1.0, 0, 0]), e) == 0.0


def test_ellipsoid_axis_convention(orc):
    """Rotation columns are the ellipsoid's axes in world coordinates: a
    quarter turn about Z carries the long semi-axis (5) onto world Y."""
    e = np.zeros((1, 16))
    e[0, 3:6] = (5.0, 2.0, 1.0)
    e[0, 6:15] = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], float).reshape(-1)
    e[0, 15] = 1.0
    assert orc.ray_integral(np.array([-30.0, 0, 0]), np.array([1.0, 0, 0]), e) == pytest.approx(4.0)
    assert orc.ray_integral(np.array([0, -30.0, 0]), np.array([0, 1.0, 0]), e) == pytest.approx(10.0)
    assert orc.ray_integral(np.array([0, 0, -30.0]), np.array([0, 0, 1.0]), e) == pytest.approx(2.0)
    pts = np.array([[0, 4.9, 0], [0, 5.1, 0], [1.9, 0, 0], [2.1, 0, 0]])
    assert list(orc.phantom_density(e, pts)) == [1.0, 0.0, 1.0, 0.0]


def test_overlapping_densities_add(orc):
    e = np.concatenate([sphere(2.0, 0.5), sphere(1.0, 0.25, (0.5, 0, 0))])
    src, d = np.array([-10.0, 0, 0]), np.array([1.0, 0, 0])
    assert orc.ray_integral(src, d, e) == pytest.approx(2 * 2 * 0.5 + 2 * 1 * 0.25, rel=1e-13)
    assert orc.phantom_density(e, np.array([[0.4, 0, 0]]))[0] == pytest.approx(0.75)


def test_small_sphere_projects_where_P_says(orc):
    g = synth.Geom(nx=16, ny=16, nz=16, nu=40, nv=36, sod=60.0, sdd=100.0, du=1.0, dv=1.0)
    for beta, ijk in [(0.4, (3, 12, 5)), (2.2, (10, 2, 13)), (5.0, (8, 8, 1))]:
        c = orc.voxel_world(g, ijk)[0]
        e = orc.phantom_project(g, [beta], sphere(0.35, 1.0, c))[0]
        P = orc.projection_matrix(g, beta)
        x, y, z = P @ np.array([*ijk, 1.0])
        b, a = np.unravel_index(np.argmax(e), e.shape)
        assert abs(a - x / z) <= 0.5 + 1e-9 and abs(b - y / z) <= 0.5 + 1e-9


def test_cos_weight_is_cosine_of_ray_angle(orc):
    g = synth.Geom(nx=8, ny=8, nz=8, nu=30, nv=22, sod=40.0, sdd=70.0, du=1.5, dv=1.2,
                   off_u=1.25, off_v=-0.5)
    beta = 0.9
    cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
    assert orc.cos_weight(g, cu, cv) == pytest.approx(1.0, abs=1e-15)
    src, pc = orc.source_pixel(g, beta, cu, cv)
    c0 = pc - src
    for (u, v) in [(0, 0), (29, 21), (3.5, 17.0), (cu, 0.0)]:
        _, p = orc.source_pixel(g, beta, u, v)
        r = p - src
        cosg = r @ c0 / (np.linalg.norm(r) * np.linalg.norm(c0))
        assert orc.cos_weight(g, u, v) == pytest.approx(cosg, rel=1e-13)


@pytest.mark.parametrize("kind", ["ramlak", "shepp-logan"])
def test_filter_equals_fft_convolution(orc, kind):
    """Direct convolution against numpy's FFT of the zero-padded row (the
    convolution theorem, Sec. 2.2.3), cosine weights from ray geometry."""
    g = synth.Geom(nx=8, ny=8, nz=8, nu=37, nv=6, sod=30.0, sdd=55.0, du=0.8, dv=0.9, off_u=0.3)
    e = np.random.default_rng(3).standard_normal((2, g.nv, g.nu))
    q = orc.filter(g, e, kind)
    tau = g.du * g.sod / g.sdd
    n = g.nu
    L = 128  # >= 2 n - 1
    h = np.zeros(L)
    for m in range(-(n - 1), n):
        h[m % L] = orc.ramp_kernel(kind, m, tau)
    cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
    src, pc = orc.source_pixel(g, 0.0, cu, cv)
    for s in range(2):
        for b in range(g.nv):
            w = np.empty(n)
            for a in range(n):
                r = orc.source_pixel(g, 0.0, a, b)[1] - src
                w[a] = r @ (pc - src) / (np.linalg.norm(r) * np.linalg.norm(pc - src))
            row = np.zeros(L)
            row[:n] = e[s, b] * w
            ref = tau * np.fft.irfft(np.fft.rfft(row) * np.fft.rfft(h), L)[:n]
            assert np.abs(q[s, b] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ramp_kernels_match_textbook_responses(orc):
    """tau * sum_n h(n) cos(2 pi f n tau): |f| for Ram-Lak and
    sin(pi f tau) / (pi tau) for Shepp-Logan, up to the Nyquist frequency;
    the Ram-Lak taps sum to zero (no DC gain)."""
    tau, M = 0.7, 40000
    n = np.arange(-M, M + 1)
    for kind in ("ramlak", "shepp-logan"):
        h = np.array([orc.ramp_kernel(kind, int(m), tau) for m in range(0, M + 1)])
        hh = np.concatenate([h[:0:-1], h])
        for f in np.array([0.02, 0.1, 0.3, 0.45]) / tau:
            H = tau * np.sum(hh * np.cos(2 * math.pi * f * n * tau))
            expect = abs(f) if kind == "ramlak" else math.sin(math.pi * f * tau) / (math.pi * tau)
            assert H == pytest.approx(expect, rel=2e-4, abs=2e-5)
        if kind == "ramlak":
            assert abs(hh.sum()) * tau * tau < 1e-4


@pytest.mark.parametrize("kind", ["ramlak", "shepp-logan"])
def test_fdk_reconstructs_uniform_ball(orc, kind):
    """FDK of an analytic uniform ball (radius 0.3 N) gives its density on
    the central slice: mean over r < 0.6 R within 1 %, background near 0."""
    N, rho = 32, 0.7
    g = synth.Geom(nx=N, ny=N, nz=N, nu=48, nv=48, sod=7.8125 * N, sdd=2 * 7.8125 * N)
    ang = synth.angles(96)
    R = 0.3 * N
    e = orc.phantom_project(g, ang, sphere(R, rho))
    k = N // 2
    vox = synth.sample_voxels(0, g, 0, slices=(k,))
    vals = orc.fdk(g, ang, e, kind, voxels=vox).reshape(N, N)
    pts = orc.voxel_world(g, vox)
    r = np.sqrt((pts[:, 0] ** 2 + pts[:, 1] ** 2 + pts[:, 2] ** 2)).reshape(N, N)
    inner = vals[r < 0.6 * R].mean()
    outer = vals[(r > 1.4 * R) & (r < 1.45 * N / 2)]
    assert inner == pytest.approx(rho, rel=0.01)
    assert abs(outer.mean()) < 0.01 * rho


def test_fdk_ellipsoid_phantom_interior(orc):
    """Several random ellipsoids: FDK matches the phantom density at voxels
    well inside constant regions (loose: cone beam and discretisation)."""
    cfg = synth.config("fdk64")
    g = cfg["geom"]
    g = g.replace(nx=48, ny=48, nz=48, nu=72, nv=72, sod=375.0, sdd=750.0)
    ang = synth.angles(96)
    ell = synth.ellipsoids(cfg["seed"], 4, g)
    e = orc.phantom_project(g, ang, ell)
    vox = synth.sample_voxels(1, g, 0, slices=(18, 22, 26, 30))
    rec = orc.fdk(g, ang, e, "shepp-logan", voxels=vox)
    pts = orc.voxel_world(g, vox)
    dens = orc.phantom_density(ell, pts)
    # voxels whose neighbours two voxels away have the same density
    offs = np.array([[a, b, c] for a in (-2, 0, 2) for b in (-2, 0, 2) for c in (-2, 0, 2)], float)
    same = np.ones(len(pts), bool)
    for o in offs:
        same &= orc.phantom_density(ell, pts + o) == dens
    mask = same & (dens > 0)
    assert mask.sum() > 50
    err = np.abs(rec[mask] - dens[mask])
    print('interior voxels', mask.sum(), 'median err', np.median(err))
    assert np.median(err) < 0.05 * dens[mask].max()


def test_splitmix64_known_answers(orc):
    with open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")) as f:
        ref = [int(x) for x in f.read().split("\n") if x and not x.startswith("#")]
    assert [orc.splitmix64(1234567, c) for c in range(3)] == ref


def test_generated_values_grid_and_range(orc):
    v = orc.hash_values(5, np.arange(200000, dtype=np.uint64))
    assert v.min() >= -1.0 and v.max() < 1.0
    assert np.all(v * 2 ** 23 == np.round(v * 2 ** 23))
    assert abs(v.mean()) < 0.01 and v.std() == pytest.approx(1 / math.sqrt(3), rel=0.01)


def test_rounding_matches_numpy_f16_and_torch_bf16(orc):
    import torch
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-1, 1, 3000),
                        rng.uniform(-1, 1, 1000) * 1e-5,      # binary16 subnormal range
                        rng.standard_normal(1000) * 100.0,
                        (np.arange(-2048, 2048) + 0.5) * 2.0 ** -10])  # exact ties
    f16 = np.array([orc.round_f16(t) for t in x])
    assert np.array_equal(f16, x.astype(np.float16).astype(np.float64))
    xf = x.astype(np.float32)  # torch rounds from float32; these are exact in both
    bf = np.array([orc.round_bf16(float(t)) for t in xf])
    ref = torch.from_numpy(xf).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf, ref)


@pytest.mark.parametrize("kind", ["ramlak", "shepp-logan"])
def test_filter_adjoint_is_transpose(orc, kind):
    """The oracle's adjoint filter is the transpose of its filter: matrix
    columns built by filtering unit images equal the adjoint's rows (brute
    force on a small detector), and the dot-product identity holds on random
    data. A non-square, offset detector keeps the cosine weight asymmetric
    in u and v, so a weight applied on the wrong side fails."""
    g = synth.Geom(nx=8, ny=8, nz=8, nu=9, nv=4, sod=30.0, sdd=55.0, du=3.0, dv=2.5,
                   off_u=0.6, off_v=-0.3)
    n = g.nv * g.nu
    A = np.empty((n, n))
    for m in range(n):
        e = np.zeros((1, g.nv, g.nu))
        e.reshape(-1)[m] = 1.0
        A[:, m] = orc.filter(g, e, kind).reshape(-1)
    At = np.empty((n, n))
    for m in range(n):
        gq = np.zeros((1, g.nv, g.nu))
        gq.reshape(-1)[m] = 1.0
        At[:, m] = orc.filter_adjoint(g, gq, kind).reshape(-1)
    assert np.abs(At - A.T).max() <= 1e-13 * np.abs(A).max()
    # rows never mix: the operator is block diagonal over detector rows
    assert np.all(A.reshape(g.nv, g.nu, g.nv, g.nu)[0, :, 1, :] == 0.0)
    # the weight makes it non-symmetric, so the transpose test has teeth
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()
    rng = np.random.default_rng(9)
    e = rng.standard_normal((3, g.nv, g.nu))
    gq = rng.standard_normal((3, g.nv, g.nu))
    lhs = np.vdot(orc.filter(g, e, kind), gq)
    rhs = np.vdot(e, orc.filter_adjoint(g, gq, kind))
    assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(e) * np.linalg.norm(gq))
