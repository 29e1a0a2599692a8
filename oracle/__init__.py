"""FP64 CPU oracle for FDK cone-beam back-projection (ctypes over oracle.c).

TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct reference the
GPU library is checked against. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product package never does.
It shares no code with the GPU path.

Functions take a geometry object with the attributes of ``synth.Geom`` (any
object with nx, ny, nz, dx, dy, dz, nu, nv, du, dv, off_u, off_v, sod, sdd).
Arrays: volume (Nz, Ny, Nx) x fastest; projections (Np, Nv, Nu) u fastest.

Each wrapped routine names the passage of Chen et al. (SC'19) it follows:
  projection_matrix   Eq. (2): P = (M1 Mrot M0)[0:3]
  backproject         Alg. 2 with Alg. 3 interpolation, FP64
  backproject_alg4    Alg. 4 (Theorems 1-3), written independently of Alg. 2
  forward_project     the exact transpose of backproject
  filter              Alg. 1: cosine weight, then ramp convolution per row
  filter_rows         Alg. 1 on a list of detector rows
  filter_adjoint      the transpose of Alg. 1
  sirt                SIRT (Gilbert 1972) with forward_project / backproject
  mlem                MLEM (Shepp and Vardi 1982) with the same pair
  phantom_project     analytic line integrals of an ellipsoid phantom
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int64)
_UP = C.POINTER(C.c_uint64)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        L.or_set_num_threads.restype = None
        L.or_projection_matrix.argtypes = [_DP, C.c_double, _DP]
        L.or_projection_matrix4.argtypes = [_DP, C.c_double, _DP]
        L.or_m0.argtypes = [_DP, _DP]
        L.or_splitmix64.restype = C.c_uint64
        L.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.or_hash_uniform.restype = C.c_double
        L.or_hash_uniform.argtypes = [C.c_uint64, C.c_uint64]
        L.or_round_f16.restype = C.c_double
        L.or_round_f16.argtypes = [C.c_double]
        L.or_round_bf16.restype = C.c_double
        L.or_round_bf16.argtypes = [C.c_double]
        L.or_backproject.restype = C.c_int
        L.or_backproject.argtypes = [_DP, C.c_int64, _DP, _DP, C.c_uint64, C.c_int,
                                     C.c_double, C.c_int64, _IP, _DP]
        L.or_backproject_alg4.restype = C.c_int
        L.or_backproject_alg4.argtypes = [_DP, C.c_int64, _DP, _DP, C.c_double, _DP]
        L.or_forward_project.restype = C.c_int
        L.or_forward_project.argtypes = [_DP, C.c_int64, _DP, _DP, C.c_double, _DP]
        L.or_source_pixel.argtypes = [_DP, C.c_double, C.c_double, C.c_double, _DP, _DP]
        L.or_ray_integral.restype = C.c_double
        L.or_ray_integral.argtypes = [_DP, _DP, C.c_int64, _DP]
        L.or_phantom_project.argtypes = [_DP, C.c_int64, _DP, C.c_int64, _DP, _DP]
        L.or_phantom_project_pixels.argtypes = [_DP, _DP, C.c_int64, _IP, C.c_int64, _DP, _DP]
        L.or_phantom_density.argtypes = [C.c_int64, _DP, C.c_int64, _DP, _DP]
        L.or_ramp_kernel.restype = C.c_double
        L.or_ramp_kernel.argtypes = [C.c_int, C.c_int64, C.c_double]
        L.or_cos_weight.restype = C.c_double
        L.or_cos_weight.argtypes = [_DP, C.c_double, C.c_double]
        L.or_filter.restype = C.c_int
        L.or_filter.argtypes = [_DP, C.c_int64, C.c_int, _DP, _DP]
        L.or_filter_adjoint.restype = C.c_int
        L.or_filter_adjoint.argtypes = [_DP, C.c_int64, C.c_int, _DP, _DP]
        L.or_filter_rows.restype = C.c_int
        L.or_filter_rows.argtypes = [_DP, C.c_int64, _IP, C.c_int, _DP, _DP]
        L.or_hash_fill.argtypes = [C.c_uint64, C.c_int64, _UP, C.c_int, _DP]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_DP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gvec(geom) -> np.ndarray:
    """Geometry as the oracle's 14-double vector (see oracle.c)."""
    return np.array([geom.nx, geom.ny, geom.nz, geom.dx, geom.dy, geom.dz,
                     geom.nu, geom.nv, geom.du, geom.dv, geom.off_u, geom.off_v,
                     geom.sod, geom.sdd], dtype=np.float64)


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


def num_threads() -> int:
    return lib().or_num_threads()


def m0(geom) -> np.ndarray:
    out = np.zeros(16)
    lib().or_m0(_d(gvec(geom)), _d(out))
    return out.reshape(4, 4)


def projection_matrix(geom, beta: float, full: bool = False) -> np.ndarray:
    """Eq. (2): the 3x4 matrix P (or the 4x4 P-hat with full=True)."""
    g = gvec(geom)
    if full:
        out = np.zeros(16)
        lib().or_projection_matrix4(_d(g), float(beta), _d(out))
        return out.reshape(4, 4)
    out = np.zeros(12)
    lib().or_projection_matrix(_d(g), float(beta), _d(out))
    return out.reshape(3, 4)


ROUND = {None: 0, "none": 0, "f16": 1, "bf16": 2}


def backproject(geom, angles, q=None, *, seed=None, rnd=None, scale=1.0, voxels=None):
    """Alg. 2 in FP64: scale * sum_s W_dis * interp2(Q_s, u, v).

    q       (Np, Nv, Nu) projections, or None with `seed` to regenerate the
            taps from the counter-based generator (rnd: None, 'f16', 'bf16'
            rounds each generated value to that format first).
    voxels  None for the full (Nz, Ny, Nx) volume, else an (n, 3) array of
            global (i, j, k) indices; returns n values."""
    g = gvec(geom)
    ang = _f64(angles)
    np_ = ang.size
    if q is not None:
        q = _f64(q)
        assert q.shape == (np_, geom.nv, geom.nu), q.shape
        qp = _d(q)
    else:
        assert seed is not None
        qp = _DP()
    if voxels is None:
        out = np.zeros((geom.nz, geom.ny, geom.nx))
        n, ip = 0, _IP()
    else:
        vox = np.ascontiguousarray(voxels, dtype=np.int64)
        out = np.zeros(vox.shape[0])
        n, ip = vox.shape[0], vox.ctypes.data_as(_IP)
    rc = lib().or_backproject(_d(g), np_, _d(ang), qp, int(seed or 0), ROUND[rnd],
                              float(scale), n, ip, _d(out))
    if rc:
        raise MemoryError("oracle backproject")
    return out


def backproject_alg4(geom, angles, q, scale=1.0):
    """Alg. 4 (reduced-cost, mirrored) over the full volume, FP64."""
    g = gvec(geom)
    ang = _f64(angles)
    q = _f64(q)
    assert q.shape == (ang.size, geom.nv, geom.nu)
    out = np.zeros((geom.nz, geom.ny, geom.nx))
    lib().or_backproject_alg4(_d(g), ang.size, _d(ang), _d(q), float(scale), _d(out))
    return out


def forward_project(geom, angles, vol, scale=1.0):
    """Exact adjoint of backproject over the full volume, FP64."""
    g = gvec(geom)
    ang = _f64(angles)
    vol = _f64(vol)
    assert vol.shape == (geom.nz, geom.ny, geom.nx)
    out = np.zeros((ang.size, geom.nv, geom.nu))
    if lib().or_forward_project(_d(g), ang.size, _d(ang), _d(vol), float(scale), _d(out)):
        raise MemoryError("oracle forward_project")
    return out


def source_pixel(geom, beta, u, v):
    src, pix = np.zeros(3), np.zeros(3)
    lib().or_source_pixel(_d(gvec(geom)), float(beta), float(u), float(v), _d(src), _d(pix))
    return src, pix


def ray_integral(src, direction, ell) -> float:
    ell = _f64(ell).reshape(-1, 16)
    return lib().or_ray_integral(_d(_f64(src)), _d(_f64(direction)), ell.shape[0], _d(ell))


def phantom_project(geom, angles, ell) -> np.ndarray:
    """Line integrals E (Np, Nv, Nu) through the ellipsoid phantom."""
    ang = _f64(angles)
    ell = _f64(ell).reshape(-1, 16)
    out = np.zeros((ang.size, geom.nv, geom.nu))
    lib().or_phantom_project(_d(gvec(geom)), ang.size, _d(ang), ell.shape[0], _d(ell), _d(out))
    return out


def phantom_project_pixels(geom, angles, svu, ell) -> np.ndarray:
    """Line integrals for an (n, 3) list of (view, row v, column u)."""
    ang = _f64(angles)
    svu = np.ascontiguousarray(svu, dtype=np.int64)
    ell = _f64(ell).reshape(-1, 16)
    out = np.zeros(svu.shape[0])
    lib().or_phantom_project_pixels(_d(gvec(geom)), _d(ang), svu.shape[0],
                                    svu.ctypes.data_as(_IP), ell.shape[0], _d(ell), _d(out))
    return out


def phantom_density(ell, pts) -> np.ndarray:
    ell = _f64(ell).reshape(-1, 16)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    lib().or_phantom_density(ell.shape[0], _d(ell), pts.shape[0], _d(pts), _d(out))
    return out


def voxel_world(geom, ijk) -> np.ndarray:
    """World coordinates of voxel centres: M0 (i, j, k, 1)."""
    M = m0(geom)
    ijk = np.asarray(ijk, dtype=np.float64).reshape(-1, 3)
    h = np.concatenate([ijk, np.ones((ijk.shape[0], 1))], 1)
    return (h @ M.T)[:, :3]


FILTERS = {"ramlak": 0, "ram-lak": 0, "shepp-logan": 1, "shepplogan": 1}


def ramp_kernel(kind, n, tau) -> float:
    return lib().or_ramp_kernel(FILTERS[kind], int(n), float(tau))


def cos_weight(geom, u, v) -> float:
    return lib().or_cos_weight(_d(gvec(geom)), float(u), float(v))


def filter(geom, e, kind="ramlak") -> np.ndarray:
    """Alg. 1: cosine weighting then ramp convolution, FP64, (nviews, Nv, Nu)."""
    e = _f64(e)
    assert e.shape[1:] == (geom.nv, geom.nu)
    out = np.zeros_like(e)
    if lib().or_filter(_d(gvec(geom)), e.shape[0], FILTERS[kind], _d(e), _d(out)):
        raise MemoryError("oracle filter")
    return out


def filter_adjoint(geom, gq, kind="ramlak") -> np.ndarray:
    """Transpose of the filtering stage (Alg. 1), FP64, (nviews, Nv, Nu)."""
    gq = _f64(gq)
    assert gq.shape[1:] == (geom.nv, geom.nu)
    out = np.zeros_like(gq)
    if lib().or_filter_adjoint(_d(gvec(geom)), gq.shape[0], FILTERS[kind], _d(gq), _d(out)):
        raise MemoryError("oracle filter adjoint")
    return out


def filter_rows(geom, e_rows, rows_v, kind="ramlak") -> np.ndarray:
    """Alg. 1 on a list of detector rows: e_rows (n, Nu); row m is detector
    row rows_v[m], whose cosine weights depend on it."""
    e = _f64(e_rows)
    rv = np.ascontiguousarray(rows_v, dtype=np.int64)
    assert e.ndim == 2 and e.shape == (rv.size, geom.nu)
    out = np.zeros_like(e)
    if lib().or_filter_rows(_d(gvec(geom)), rv.size, rv.ctypes.data_as(_IP), FILTERS[kind],
                            _d(e), _d(out)):
        raise MemoryError("oracle filter")
    return out


def fdk_scale(geom, n_views: int) -> float:
    """pi d^2 / Np: the FDK constant (1/2) * (2 pi / Np) * d^2 for a full
    circle, because W_dis = 1/z^2 carries no d^2."""
    return math.pi * geom.sod ** 2 / n_views


def fdk(geom, angles, e, kind="ramlak", voxels=None) -> np.ndarray:
    """Full FDK: filter, then back-project with the FDK constant."""
    q = filter(geom, e, kind)
    return backproject(geom, angles, q, scale=fdk_scale(geom, len(angles)), voxels=voxels)


def splitmix64(seed: int, counter: int) -> int:
    return lib().or_splitmix64(seed, counter)


def hash_values(seed: int, counters, rnd=None) -> np.ndarray:
    c = np.ascontiguousarray(counters, dtype=np.uint64)
    out = np.zeros(c.size)
    lib().or_hash_fill(seed, c.size, c.ctypes.data_as(_UP), ROUND[rnd], _d(out))
    return out


def round_f16(x: float) -> float:
    return lib().or_round_f16(float(x))


def round_bf16(x: float) -> float:
    return lib().or_round_bf16(float(x))


SIRT_FLOOR = 1e-3


def sirt_weights(geom, angles):
    """Inverse row and column sums of the forward projector F (the
    transpose of backproject), each sum raised to at least 1e-3 of the
    largest: R = 1 / max(F 1, .), C = 1 / max(B 1, .)."""
    ang = _f64(angles)
    rs = forward_project(geom, ang, np.ones((geom.nz, geom.ny, geom.nx)))
    cs = backproject(geom, ang, np.ones((ang.size, geom.nv, geom.nu)))
    return 1.0 / np.maximum(rs, SIRT_FLOOR * rs.max()), 1.0 / np.maximum(cs, SIRT_FLOOR * cs.max())


def sirt(geom, angles, p, n_iter, lam=1.0, nonneg=False, x0=None):
    """SIRT: x <- x + lam C B(R (p - F x)), FP64, full volume."""
    R, Cw = sirt_weights(geom, angles)
    x = np.zeros((geom.nz, geom.ny, geom.nx)) if x0 is None else _f64(x0).copy()
    for _ in range(n_iter):
        r = R * (_f64(p) - forward_project(geom, angles, x))
        x = x + lam * Cw * backproject(geom, angles, r)
        if nonneg:
            x = np.maximum(x, 0.0)
    return x


MLEM_FLOOR = 1e-3  # ratio denominators below this fraction of the largest are raised to it


def mlem(geom, angles, p, n_iter, x0=None):
    """MLEM (Shepp and Vardi 1982): x <- x C B(p / F x), FP64, full volume,
    with C the inverse column sums of sirt_weights (1 / B 1, raised like
    there) and each ratio's denominator raised to at least MLEM_FLOOR of the
    largest F x of that iteration (rays that barely touch the support would
    otherwise divide by next to nothing). Starts from x0, default ones."""
    _, Cw = sirt_weights(geom, angles)
    x = np.ones((geom.nz, geom.ny, geom.nx)) if x0 is None else _f64(x0).copy()
    pf = _f64(p)
    for _ in range(n_iter):
        fx = forward_project(geom, angles, x)
        den = np.maximum(fx, MLEM_FLOOR * fx.max())
        ratio = np.divide(pf, den, out=np.zeros_like(pf), where=den > 0)  # 0 where F x is 0
        x = x * Cw * backproject(geom, angles, ratio)
    return x

