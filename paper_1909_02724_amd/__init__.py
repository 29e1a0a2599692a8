"""MI355X-native FDK cone-beam back-projection (after iFDK, Chen et al., SC'19).

Thin ctypes binding over libfdk.so (C ABI in include/fdk.h). Every step of
the path runs in the library's HIP kernels; PyTorch only provides device
memory and the current stream. There is no CPU fallback: if libfdk.so is
missing, every call raises.

Arrays: volume (Nz_local, Ny, Nx) float32, x fastest; projections
(nviews, Nv, Nu), u fastest, float32 / float16 / bfloat16 storage.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

__all__ = [
    "Geometry", "FDKError", "lib", "backproject", "forward_project", "filter",
    "filter_adjoint", "slab_rows", "fdk_scale", "FDKBackprojection", "fdk_backprojection",
    "FDKReconstruction", "fdk_reconstruction", "sirt_weights", "sirt_iteration",
    "sirt_iteration_noalloc", "sirt",
    "mlem_iteration", "mlem",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdk.so")

FDK_OK, FDK_ERR_INVALID_ARG, FDK_ERR_UNSUPPORTED, FDK_ERR_HIP, FDK_ERR_OOM = range(5)
FDK_ACCUMULATE = 1
FDK_NONNEG = 2
FDK_DIRECT = 4
FDK_FIXED_SUMS = 8
_DTYPES = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}
_FILTERS = {"ramlak": 0, "ram-lak": 0, "shepp-logan": 1, "shepplogan": 1}
_SLABS = {"contiguous": 0, "mirror_pair": 1}


@dataclass(frozen=True)
class Geometry:
    """Circular cone-beam geometry (Table 1 of the paper); one length unit.

    nx, ny, nz: voxels; dx, dy, dz: voxel pitch; nu, nv: detector pixels;
    du, dv: pixel pitch; off_u, off_v: principal-point shift in pixels;
    sod: source to rotation axis (d); sdd: source to detector (D)."""
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
    du: float = 1.0
    dv: float = 1.0
    off_u: float = 0.0
    off_v: float = 0.0


class _CGeometry(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("nu", C.c_int32), ("nv", C.c_int32),
        ("du", C.c_double), ("dv", C.c_double),
        ("off_u", C.c_double), ("off_v", C.c_double),
        ("sod", C.c_double), ("sdd", C.c_double),
        ("np", C.c_int32), ("angles", C.POINTER(C.c_double)),
    ]


class FDKError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fdk status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libfdk.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1909_02724_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(_CGeometry)
        L.fdk_backproject.restype = C.c_int
        L.fdk_backproject.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_int, C.c_void_p,
                                      C.c_int32, C.c_int32, C.c_int, C.c_float, C.c_uint32,
                                      C.c_void_p]
        L.fdk_forward_project.restype = C.c_int
        L.fdk_forward_project.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                          C.c_int32, C.c_int, C.c_void_p, C.c_float, C.c_uint32,
                                          C.c_void_p]
        L.fdk_filter.restype = C.c_int
        L.fdk_filter.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int,
                                 C.c_int, C.c_void_p]
        L.fdk_filter_rows.restype = C.c_int
        L.fdk_filter_rows.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_int,
                                      C.c_void_p]
        L.fdk_filter_adjoint.restype = C.c_int
        L.fdk_filter_adjoint.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int,
                                         C.c_void_p]
        L.fdk_sirt_weights.restype = C.c_int
        L.fdk_sirt_weights.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.fdk_sirt_iteration.restype = C.c_int
        L.fdk_sirt_iteration.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int,
                                         C.c_float, C.c_uint32, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
        L.fdk_sirt_iteration_noalloc.restype = C.c_int
        L.fdk_sirt_iteration_noalloc.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                                 C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                                 C.c_int, C.c_float, C.c_uint32, C.c_void_p]
        L.fdk_mlem_iteration.restype = C.c_int
        L.fdk_mlem_iteration.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_int32, C.c_int32, C.c_int, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
        L.fdk_slab_rows.restype = C.c_int
        L.fdk_slab_rows.argtypes = [P, C.c_int32, C.c_int32, C.c_int, C.POINTER(C.c_int32)]
        L.fdk_fdk_scale.restype = C.c_double
        L.fdk_fdk_scale.argtypes = [P]
        L.fdk_projection_matrix.restype = C.c_int
        L.fdk_projection_matrix.argtypes = [P, C.c_int32, C.POINTER(C.c_double)]
        L.fdk_last_error.restype = C.c_char_p
        L.fdk_last_error.argtypes = []
        _lib = L
    return _lib


def _cgeom(geom, angles):
    ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
    cg = _CGeometry(int(geom.nx), int(geom.ny), int(geom.nz),
                    float(geom.dx), float(geom.dy), float(geom.dz),
                    int(geom.nu), int(geom.nv), float(geom.du), float(geom.dv),
                    float(geom.off_u), float(geom.off_v), float(geom.sod), float(geom.sdd),
                    int(ang.size), ang.ctypes.data_as(C.POINTER(C.c_double)))
    return cg, ang  # keep `ang` alive for the duration of the call


def _check(status: int):
    if status != FDK_OK:
        raise FDKError(status, lib().fdk_last_error().decode())


def _stream(t: torch.Tensor):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (no CPU fallback)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _slab(geom, z0, nz_local, slab):
    nz_local = geom.nz - z0 if nz_local is None else nz_local
    return int(z0), int(nz_local), _SLABS[slab]


def _flags(accumulate: bool, direct: bool) -> int:
    return (FDK_ACCUMULATE if accumulate else 0) | (FDK_DIRECT if direct else 0)


def backproject(q: torch.Tensor, geom, angles, *, view0: int = 0, out: torch.Tensor | None = None,
                z0: int = 0, nz_local: int | None = None, slab: str = "contiguous",
                scale: float = 1.0, accumulate: bool = False,
                direct: bool = False) -> torch.Tensor:
    """Back-project views [view0, view0 + q.shape[0]) of `q` (nviews, Nv, Nu)
    into a (nz_local, Ny, Nx) float32 slab: Alg. 2 computed as Alg. 4.
    direct=True runs the direct variant (taps from global memory) instead of
    the LDS-tiled one."""
    _dev(q, "q")
    if q.dtype not in _DTYPES:
        raise ValueError(f"unsupported projection dtype {q.dtype}")
    if q.dim() != 3 or q.shape[1:] != (geom.nv, geom.nu):
        raise ValueError(f"q must be (nviews, {geom.nv}, {geom.nu}), got {tuple(q.shape)}")
    z0, nzl, sk = _slab(geom, z0, nz_local, slab)
    if out is None:
        out = torch.empty((nzl, geom.ny, geom.nx), dtype=torch.float32, device=q.device)
        accumulate = False
    _dev(out, "out")
    if out.dtype != torch.float32 or tuple(out.shape) != (nzl, geom.ny, geom.nx):
        raise ValueError(f"out must be float32 ({nzl}, {geom.ny}, {geom.nx})")
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_backproject(C.byref(cg), view0, q.shape[0], C.c_void_p(q.data_ptr()),
                                 _DTYPES[q.dtype], C.c_void_p(out.data_ptr()), z0, nzl, sk,
                                 float(scale), _flags(accumulate, direct), _stream(q)))
    return out


def forward_project(vol: torch.Tensor, geom, angles, *, view0: int = 0,
                    nviews: int | None = None, out: torch.Tensor | None = None, z0: int = 0,
                    slab: str = "contiguous", scale: float = 1.0,
                    accumulate: bool = False, direct: bool = False,
                    fixed_sums: bool = False) -> torch.Tensor:
    """Matched forward projection (exact adjoint of backproject) of a
    float32 slab into (nviews, Nv, Nu) float32 projections. direct=True runs
    the direct variant instead of the LDS-tiled one; fixed_sums=True sums
    wide-range bricks in 32-bit fixed point too (FDK_FIXED_SUMS)."""
    _dev(vol, "vol")
    if vol.dtype != torch.float32 or vol.dim() != 3 or vol.shape[1:] != (geom.ny, geom.nx):
        raise ValueError(f"vol must be float32 (nz_local, {geom.ny}, {geom.nx})")
    nviews = len(angles) - view0 if nviews is None else nviews
    z0, nzl, sk = _slab(geom, z0, vol.shape[0], slab)
    if out is None:
        out = torch.empty((nviews, geom.nv, geom.nu), dtype=torch.float32, device=vol.device)
        accumulate = False
    _dev(out, "out")
    if out.dtype != torch.float32 or tuple(out.shape) != (nviews, geom.nv, geom.nu):
        raise ValueError(f"out must be float32 ({nviews}, {geom.nv}, {geom.nu})")
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_forward_project(C.byref(cg), view0, nviews, C.c_void_p(vol.data_ptr()), z0,
                                     nzl, sk, C.c_void_p(out.data_ptr()), float(scale),
                                     _flags(accumulate, direct) | (FDK_FIXED_SUMS if fixed_sums else 0),
                                     _stream(vol)))
    return out


def filter(e: torch.Tensor, geom, angles, *, view0: int = 0, kind: str = "ramlak",
           dtype: torch.dtype = torch.float32, out: torch.Tensor | None = None,
           rows: tuple[int, int] | None = None) -> torch.Tensor:
    """Filtering stage (Alg. 1): cosine weight and ramp convolution of
    float32 line integrals (nviews, Nv, Nu); output in `dtype` storage.

    rows=(v0, nrows) filters only detector rows [v0, v0 + nrows): `e` and
    `out` are then (nviews, nrows, Nu) and may be views into larger arrays
    (row-contiguous, any view stride)."""
    if not e.is_cuda:
        raise ValueError("e must be a GPU tensor (no CPU fallback)")
    v0, nrows = (0, geom.nv) if rows is None else (int(rows[0]), int(rows[1]))
    if e.dtype != torch.float32 or e.dim() != 3 or tuple(e.shape[1:]) != (nrows, geom.nu):
        raise ValueError(f"e must be float32 (nviews, {nrows}, {geom.nu})")
    if out is None:
        out = torch.empty(e.shape, dtype=dtype, device=e.device)
    if not out.is_cuda or out.dtype not in _DTYPES or out.shape != e.shape:
        raise ValueError("out must match e's shape with a float32/float16/bfloat16 dtype")
    for t, name in ((e, "e"), (out, "out")):
        if t.stride(2) != 1 or (nrows > 1 and t.stride(1) != geom.nu):
            raise ValueError(f"{name} rows must be contiguous")
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_filter_rows(C.byref(cg), view0, e.shape[0], v0, nrows,
                                 C.c_void_p(e.data_ptr()), e.stride(0) if e.shape[0] > 1 else nrows * geom.nu,
                                 C.c_void_p(out.data_ptr()),
                                 out.stride(0) if out.shape[0] > 1 else nrows * geom.nu,
                                 _DTYPES[out.dtype], _FILTERS[kind], _stream(e)))
    return out


def slab_rows(geom, angles, *, z0: int = 0, nz_local: int | None = None,
              slab: str = "contiguous") -> list[tuple[int, int]]:
    """Detector row bands [(v0, nrows), ...] (at most two, ascending) that
    the back-projection of this slab reads over all views of the scan."""
    z0, nzl, sk = _slab(geom, z0, nz_local, slab)
    cg, _keep = _cgeom(geom, angles)
    band = (C.c_int32 * 4)()
    _check(lib().fdk_slab_rows(C.byref(cg), z0, nzl, sk, band))
    return [(band[2 * n], band[2 * n + 1]) for n in range(2) if band[2 * n + 1] > 0]


def filter_adjoint(gq: torch.Tensor, geom, angles, *, view0: int = 0, kind: str = "ramlak",
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """Transpose of the filtering stage for float32 (nviews, Nv, Nu)
    gradients: the row convolution, then the cosine weight."""
    _dev(gq, "gq")
    if gq.dtype != torch.float32 or gq.dim() != 3 or tuple(gq.shape[1:]) != (geom.nv, geom.nu):
        raise ValueError(f"gq must be float32 (nviews, {geom.nv}, {geom.nu})")
    if out is None:
        out = torch.empty_like(gq)
    _dev(out, "out")
    if out.dtype != torch.float32 or out.shape != gq.shape:
        raise ValueError("out must be float32 with gq's shape")
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_filter_adjoint(C.byref(cg), view0, gq.shape[0], C.c_void_p(gq.data_ptr()),
                                    C.c_void_p(out.data_ptr()), _FILTERS[kind], _stream(gq)))
    return out


def projection_matrix(geom, angles, view: int) -> np.ndarray:
    """The (3, 4) matrix P of Eq. 2 the kernels use for view `view`:
    [x, y, z] = P [i, j, k, 1], (u, v) = (x / z, y / z) in pixels."""
    cg, _keep = _cgeom(geom, angles)
    out = (C.c_double * 12)()
    _check(lib().fdk_projection_matrix(C.byref(cg), int(view), out))
    return np.array(out[:], dtype=np.float64).reshape(3, 4)


def fdk_scale(geom, angles) -> float:
    """pi d^2 / Np, the FDK constant for a full circular scan."""
    cg, _keep = _cgeom(geom, angles)
    return lib().fdk_fdk_scale(C.byref(cg))


def _same_views(t: torch.Tensor, angles: np.ndarray):
    # The backward pass projects onto every angle, so the forward pass must
    # use every angle too: one view of the input per angle.
    if t.dim() < 3 or t.shape[-3] != angles.size:
        raise ValueError(f"input has {t.shape[-3] if t.dim() >= 3 else '?'} views for "
                         f"{angles.size} angles; the differentiable operators need one per angle")


class FDKBackprojection(torch.autograd.Function):
    """Differentiable back-projection. forward: q (B, nviews, Nv, Nu) or
    (nviews, Nv, Nu) -> volume (B, Nz, Ny, Nx) / (Nz, Ny, Nx). backward: the
    matched forward projector applied to the incoming volume gradient, which
    recomputes every coordinate rather than storing them."""

    @staticmethod
    def forward(ctx, q, geom, angles, scale=1.0):
        ctx.geom, ctx.angles, ctx.scale = geom, np.asarray(angles, np.float64), float(scale)
        _same_views(q, ctx.angles)
        ctx.qshape, ctx.qdtype = q.shape, q.dtype
        batched = q.dim() == 4
        qs = q if batched else q.unsqueeze(0)
        vols = [backproject(qs[b].contiguous(), geom, ctx.angles, scale=ctx.scale)
                for b in range(qs.shape[0])]
        out = torch.stack(vols)
        return out if batched else out[0]

    @staticmethod
    def backward(ctx, gvol):
        batched = gvol.dim() == 4
        gv = gvol if batched else gvol.unsqueeze(0)
        gq = torch.stack([forward_project(gv[b].to(torch.float32).contiguous(), ctx.geom,
                                          ctx.angles, scale=ctx.scale)
                          for b in range(gv.shape[0])])
        gq = gq if batched else gq[0]
        return gq.to(ctx.qdtype), None, None, None


def fdk_backprojection(q, geom, angles, scale=1.0):
    return FDKBackprojection.apply(q, geom, angles, scale)


class FDKReconstruction(torch.autograd.Function):
    """Differentiable FDK from line integrals: forward filters E (cosine
    weight and ramp, Alg. 1, FP32) and back-projects; backward applies the
    matched forward projector and then the filter's transpose, so gradients
    reach the raw line integrals. e: (B, nviews, Nv, Nu) or (nviews, Nv, Nu)
    float32."""

    @staticmethod
    def forward(ctx, e, geom, angles, kind="ramlak", scale=1.0):
        ctx.geom, ctx.angles = geom, np.asarray(angles, np.float64)
        _same_views(e, ctx.angles)
        ctx.kind, ctx.scale = kind, float(scale)
        batched = e.dim() == 4
        es = e if batched else e.unsqueeze(0)
        vols = [backproject(filter(es[b].contiguous(), geom, ctx.angles, kind=kind), geom,
                            ctx.angles, scale=ctx.scale) for b in range(es.shape[0])]
        out = torch.stack(vols)
        return out if batched else out[0]

    @staticmethod
    def backward(ctx, gvol):
        batched = gvol.dim() == 4
        gv = gvol if batched else gvol.unsqueeze(0)
        ge = torch.stack([
            filter_adjoint(forward_project(gv[b].to(torch.float32).contiguous(), ctx.geom,
                                           ctx.angles, scale=ctx.scale),
                           ctx.geom, ctx.angles, kind=ctx.kind)
            for b in range(gv.shape[0])])
        return (ge if batched else ge[0]), None, None, None, None


def fdk_reconstruction(e, geom, angles, kind="ramlak", scale=None):
    """FDK of line integrals e, differentiable with respect to e. scale
    defaults to the FDK constant pi d^2 / Np."""
    if scale is None:
        scale = fdk_scale(geom, angles)
    return FDKReconstruction.apply(e, geom, angles, kind, scale)


def _f32_dev(t, shape, name):
    _dev(t, name)
    if t.dtype != torch.float32 or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be float32 {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def sirt_weights(geom, angles, *, view0: int = 0, nviews: int | None = None, z0: int = 0,
                 nz_local: int | None = None, slab: str = "contiguous", device="cuda"):
    """Inverse row sums R (nviews, Nv, Nu) and column sums C (slab) of the
    forward projector, for SIRT."""
    nviews = len(angles) - view0 if nviews is None else int(nviews)
    z0, nzl, sk = _slab(geom, z0, nz_local, slab)
    row_inv = torch.empty((nviews, geom.nv, geom.nu), dtype=torch.float32, device=device)
    col_inv = torch.empty((nzl, geom.ny, geom.nx), dtype=torch.float32, device=device)
    tmp = torch.empty_like(col_inv)
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_sirt_weights(C.byref(cg), view0, nviews, z0, nzl, sk,
                                  C.c_void_p(row_inv.data_ptr()), C.c_void_p(col_inv.data_ptr()),
                                  C.c_void_p(tmp.data_ptr()), _stream(tmp)))
    return row_inv, col_inv


def sirt_iteration(x, p, row_inv, col_inv, geom, angles, *, view0: int = 0, z0: int = 0,
                   slab: str = "contiguous", lam: float = 1.0, nonneg: bool = False,
                   proj_tmp=None, vol_tmp=None):
    """One SIRT update of x (slab, in place) towards projections p."""
    z0, nzl, sk = _slab(geom, z0, x.shape[0], slab)
    _f32_dev(x, (nzl, geom.ny, geom.nx), "x")
    _f32_dev(p, (p.shape[0], geom.nv, geom.nu), "p")
    _f32_dev(row_inv, p.shape, "row_inv")
    _f32_dev(col_inv, x.shape, "col_inv")
    proj_tmp = torch.empty_like(p) if proj_tmp is None else proj_tmp
    vol_tmp = torch.empty_like(x) if vol_tmp is None else vol_tmp
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_sirt_iteration(C.byref(cg), view0, p.shape[0], C.c_void_p(p.data_ptr()),
                                    C.c_void_p(row_inv.data_ptr()), C.c_void_p(col_inv.data_ptr()),
                                    C.c_void_p(x.data_ptr()), z0, nzl, sk, float(lam),
                                    FDK_NONNEG if nonneg else 0, C.c_void_p(proj_tmp.data_ptr()),
                                    C.c_void_p(vol_tmp.data_ptr()), _stream(x)))
    return x


def sirt_iteration_noalloc(x, p, row_inv, col_inv, geom, angles, *, view0: int = 0, z0: int = 0,
                           slab: str = "contiguous", lam: float = 1.0, nonneg: bool = False):
    """sirt_iteration with the library's static per-GPU workspace (64 MiB):
    allocates nothing, for callers that cannot; calls that overlap on one
    GPU race."""
    z0, nzl, sk = _slab(geom, z0, x.shape[0], slab)
    _f32_dev(x, (nzl, geom.ny, geom.nx), "x")
    _f32_dev(p, (p.shape[0], geom.nv, geom.nu), "p")
    _f32_dev(row_inv, p.shape, "row_inv")
    _f32_dev(col_inv, x.shape, "col_inv")
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_sirt_iteration_noalloc(
        C.byref(cg), view0, p.shape[0], C.c_void_p(p.data_ptr()), C.c_void_p(row_inv.data_ptr()),
        C.c_void_p(col_inv.data_ptr()), C.c_void_p(x.data_ptr()), z0, nzl, sk, float(lam),
        FDK_NONNEG if nonneg else 0, _stream(x)))
    return x


def sirt(p, geom, angles, n_iter: int, *, lam: float = 1.0, nonneg: bool = False, x0=None,
         z0: int = 0, nz_local: int | None = None, slab: str = "contiguous"):
    """n_iter SIRT iterations from x0 (default zero) for projections p
    (nviews, Nv, Nu) float32 of views [0, nviews)."""
    row_inv, col_inv = sirt_weights(geom, angles, nviews=p.shape[0], z0=z0, nz_local=nz_local,
                                    slab=slab, device=p.device)
    x = torch.zeros_like(col_inv) if x0 is None else x0.clone()
    proj_tmp, vol_tmp = torch.empty_like(p), torch.empty_like(x)
    for _ in range(n_iter):
        sirt_iteration(x, p, row_inv, col_inv, geom, angles, z0=z0, slab=slab, lam=lam,
                       nonneg=nonneg, proj_tmp=proj_tmp, vol_tmp=vol_tmp)
    return x


def mlem_iteration(x, p, col_inv, geom, angles, *, view0: int = 0, z0: int = 0,
                   slab: str = "contiguous", proj_tmp=None, vol_tmp=None):
    """One MLEM update of x (non-negative slab, in place) towards
    non-negative projections p; col_inv from sirt_weights."""
    z0, nzl, sk = _slab(geom, z0, x.shape[0], slab)
    _f32_dev(x, (nzl, geom.ny, geom.nx), "x")
    _f32_dev(p, (p.shape[0], geom.nv, geom.nu), "p")
    _f32_dev(col_inv, x.shape, "col_inv")
    proj_tmp = torch.empty_like(p) if proj_tmp is None else proj_tmp
    vol_tmp = torch.empty_like(x) if vol_tmp is None else vol_tmp
    cg, _keep = _cgeom(geom, angles)
    _check(lib().fdk_mlem_iteration(C.byref(cg), view0, p.shape[0], C.c_void_p(p.data_ptr()),
                                    C.c_void_p(col_inv.data_ptr()), C.c_void_p(x.data_ptr()), z0,
                                    nzl, sk, C.c_void_p(proj_tmp.data_ptr()),
                                    C.c_void_p(vol_tmp.data_ptr()), _stream(x)))
    return x


def mlem(p, geom, angles, n_iter: int, *, x0=None, z0: int = 0, nz_local: int | None = None,
         slab: str = "contiguous"):
    """n_iter MLEM iterations from x0 (default all ones) for non-negative
    projections p (nviews, Nv, Nu) float32 of views [0, nviews)."""
    _, col_inv = sirt_weights(geom, angles, nviews=p.shape[0], z0=z0, nz_local=nz_local,
                              slab=slab, device=p.device)
    x = torch.ones_like(col_inv) if x0 is None else x0.clone()
    proj_tmp, vol_tmp = torch.empty_like(p), torch.empty_like(x)
    for _ in range(n_iter):
        mlem_iteration(x, p, col_inv, geom, angles, z0=z0, slab=slab, proj_tmp=proj_tmp,
                       vol_tmp=vol_tmp)
    return x
