"""GPU-side synthetic inputs (benchmark and test infrastructure).

ctypes over synth/libsynth_gpu.so (built from synth/gpu.hip): SplitMix64
counter-based values written straight into device memory, an analytic
ellipsoid-phantom projector (whole views or a band of rows) and counter-keyed
Gaussian noise. None of it holds any reconstruction arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "gpu.hip")
LIB = os.path.join(_HERE, "libsynth_gpu.so")
_lib = None
_DT = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}


def build() -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.run([hipcc, "-std=c++17", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-x", "hip", SRC, "-o", tmp], check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing; run synth.gpu.build()")
        L = C.CDLL(LIB)
        L.synth_hash_fill.restype = C.c_int
        L.synth_hash_fill.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_void_p, C.c_int,
                                      C.c_void_p]
        L.synth_phantom_project.restype = C.c_int
        L.synth_phantom_project.argtypes = [C.c_int32, C.c_int32] + [C.c_double] * 6 + [
            C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.synth_phantom_rows.restype = C.c_int
        L.synth_phantom_rows.argtypes = [C.c_int32, C.c_int32] + [C.c_double] * 6 + [
            C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_uint64,
            C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.synth_view_sigma.restype = C.c_int
        L.synth_view_sigma.argtypes = [C.c_int32, C.c_int32] + [C.c_double] * 6 + [
            C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _stream(t):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def hash_fill(out: torch.Tensor, seed: int, counter0: int = 0) -> torch.Tensor:
    """out.view(-1)[m] = SplitMix64 uniform(seed, counter0 + m), in out's dtype."""
    assert out.is_cuda and out.is_contiguous() and out.dtype in _DT
    rc = lib().synth_hash_fill(seed, counter0, out.numel(), C.c_void_p(out.data_ptr()),
                               _DT[out.dtype], _stream(out))
    if rc:
        raise RuntimeError(f"synth_hash_fill: HIP error {rc}")
    return out


def phantom_project(geom, angles, ell, out: torch.Tensor | None = None,
                    device="cuda") -> torch.Tensor:
    """Line integrals (nviews, Nv, Nu) float32 of an ellipsoid phantom."""
    ang = torch.as_tensor(np.asarray(angles, np.float64), device=device)
    e = torch.as_tensor(np.ascontiguousarray(ell, np.float64).reshape(-1), device=device)
    n = ang.numel()
    if out is None:
        out = torch.empty((n, geom.nv, geom.nu), dtype=torch.float32, device=device)
    rc = lib().synth_phantom_project(geom.nu, geom.nv, geom.du, geom.dv, geom.off_u, geom.off_v,
                                     geom.sod, geom.sdd, C.c_void_p(ang.data_ptr()), n,
                                     C.c_void_p(e.data_ptr()), e.numel() // 16,
                                     C.c_void_p(out.data_ptr()), _stream(out))
    if rc:
        raise RuntimeError(f"synth_phantom_project: HIP error {rc}")
    return out


def _geo_args(geom):
    return (geom.nu, geom.nv, geom.du, geom.dv, geom.off_u, geom.off_v, geom.sod, geom.sdd)


def view_sigma(geom, angles, ell, rel: float, device="cuda") -> torch.Tensor:
    """Noise level per view (float64, device): rel times the largest clean
    line integral on the detector row floor(cv) through the principal point."""
    ang = torch.as_tensor(np.asarray(angles, np.float64), device=device)
    e = torch.as_tensor(np.ascontiguousarray(ell, np.float64).reshape(-1), device=device)
    out = torch.empty(ang.numel(), dtype=torch.float64, device=device)
    rc = lib().synth_view_sigma(*_geo_args(geom), C.c_void_p(ang.data_ptr()), ang.numel(),
                                C.c_void_p(e.data_ptr()), e.numel() // 16, float(rel),
                                C.c_void_p(out.data_ptr()), _stream(out))
    if rc:
        raise RuntimeError(f"synth_view_sigma: HIP error {rc}")
    return out


def phantom_rows(geom, angles: torch.Tensor, ell: torch.Tensor, v0: int, out: torch.Tensor,
                 view_index0: int = 0, seed: int = 0,
                 sigma: torch.Tensor | None = None) -> torch.Tensor:
    """Rows [v0, v0 + out.shape[1]) of the views whose angles are `angles`
    (device float64; global view numbers view_index0 + s) into `out`
    (float32 (nviews, nrows, Nu), rows contiguous, any view stride): line
    integrals plus sigma[s] * standard normal keyed (seed, view, row, column)."""
    n, nrows = out.shape[0], out.shape[1]
    assert out.is_cuda and out.dtype == torch.float32 and out.shape[2] == geom.nu
    assert out.stride(2) == 1 and (nrows <= 1 or out.stride(1) == geom.nu)
    assert angles.is_cuda and angles.dtype == torch.float64 and angles.numel() == n
    assert ell.is_cuda and ell.dtype == torch.float64
    if sigma is not None:
        assert sigma.is_cuda and sigma.dtype == torch.float64 and sigma.numel() == n
    vstride = out.stride(0) if n > 1 else nrows * geom.nu
    rc = lib().synth_phantom_rows(*_geo_args(geom), C.c_void_p(angles.data_ptr()), n, int(v0),
                                  nrows, C.c_void_p(ell.data_ptr()), ell.numel() // 16,
                                  int(seed), int(view_index0),
                                  None if sigma is None else C.c_void_p(sigma.data_ptr()),
                                  C.c_void_p(out.data_ptr()), vstride, _stream(out))
    if rc:
        raise RuntimeError(f"synth_phantom_rows: HIP error {rc}")
    return out
