"""CPU checks of the C ABI: the library loads, exports every function its
header declares, lays out fdk_geometry as C does, and rejects invalid
arguments on the host with the documented status and a message, before
any HIP call (so these run without a GPU)."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1909_02724_amd as fdk
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdk_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    L = fdk.lib()
    names = declared_functions()
    assert {"fdk_filter", "fdk_filter_rows", "fdk_filter_adjoint", "fdk_backproject",
            "fdk_forward_project", "fdk_slab_rows", "fdk_fdk_scale",
            "fdk_last_error"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", fdk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (fdk_\w+)", out))
    assert set(names) <= exported


def test_geometry_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "fdk.h"\n'
        "int main(void){printf(\"%zu\", sizeof(fdk_geometry));\n"
        + "".join(f'printf(" %zu", offsetof(fdk_geometry, {f}));\n'
                  for f, _ in fdk._CGeometry._fields_)
        + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == C.sizeof(fdk._CGeometry)
    assert vals[1:] == [getattr(fdk._CGeometry, f).offset for f, _ in fdk._CGeometry._fields_]


GOOD = fdk.Geometry(nx=16, ny=16, nz=8, nu=24, nv=20, sod=100.0, sdd=200.0, du=2.0, dv=2.0)
ANG = np.linspace(0, 2 * math.pi, 12, endpoint=False)
FAKE = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def call_bp(g=GOOD, ang=ANG, view0=0, nviews=4, q=FAKE, dtype=0, vol=FAKE, z0=0, nzl=8,
            slab=0, scale=1.0, flags=0):
    cg, keep = fdk._cgeom(g, ang)
    st = fdk.lib().fdk_backproject(C.byref(cg), view0, nviews, q, dtype, vol, z0, nzl, slab,
                                   scale, flags, None)
    return st, fdk.lib().fdk_last_error().decode()


@pytest.mark.parametrize("kw, status, msg", [
    (dict(g=GOOD.__class__(**{**GOOD.__dict__, "nx": 0})), 1, "volume size"),
    (dict(g=GOOD.__class__(**{**GOOD.__dict__, "dv": -1.0})), 1, "pixel pitch"),
    (dict(g=GOOD.__class__(**{**GOOD.__dict__, "sod": 10.0})), 1, "half-diagonal"),
    (dict(g=GOOD.__class__(**{**GOOD.__dict__, "sdd": float("nan")})), 1, "sod and sdd"),
    (dict(g=GOOD.__class__(**{**GOOD.__dict__, "sdd": GOOD.sod})), 1, "must exceed sod"),
    (dict(g=GOOD.__class__(**{**GOOD.__dict__, "sdd": 0.5 * GOOD.sod})), 1, "must exceed sod"),
    (dict(ang=np.array([0.0, float("inf"), 1.0, 2.0])), 1, "not finite"),
    (dict(view0=10, nviews=4), 1, "view range"),
    (dict(view0=-1), 1, "view range"),
    (dict(q=None), 1, "projection pointer"),
    (dict(vol=None), 1, "volume pointer"),
    (dict(dtype=7), 2, "dtype"),
    (dict(z0=4, nzl=8), 1, "exceeds"),
    (dict(nzl=0), 1, "nz_local"),
    (dict(slab=1, nzl=5), 1, "even"),
    (dict(slab=1, z0=2, nzl=8), 1, "overlap"),
    (dict(slab=3), 2, "slab kind"),
    (dict(scale=float("nan")), 1, "scale"),
    (dict(flags=8), 1, "flags"),
])
def test_backproject_validation(kw, status, msg):
    st, err = call_bp(**kw)
    assert st == status and msg in err, (st, err)


def test_forward_and_filter_validation():
    L = fdk.lib()
    cg, keep = fdk._cgeom(GOOD, ANG)
    assert L.fdk_forward_project(C.byref(cg), 0, 4, None, 0, 8, 0, FAKE, 1.0, 0, None) == 1
    assert "volume pointer" in L.fdk_last_error().decode()
    assert L.fdk_forward_project(C.byref(cg), 11, 4, FAKE, 0, 8, 0, FAKE, 1.0, 0, None) == 1
    assert L.fdk_forward_project(C.byref(cg), 0, 4, FAKE, 0, 8, 0, FAKE, 1.0, 16, None) == 1
    assert "flags" in L.fdk_last_error().decode()
    assert L.fdk_filter(C.byref(cg), 0, 4, FAKE, FAKE, 0, 9, None) == 2
    assert "filter kind" in L.fdk_last_error().decode()
    assert L.fdk_filter(C.byref(cg), 0, 4, FAKE, FAKE, 5, 0, None) == 2
    assert L.fdk_filter(C.byref(cg), 0, 4, C.c_void_p(0x1000), C.c_void_p(0x1004), 0, 0, None) == 1
    assert "overlap" in L.fdk_last_error().decode()
    wide = GOOD.__class__(**{**GOOD.__dict__, "nu": 9000})
    cw, keep2 = fdk._cgeom(wide, ANG)
    assert L.fdk_filter(C.byref(cw), 0, 4, FAKE, C.c_void_p(0x10000000), 0, 0, None) == 2
    assert L.fdk_backproject(None, 0, 1, FAKE, 0, FAKE, 0, 8, 0, 1.0, 0, None) == 1
    assert "NULL" in L.fdk_last_error().decode()


def test_filter_rows_validation():
    L = fdk.lib()
    cg, keep = fdk._cgeom(GOOD, ANG)
    band = 5 * GOOD.nu
    assert L.fdk_filter_rows(C.byref(cg), 0, 2, 18, 5, FAKE, band, C.c_void_p(0x100000), band,
                             0, 0, None) == 1
    assert "row band" in L.fdk_last_error().decode()
    assert L.fdk_filter_rows(C.byref(cg), 0, 2, 0, 5, FAKE, band - 1, C.c_void_p(0x100000), band,
                             0, 0, None) == 1
    assert "view stride" in L.fdk_last_error().decode()
    assert L.fdk_filter_rows(C.byref(cg), 0, 2, 0, 5, C.c_void_p(0x1000), band,
                             C.c_void_p(0x1000 + 8), band, 0, 0, None) == 1
    assert "overlap" in L.fdk_last_error().decode()
    # an empty band is a successful no-op (nothing enqueued)
    assert L.fdk_filter_rows(C.byref(cg), 0, 2, 3, 0, FAKE, band, FAKE, band, 0, 0, None) == 0


def test_fdk_scale():
    cg, keep = fdk._cgeom(GOOD, ANG)
    assert fdk.lib().fdk_fdk_scale(C.byref(cg)) == pytest.approx(math.pi * 100.0 ** 2 / 12)
    assert math.isnan(fdk.lib().fdk_fdk_scale(None))


def test_python_layer_refuses_cpu_tensors():
    import torch
    with pytest.raises(ValueError, match="GPU tensor"):
        fdk.backproject(torch.zeros(4, 20, 24), GOOD, ANG)


def _tap_rows(g, ang, ks):
    """Rows of every bilinear tap of every voxel with global slice in ks, by
    the oracle's projection matrices (Eq. 2, Alg. 3)."""
    import oracle
    ii, jj, kk = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.asarray(ks), indexing="ij")
    h = np.stack([ii.ravel(), jj.ravel(), kk.ravel(), np.ones(ii.size)], 0).astype(np.float64)
    rows = set()
    for beta in ang:
        x, y, z = oracle.projection_matrix(g, beta) @ h
        nv = np.floor(y / z).astype(np.int64)
        rows.update(np.unique(nv).tolist())
        rows.update(np.unique(nv + 1).tolist())
    return {r for r in rows if 0 <= r < g.nv}


@pytest.mark.parametrize("slab, z0, nzl", [("contiguous", 0, 20), ("contiguous", 11, 6),
                                           ("contiguous", 0, 40), ("mirror_pair", 0, 8),
                                           ("mirror_pair", 9, 20), ("mirror_pair", 3, 2)])
def test_slab_rows_cover_every_tap(slab, z0, nzl):
    """The bands hold every row any voxel of the slab taps, in every view,
    and little else (one spare row a side plus the spread over views)."""
    import synth
    g = synth.Geom(nx=24, ny=20, nz=40, nu=48, nv=60, sod=90.0, sdd=200.0, du=1.5, dv=1.5)
    ang = synth.angles(24, start=0.05)
    if slab == "contiguous":
        ks = np.arange(z0, z0 + nzl)
    else:
        h = nzl // 2
        ks = np.concatenate([np.arange(z0, z0 + h), np.arange(g.nz - z0 - h, g.nz - z0)])
    bands = fdk.slab_rows(g, ang, z0=z0, nz_local=nzl, slab=slab)
    held = set()
    for v0, n in bands:
        assert 0 <= v0 and v0 + n <= g.nv and n > 0
        held.update(range(v0, v0 + n))
    need = _tap_rows(g, ang, ks)
    assert need <= held, sorted(need - held)
    # no more than two spare rows per band edge beyond the taps' extent
    assert len(held) <= len(need) + 4 * len(bands)
    if len(bands) == 2:
        assert bands[0][0] + bands[0][1] < bands[1][0]


def test_slab_rows_validation():
    cg, keep = fdk._cgeom(GOOD, ANG)
    L = fdk.lib()
    band = (C.c_int32 * 4)()
    assert L.fdk_slab_rows(C.byref(cg), 0, 8, 0, None) == 1
    assert "band" in L.fdk_last_error().decode()
    assert L.fdk_slab_rows(C.byref(cg), 4, 8, 0, band) == 1
    assert L.fdk_slab_rows(C.byref(cg), 0, 5, 1, band) == 1
    assert L.fdk_slab_rows(C.byref(cg), 0, 8, 0, band) == 0
    assert band[1] > 0


def test_filter_adjoint_validation():
    L = fdk.lib()
    cg, keep = fdk._cgeom(GOOD, ANG)
    assert L.fdk_filter_adjoint(C.byref(cg), 0, 4, FAKE, FAKE, 9, None) == 2
    assert "filter kind" in L.fdk_last_error().decode()
    assert L.fdk_filter_adjoint(C.byref(cg), 10, 4, FAKE, C.c_void_p(0x10000000), 0, None) == 1
    assert "view range" in L.fdk_last_error().decode()
    assert L.fdk_filter_adjoint(C.byref(cg), 0, 4, C.c_void_p(0x1000), C.c_void_p(0x1004), 0,
                                None) == 1
    assert "overlap" in L.fdk_last_error().decode()
    assert L.fdk_filter_adjoint(None, 0, 4, FAKE, FAKE, 0, None) == 1


def test_sirt_validation():
    L = fdk.lib()
    cg, keep = fdk._cgeom(GOOD, ANG)
    A, B_, C_, D_ = (C.c_void_p(0x1000 * k) for k in (1, 2, 3, 4))
    assert L.fdk_sirt_weights(C.byref(cg), 0, 4, 0, 8, 0, None, B_, C_, None) == 1
    assert "NULL" in L.fdk_last_error().decode()
    assert L.fdk_sirt_weights(C.byref(cg), 0, 4, 0, 8, 0, A, B_, B_, None) == 1
    assert L.fdk_sirt_weights(C.byref(cg), 0, 0, 0, 8, 0, A, B_, C_, None) == 1
    assert L.fdk_sirt_weights(C.byref(cg), 0, 4, 4, 8, 0, A, B_, C_, None) == 1  # slab past Nz
    E_, F_ = C.c_void_p(0x5000), C.c_void_p(0x6000)
    it = L.fdk_sirt_iteration
    assert it(C.byref(cg), 0, 4, A, B_, C_, D_, 0, 8, 0, 1.0, 0, A, F_, None) == 1
    assert "alias" in L.fdk_last_error().decode()
    assert it(C.byref(cg), 0, 4, A, B_, C_, D_, 0, 8, 0, float("nan"), 0, E_, F_, None) == 1
    assert it(C.byref(cg), 0, 4, A, B_, C_, D_, 0, 8, 0, 1.0, 8, E_, F_, None) == 1
    assert "flags" in L.fdk_last_error().decode()


def test_sirt_noalloc_validation():
    """The static-workspace SIRT iteration refuses, on the host, inputs whose
    workspace (projections rounded up to 64 floats, plus the slab) exceeds
    its 2^24 floats, and otherwise validates like fdk_sirt_iteration."""
    L = fdk.lib()
    it = L.fdk_sirt_iteration_noalloc
    A, B_, C_, D_ = (C.c_void_p(0x1000 * k) for k in (1, 2, 3, 4))
    cg, keep = fdk._cgeom(GOOD, ANG)
    assert it(C.byref(cg), 0, 0, A, B_, C_, D_, 0, 8, 0, 1.0, 0, None) == 1      # no views
    assert it(C.byref(cg), 0, 4, A, B_, C_, D_, 0, 0, 0, 1.0, 0, None) == 1      # empty slab
    big = synth.Geom(nx=256, ny=256, nz=256, nu=256, nv=256, sod=2000.0, sdd=4000.0)
    ang = synth.angles(4)
    cgb, keepb = fdk._cgeom(big, ang)
    # 4 x 256^2 projection values + 256^3 voxels = 2^24 + 2^18 > 2^24
    assert it(C.byref(cgb), 0, 4, A, B_, C_, D_, 0, 256, 0, 1.0, 0, None) == 1
    assert "static" in L.fdk_last_error().decode()
    # a slab of 255 slices fits exactly: (2^18 + 255 * 2^16) <= 2^24, so the
    # size check passes and the next check (the NaN lambda) fails instead
    assert it(C.byref(cgb), 0, 4, A, B_, C_, D_, 0, 252, 0, float("nan"), 0, None) == 1
    assert "lambda" in L.fdk_last_error().decode()


def test_mlem_validation():
    L = fdk.lib()
    cg, keep = fdk._cgeom(GOOD, ANG)
    A, B_, X, E_, F_ = (C.c_void_p(0x1000 * k) for k in (1, 2, 3, 5, 6))
    it = L.fdk_mlem_iteration
    assert it(C.byref(cg), 0, 4, None, B_, X, 0, 8, 0, E_, F_, None) == 1
    assert "NULL" in L.fdk_last_error().decode()
    assert it(C.byref(cg), 0, 4, A, B_, X, 0, 8, 0, A, F_, None) == 1      # proj_tmp is p
    assert "alias" in L.fdk_last_error().decode()
    assert it(C.byref(cg), 0, 4, A, B_, X, 0, 8, 0, E_, X, None) == 1      # vol_tmp is x
    assert it(C.byref(cg), 0, 4, A, B_, X, 0, 8, 0, E_, B_, None) == 1     # vol_tmp is col_inv
    assert it(C.byref(cg), 0, 0, A, B_, X, 0, 8, 0, E_, F_, None) == 1     # no views
    assert it(C.byref(cg), 0, 4, A, B_, X, 4, 8, 0, E_, F_, None) == 1     # slab past Nz
    assert it(C.byref(cg), 0, 4, A, B_, X, 0, 8, 5, E_, F_, None) == 2     # unknown slab kind


@pytest.mark.parametrize("gi", [0, 1, 2])
def test_projection_matrix_matches_oracle(orc, gi):
    """The host geometry the kernels are built from (fdk_projection_matrix,
    no HIP call) equals the oracle's literal product M1 Mrot(b) M0 (Eq. 2)
    for offset principal points, anisotropic pitches and any angle."""
    geoms = [
        synth.Geom(nx=12, ny=10, nz=8, nu=20, nv=14, sod=60.0, sdd=110.0,
                   dx=1.0, dy=1.3, dz=0.8, du=1.7, dv=1.1),
        synth.Geom(nx=9, ny=9, nz=7, nu=16, nv=11, sod=45.0, sdd=80.0,
                   dx=0.9, dy=0.9, dz=1.2, du=2.0, dv=2.0, off_u=0.75, off_v=-1.25),
        synth.config("bp2048")["geom"],
    ]
    g = geoms[gi]
    ang = np.array([0.0, 0.3, 1.1, np.pi / 2, 2.5, np.pi, 4.0, 5.9, -7.3])
    for s, beta in enumerate(ang):
        got = fdk.projection_matrix(g, ang, s)
        ref = orc.projection_matrix(g, beta)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_projection_matrix_validation():
    g = synth.Geom(nx=8, ny=8, nz=8, nu=12, nv=12, sod=40.0, sdd=80.0)
    ang = np.array([0.0, 1.0])
    with pytest.raises(fdk.FDKError):
        fdk.projection_matrix(g, ang, 2)
    with pytest.raises(fdk.FDKError):
        fdk.projection_matrix(g, ang, -1)
    with pytest.raises(fdk.FDKError):
        fdk.projection_matrix(g, np.array([0.0, np.nan]), 1)
    L = fdk.lib()
    cg, _keep = fdk._cgeom(g, ang)
    assert L.fdk_projection_matrix(C.byref(cg), 0, None) == fdk.FDK_ERR_INVALID_ARG


def test_autograd_functions_need_one_view_per_angle():
    """The differentiable operators' backward passes project onto every
    angle, so a forward pass over fewer views than angles is rejected before
    any device work (here with a host tensor, which never reaches the GPU)."""
    import torch
    g = fdk.Geometry(nx=8, ny=8, nz=8, nu=12, nv=10, sod=40.0, sdd=80.0)
    ang = np.linspace(0, 2 * math.pi, 6, endpoint=False)
    with pytest.raises(ValueError, match="one per angle"):
        fdk.fdk_backprojection(torch.zeros(4, g.nv, g.nu), g, ang)
    with pytest.raises(ValueError, match="one per angle"):
        fdk.fdk_reconstruction(torch.zeros(2, 5, g.nv, g.nu), g, ang, scale=1.0)
