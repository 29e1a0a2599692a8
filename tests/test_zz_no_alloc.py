"""The SIRT iteration that allocates nothing (fdk_sirt_iteration_noalloc,
workspace in the library's static per-GPU array) against the one that takes
its workspaces as arguments (fdk_sirt_iteration), through the C ABI: two
calls in a row on the same GPU, the second on a smaller input (the array
keeps the first call's contents), each with a mirrored and a plain slab.
The two share their kernels; the forward projection adds through FP32
atomics in no fixed order, so they agree to FP32 rounding, not bitwise."""
import numpy as np
import pytest
import torch

import synth

fdk = pytest.importorskip("paper_1909_02724_amd")

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

CASES = [
    # (geometry, views): the larger first, then a smaller one reusing the array
    (synth.Geom(nx=48, ny=44, nz=40, nu=64, nv=52, sod=300.0, sdd=600.0), 30),
    (synth.Geom(nx=20, ny=18, nz=14, nu=30, nv=22, sod=150.0, sdd=330.0, off_v=0.27), 11),
]


def rel_l2(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_sirt_iteration_matches_workspace_entry_point():
    for n, (g, nviews) in enumerate(CASES):
        ang = synth.angles(nviews, start=0.3 + n)
        p = torch.from_numpy(synth.random_projections(40 + n, nviews, g, smooth=True)).to(DEV)
        p.clamp_(min=0.0)
        row_inv, col_inv = fdk.sirt_weights(g, ang, device=DEV)
        x0 = torch.from_numpy(np.random.default_rng(50 + n).uniform(
            0.0, 1.0, (g.nz, g.ny, g.nx)).astype(np.float32)).to(DEV)
        x_ws, x_na = x0.clone(), x0.clone()
        for it in range(2):
            fdk.sirt_iteration(x_ws, p, row_inv, col_inv, g, ang, lam=0.9)
            fdk.sirt_iteration_noalloc(x_na, p, row_inv, col_inv, g, ang, lam=0.9)
            torch.cuda.synchronize()
            err = rel_l2(x_na, x_ws)
            step = rel_l2(x_ws, x0)
            print(f"noalloc case {n} iteration {it}: rel-L2 vs workspace entry point {err:.2e} "
                  f"(update size {step:.2e})", flush=True)
            assert np.all(np.isfinite(x_na.cpu().numpy()))
            assert err <= 1e-6
