"""HIP graph capture of the library's entry points (torch.cuda.graph on the
caller's stream): every entry point is capturable, since none allocates,
copies, synchronises or sets memory with a memset. Each graph is replayed
several times with eager work and synchronisations in between, and every
replay is checked against the eager result: bit for bit where the kernels
are deterministic (filter, back-projection), to 1e-6 where FP32 global
atomics order the sums (forward projection, SIRT)."""
import numpy as np
import pytest
import torch

import synth

fdk = pytest.importorskip("paper_1909_02724_amd")

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def announce(msg):
    print(msg, flush=True)


def capture(fn):
    """Warm up on a side stream, then capture fn into a graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    return graph


def rel(a, b):
    return float((a.double() - b.double()).norm() / b.double().norm())


def test_fdk64_graph_replays_bitwise():
    """Filter + back-projection of the 64^3 scan in one graph; replays equal
    the eager result exactly, and an input doubled in place doubles the
    output exactly (both stages are linear; scaling by 2 is exact)."""
    c = synth.config("fdk64")
    g, ang = c["geom"], synth.angles(c["np"])
    announce("graph fdk64")
    rng = np.random.default_rng(61)
    e = torch.from_numpy(rng.uniform(0, 5, (c["np"], g.nv, g.nu)).astype(np.float32)).to(DEV)
    q = torch.empty_like(e)
    vol = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=DEV)
    sc = fdk.fdk_scale(g, ang)

    def step():
        fdk.filter(e, g, ang, kind="ramlak", out=q)
        fdk.backproject(q, g, ang, out=vol, scale=sc)

    step()
    torch.cuda.synchronize()
    ref = vol.clone()
    graph = capture(step)
    for k in range(3):
        vol.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(vol, ref), f"replay {k}"
    e.mul_(2.0)
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(vol, 2.0 * ref)


def test_fft_filter_8192_graph():
    """The 8192-point FFT filter (70 KB of LDS, raised once per device before
    capture) and an FP16 store, captured and replayed."""
    g = synth.Geom(nx=64, ny=64, nz=64, nu=4096, nv=5, sod=4.0e4, sdd=8.0e4)
    ang = synth.angles(3)
    announce("graph filter nu=4096")
    e = torch.empty((3, g.nv, g.nu), dtype=torch.float32, device=DEV).uniform_(0.0, 3.0)
    q = torch.empty((3, g.nv, g.nu), dtype=torch.float16, device=DEV)
    fdk.filter(e, g, ang, kind="shepp-logan", out=q)
    torch.cuda.synchronize()
    ref = q.clone()
    graph = capture(lambda: fdk.filter(e, g, ang, kind="shepp-logan", out=q))
    for k in range(3):
        q.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(q, ref), f"replay {k}"


def test_forward_projection_and_sirt_graph():
    """Forward projection, and a SIRT iteration (fills, max-reduction,
    inversion, both projectors, fused element-wise steps) captured and
    replayed against eager runs from the same state."""
    g = synth.Geom(nx=40, ny=36, nz=24, nu=56, nv=40, sod=300.0, sdd=600.0, du=1.5, dv=1.5)
    ang = synth.angles(30)
    announce("graph forward projection and SIRT")
    rng = np.random.default_rng(62)
    x = torch.from_numpy(rng.uniform(0, 1, (g.nz, g.ny, g.nx)).astype(np.float32)).to(DEV)
    qf = torch.empty((30, g.nv, g.nu), dtype=torch.float32, device=DEV)
    fdk.forward_project(x, g, ang, out=qf)
    torch.cuda.synchronize()
    ref = qf.clone()
    graph = capture(lambda: fdk.forward_project(x, g, ang, out=qf))
    for k in range(3):
        qf.fill_(7.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert rel(qf, ref) <= 1e-6, f"replay {k}"

    p = ref.clone()
    row_inv, col_inv = fdk.sirt_weights(g, ang, device=DEV)
    proj_tmp, vol_tmp = torch.empty_like(p), torch.empty_like(x)
    xs = torch.zeros_like(x)

    def it():
        fdk.sirt_iteration(xs, p, row_inv, col_inv, g, ang, lam=0.9, nonneg=True,
                           proj_tmp=proj_tmp, vol_tmp=vol_tmp)

    x0 = torch.zeros_like(x)
    xs.copy_(x0)
    it()
    it()
    torch.cuda.synchronize()
    eager2 = xs.clone()
    graph2 = capture(it)  # the warm-up and capture advance xs by one iteration
    for k in range(3):
        xs.copy_(x0)
        torch.cuda.synchronize()
        graph2.replay()
        graph2.replay()
        torch.cuda.synchronize()
        assert rel(xs, eager2) <= 1e-6, f"replay pair {k}"
