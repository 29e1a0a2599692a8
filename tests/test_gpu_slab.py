"""GPU parity of the streamed slab reconstruction against the FP64 oracle.

The slab workload produces noisy phantom projections on the GPU, only on the
detector rows the slab reads, filters those rows into 16-view chunk buffers
and back-projects each chunk into a mirror-pair slab while the next chunk is
produced on a second stream. The oracle recomputes the same inputs itself:
analytic line integrals (its own ray tracer), the noise from its own
SplitMix64 + Box-Muller draws (the host generator in `synth`, keyed by view,
row and column), its own filter and its own back-projection.

Tolerances (rel-L2, FP64): 1e-5 with FP32 storage; 2e-3 with FP16 storage
against the unrounded oracle; 1e-5 against the oracle fed the identically
rounded FP16 values (hash inputs)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

fdk = pytest.importorskip("paper_1909_02724_amd")
from paper_1909_02724_amd.pipeline import SlabTiming, reconstruct_slab  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def rel_l2(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def announce(msg):
    print(msg, flush=True)


def slab_slices(g, z0, nzl, slab):
    """Global slice of each slab slice."""
    if slab == "contiguous":
        return np.arange(z0, z0 + nzl)
    h = nzl // 2
    return np.concatenate([np.arange(z0, z0 + h), np.arange(g.nz - z0 - h, g.nz - z0)])


def oracle_sigma(g, ang, ell, rel):
    """rel * the largest clean line integral on row floor(cv), per view."""
    row = math.floor((g.nv - 1) / 2 + g.off_v)
    u = np.arange(g.nu)
    out = np.empty(len(ang))
    for s in range(len(ang)):
        svu = np.stack([np.full(g.nu, s), np.full(g.nu, row), u], 1)
        out[s] = rel * oracle.phantom_project_pixels(g, ang, svu, ell).max()
    return out


def oracle_noisy_rows(g, ang, ell, sigma, seed, rows, view_ids):
    """Noisy line integrals of detector rows rows = [(s, v)], s indexing
    `ang`; the noise is keyed by the global view number view_ids[s]."""
    rows = np.asarray(rows, np.int64).reshape(-1, 2)
    u = np.arange(g.nu)
    svu = np.stack([np.repeat(rows[:, 0], g.nu), np.repeat(rows[:, 1], g.nu),
                    np.tile(u, len(rows))], 1)
    clean = oracle.phantom_project_pixels(g, ang, svu, ell).reshape(len(rows), g.nu)
    vid = np.asarray(view_ids)[rows[:, 0]]
    noise = synth.normal_draws(seed, g, vid[:, None], rows[:, 1:2], u[None, :])
    return clean + sigma[rows[:, 0]][:, None] * noise


def synth_producer(g, ang, ell, seed, rel):
    """GPU producer: noisy phantom rows from the synth GPU generator."""
    import synth.gpu as sg
    ang_d = torch.as_tensor(ang, dtype=torch.float64, device=DEV)
    ell_d = torch.as_tensor(np.ascontiguousarray(ell).reshape(-1), dtype=torch.float64,
                            device=DEV)
    sigma_d = sg.view_sigma(g, ang, ell, rel, device=DEV) if rel else None

    def produce(view0, n, bands, e_bands):
        for (v0, nr), e in zip(bands, e_bands):
            sg.phantom_rows(g, ang_d[view0:view0 + n], ell_d, v0, e, view_index0=view0,
                            seed=seed, sigma=None if sigma_d is None else sigma_d[view0:view0 + n])
    return produce, sigma_d


SMALL = synth.Geom(nx=48, ny=40, nz=36, nu=64, nv=60, sod=300.0, sdd=600.0, du=1.5, dv=1.5)


def test_noisy_rows_and_sigma_match_oracle():
    import synth.gpu as sg
    for g in (SMALL, synth.config("slab4096")["geom"]):
        ang = synth.angles(12, start=0.4)
        ell = synth.ellipsoids(7, 6, g)
        sig_ref = oracle_sigma(g, ang, ell, 0.01)
        sig = sg.view_sigma(g, ang, ell, 0.01, device=DEV).cpu().numpy()
        # two FP64 ray tracers written independently: near-tangent chords
        # amplify last-bit differences in the ray direction
        rd = float(np.max(np.abs(sig - sig_ref) / sig_ref))
        announce(f"view sigma nu={g.nu}: max relative difference {rd:.2e}")
        assert rd <= 1e-8
        v0, nr = g.nv // 3, 5
        e = torch.empty((6, nr, g.nu), dtype=torch.float32, device=DEV)
        produce, sigma_d = synth_producer(g, ang, ell, 77, 0.01)
        produce(4, 6, [(v0, nr)], [e])
        got = e.double().cpu().numpy()
        rows = [(s, v) for s in range(4, 10) for v in range(v0, v0 + nr)]
        ref = oracle_noisy_rows(g, ang, ell, sig_ref, 77, rows, np.arange(12))
        ref = ref.reshape(6, nr, g.nu)
        # FP32 storage of FP64 values: half an ulp, plus last-bit libm differences
        assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref).max() + 1e-7), g
        announce(f"noisy rows nu={g.nu}: max |diff| {np.abs(got - ref).max():.2e}")


@pytest.mark.parametrize("slab, z0, nzl", [("mirror_pair", 3, 12), ("contiguous", 4, 10),
                                           ("mirror_pair", 0, 36)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_streamed_slab_matches_oracle(slab, z0, nzl, dtype):
    """Every voxel of a small slab from 40 views streamed in chunks of 16
    (the last one ragged) and back-projected in launches of up to 32 views
    (32 + 8), rows outside the slab's bands never produced."""
    g = SMALL
    n = 40
    ang = synth.angles(n, start=0.2)
    ell = synth.ellipsoids(31, 8, g)
    seed, rel = 91, 0.01
    scale = oracle.fdk_scale(g, n)
    produce, _ = synth_producer(g, ang, ell, seed, rel)
    announce(f"streamed slab {slab} z0={z0} nz_local={nzl} {dtype}")
    vol = reconstruct_slab(g, ang, produce, z0=z0, nz_local=nzl, slab=slab, chunk=16,
                           batch=32, dtype=dtype, kind="shepp-logan", scale=scale, device=DEV)
    torch.cuda.synchronize()
    sig = oracle_sigma(g, ang, ell, rel)
    rows = [(s, v) for s in range(n) for v in range(g.nv)]
    e = oracle_noisy_rows(g, ang, ell, sig, seed, rows, np.arange(n)).reshape(n, g.nv, g.nu)
    q = oracle.filter(g, e.astype(np.float32).astype(np.float64), "shepp-logan")
    ks = slab_slices(g, z0, nzl, slab)
    ii, jj, kk = np.meshgrid(np.arange(g.nx), np.arange(g.ny), ks, indexing="ij")
    vox = np.ascontiguousarray(np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int64))
    ref = oracle.backproject(g, ang, q, scale=scale, voxels=vox)
    loc = np.searchsorted(ks, vox[:, 2])  # ks is ascending
    got = vol.double().cpu().numpy()[loc, vox[:, 1], vox[:, 0]]
    err = rel_l2(got, ref)
    announce(f"  rel-L2 {err:.3e}")
    assert err <= (1e-5 if dtype == torch.float32 else 2e-3)


def c4_clusters(g, ks, seed, n_clusters=8, side=8, depth=8):
    """n_clusters blocks of side x side columns x depth consecutive slab
    slices (inside one half of the mirror pair), at seeded places that
    include both ends of each half: n_clusters * side^2 * depth voxels whose
    taps need only a few hundred detector rows per view, so the oracle can
    recompute every row they read."""
    rng = np.random.default_rng(seed)
    half = ks.size // 2
    starts = [0, half - depth, half, ks.size - depth]
    starts += list(rng.integers(0, half - depth, (n_clusters - 4) // 2))
    starts += list(half + rng.integers(0, half - depth, n_clusters - len(starts)))
    out = []
    for c, t0 in enumerate(starts):
        i0 = int(rng.integers(0, g.nx - side)) if c % 3 else 0   # some at the volume's edge
        j0 = int(rng.integers(0, g.ny - side))
        for t in range(depth):
            for j in range(j0, j0 + side):
                for i in range(i0, i0 + side):
                    out.append((i, j, ks[t0 + t]))
    return np.ascontiguousarray(np.array(out, dtype=np.int64))


def c4_voxels(g, ks, seed, n):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, g.nx, n)
    j = rng.integers(0, g.ny, n)
    k = ks[rng.integers(0, ks.size, n)]
    k[:4] = [ks[0], ks[ks.size // 2 - 1], ks[ks.size // 2], ks[-1]]  # slab edges
    return np.ascontiguousarray(np.stack([i, j, k], 1).astype(np.int64))


@pytest.mark.slow
def test_slab4096_streamed_pipeline_sampled():
    """The 4096^2 mirror-pair slab (256 slices at z0 = 0), FP16 chunks of 16
    views, noisy 64-ellipsoid phantom generated and filtered on the GPU on
    the slab's row bands only; four chunks spread over the orbit (64 views)
    so the oracle can recompute every row the sampled voxels read."""
    c = synth.config("slab4096")
    g = c["geom"]
    ang = synth.angles(c["np"])
    sl = c["slab"]
    ell = synth.ellipsoids(c["seed"], c["n_ell"], g)
    seed, rel = c["noise_seed"], c["noise"]
    scale = oracle.fdk_scale(g, c["np"])
    chunks = [0, 1024, 2048, 3072]
    produce, _ = synth_producer(g, ang, ell, seed, rel)
    announce("slab4096: streamed GPU reconstruction, 4 chunks of 16 views")
    vol = reconstruct_slab(g, ang, produce, z0=sl["z0"], nz_local=sl["nz_local"],
                           slab=sl["kind"], chunk=c["B"], dtype=torch.float16,
                           kind=c["filter"], scale=scale, chunks=chunks, device=DEV)
    ks = slab_slices(g, sl["z0"], sl["nz_local"], sl["kind"])
    vox = c4_clusters(g, ks, 205)
    announce(f"slab4096: {len(vox)} sampled voxels in 8 clusters")
    loc = np.searchsorted(ks, vox[:, 2])
    idx = torch.from_numpy(np.stack([loc, vox[:, 1], vox[:, 0]])).to(DEV)
    got = vol[idx[0], idx[1], idx[2]].double().cpu().numpy()
    del vol
    torch.cuda.empty_cache()
    views = np.concatenate([np.arange(v0, v0 + c["B"]) for v0 in chunks])
    angs = ang[views]
    # rows the sampled voxels tap in each view (Alg. 3), by the oracle's matrices
    h = np.concatenate([vox.T.astype(np.float64), np.ones((1, len(vox)))])
    need = set()
    for s, beta in enumerate(angs):
        _, y, z = oracle.projection_matrix(g, beta) @ h
        nv = np.floor(y / z).astype(np.int64)
        for r in np.concatenate([nv, nv + 1]):
            if 0 <= r < g.nv:
                need.add((s, int(r)))
    rows = sorted(need)
    announce(f"slab4096: oracle recomputes {len(rows)} detector rows")
    sig = oracle_sigma(g, angs, ell, rel)
    e = oracle_noisy_rows(g, angs, ell, sig, seed, rows, views)
    qr = oracle.filter_rows(g, e.astype(np.float32).astype(np.float64),
                            [v for _, v in rows], c["filter"])
    q = np.zeros((len(views), g.nv, g.nu))  # untouched rows stay unmapped zero pages
    for m, (s, v) in enumerate(rows):
        q[s, v] = qr[m]
    ref = oracle.backproject(g, angs, q, scale=scale, voxels=vox)
    err = rel_l2(got, ref)
    announce(f"slab4096 streamed FP16: rel-L2 vs FP64 oracle {err:.3e}")
    assert err <= 2e-3


@pytest.mark.slow
def test_slab4096_all_views_hash_sampled():
    """Back-projection at the slab's full shape: all 4096 views, FP16, 96
    views per launch (the launch configuration the slab benchmark times:
    six 16-view chunks per launch, the last launch 64 views), with
    SplitMix64 values both sides regenerate, on sampled voxels."""
    import synth.gpu as sg
    c = synth.config("slab4096")
    g = c["geom"]
    n = c["np"]
    ang = synth.angles(n)
    sl = c["slab"]
    seed = 4096
    B = 96  # views per launch
    vol = torch.empty((sl["nz_local"], g.ny, g.nx), dtype=torch.float32, device=DEV)
    qc = torch.empty((B, g.nv, g.nu), dtype=torch.float16, device=DEV)
    announce("slab4096: 43 launches of up to 96 hashed FP16 views into the 16 GiB slab")
    for view0 in range(0, n, B):
        m = min(B, n - view0)
        sg.hash_fill(qc[:m], seed, counter0=view0 * g.nv * g.nu)
        fdk.backproject(qc[:m], g, ang, view0=view0, out=vol, z0=sl["z0"], nz_local=sl["nz_local"],
                        slab=sl["kind"], accumulate=view0 > 0)
    ks = slab_slices(g, sl["z0"], sl["nz_local"], sl["kind"])
    vox = c4_voxels(g, ks, 206, 4096)
    loc = np.searchsorted(ks, vox[:, 2])
    idx = torch.from_numpy(np.stack([loc, vox[:, 1], vox[:, 0]])).to(DEV)
    got = vol[idx[0], idx[1], idx[2]].double().cpu().numpy()
    del vol, qc
    torch.cuda.empty_cache()
    announce(f"slab4096: oracle on {len(vox)} voxels x {n} views")
    ref16 = oracle.backproject(g, ang, seed=seed, rnd="f16", voxels=vox)
    ref32 = oracle.backproject(g, ang, seed=seed, voxels=vox)
    e_same, e_f32 = rel_l2(got, ref16), rel_l2(got, ref32)
    announce(f"slab4096 hash FP16: rel-L2 vs rounded-input oracle {e_same:.3e}, "
             f"vs FP32-input oracle {e_f32:.3e}")
    assert e_same <= 1e-5
    assert e_f32 <= 2e-3


def test_reconstruct_slab_timing_and_empty():
    g = SMALL
    ang = synth.angles(20)
    produce, _ = synth_producer(g, ang, synth.ellipsoids(3, 4, g), 5, 0.0)
    t = SlabTiming()
    vol = reconstruct_slab(g, ang, produce, z0=2, nz_local=6, slab="mirror_pair", chunk=8,
                           batch=8, dtype=torch.float32, scale=1.0, device=DEV, timing=t)
    assert len(t.bp_ms) == 3 and all(x > 0 for x in t.bp_ms) and t.wall_ms >= sum(t.bp_ms) * 0.5
    assert float(vol.abs().max()) > 0
    # gathering chunks into launches of up to 16 views changes only rounding
    t2 = SlabTiming()
    vol16 = reconstruct_slab(g, ang, produce, z0=2, nz_local=6, slab="mirror_pair", chunk=8,
                             batch=16, dtype=torch.float32, scale=1.0, device=DEV, timing=t2)
    assert len(t2.bp_ms) == 2
    assert rel_l2(vol16.double().cpu().numpy(), vol.double().cpu().numpy()) <= 1e-6
    # no chunks: the slab is zero
    vol2 = reconstruct_slab(g, ang, produce, z0=2, nz_local=6, slab="mirror_pair", chunk=8,
                            chunks=[], out=vol, device=DEV)
    torch.cuda.synchronize()
    assert float(vol2.abs().max()) == 0.0
