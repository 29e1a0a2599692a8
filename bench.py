#!/usr/bin/env python3
"""Back-projection benchmark: GUPS of the FDK back-projector on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload bp2048|slab4096]

Workload (default): 2048^3 FP32 volume, 2048 views of 2048^2 pixels over a
full circle, in 22 launches of 93 or 94 views. A step is one complete back-projection
of all 2048 views into the volume (every voxel x view update, 2^44 of them),
with the filtered projections already resident in HBM. GUPS is
Nx*Ny*Nz*Np / (T * 2^30), T the kernel time of the step, measured with HIP
events on the stream the library launches on (host-device copies excluded).

Beside the FP32 figure the line reports FP16 and BF16 projection storage
(FP32 accumulation) and the matched adjoint forward projector on the same
workload, the dominant kernel against its roofline, and the FP64 CPU oracle
timed on a bounded sample of the same workload on this host.

Inputs are synthetic and seeded: the analytic line integrals of a sum of 32
random ellipsoids (stand-in for the paper's Shepp-Logan projections),
cosine-weighted and Shepp-Logan filtered by the library's own filter.

Workload slab4096: one GPU's share of a 4096^3 reconstruction, a mirror pair
of 128-slice slabs at the volume's top and bottom (16 GiB), from 4096 views
of 4096^2 pixels streamed in 16-view FP16 chunks: the noisy 64-ellipsoid
line integrals (noise 1%) of the slab's detector row bands are generated
into HBM first (untimed); then a producer stream filters them chunk by chunk
into FP16 buffers while the previous 96 views (six chunks) back-project. A step is one pass over all 4096 views; GUPS counts
the back-projection launches' event time (the rate the paper reports) and,
beside it, the whole pipeline's wall time. The default run adds one such
pass to its line (--no-slab skips it), and the time of a SIRT iteration
(forward projection, weighted residual, back-projection, update) at 256^3
from 360 views of 384^2 (--no-sirt skips it), and the other workloads of the
scan list (64^3 FDK, 512^3 back-projection, one forward and backward step on
four 256^3 volumes; --no-configs skips them).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "back-projection GUPS at 2048³/2048 views; FP16-store vs FP32; adjoint GUPS"

# Chip constants (MI355X, gfx950), measured with one-kernel microbenchmarks:
# 256 CUs at 2.4 GHz; a SIMD retires a 64-lane FP32 add, multiply or FMA (and
# moves, bitwise ops, 32-bit integer adds) every 2 clocks, 4 SIMDs per CU ->
# 128 lane-ops/clk/CU, the 157.3 TFLOP/s FP32 vector peak; conversions,
# fractions, shifts and 3-operand integer ops take 4 clocks (half rate).
# Scheme op counts below are in full-rate equivalents (a half-rate op
# counts 2).
N_CU, CLOCK_HZ, VALU_LANES_PER_CLK = 256, 2.4e9, 128
# LDS: a conflict-free 64-lane ds_read_b128 every 4.6 clocks per CU
# (222.6 B/clk/CU at 2.4 GHz); a 64-lane 64-bit integer LDS add every 6.4
# clocks (79.6 B/clk/CU of read-modify-write).
LDS_BYTES_PER_CLK = 222.6
LDS_ATOMIC64_BYTES_PER_CLK = 79.6
HBM_PEAK = 8.0e12
# VALU work per voxel-view update of the mirrored, difference-staged scheme:
# per voxel pair v (1 FMA), truncation, fraction and tap address (3 half
# rate, shared); per voxel two u-interpolations (1 FMA each on the staged
# difference), one v-interpolation (2) and the weighted accumulate (1):
# (1 + 2 * 3 + 2 * 5) / 2 = 8.5 full-rate equivalents.
VALU_OPS_PER_UPDATE = 8.5
LDS_BYTES_PER_UPDATE = 16.0  # 4 FP32 taps (value and u-difference of two rows)
# The adjoint's scheme (fixed-point tile, a row's and its mirror row's sums
# in one 64-bit word), in full-rate equivalents: per voxel W S x (1), the
# row split (2), four tap weights (4) and four round-to-fixed conversions
# (half rate: 8) -> 15; per voxel pair v (1), truncation, fraction and
# address (half rate: 6) -> 7, and for each of the four 64-bit adds the sign
# carry of the low half (a shift, half rate, and an add: 3) -> 12; per
# update (2 * 15 + 7 + 12) / 2 = 24.5, and two 8-byte LDS read-modify-writes
# (16 bytes).
ADJ_VALU_OPS_PER_UPDATE = 24.5
ADJ_LDS_BYTES_PER_UPDATE = 16.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "bp_tiled_mirror_kernel_bp2048_traffic.json")
# Most views per launch of the library's back-projector and adjoint (the
# volume is read, and written, once per launch); a call's views are split
# evenly over the fewest launches.
BP_VIEWS_PER_LAUNCH = 96
ADJ_VIEWS_PER_LAUNCH = 64
# Slab workload: views are filtered in 16-view chunks; six contiguous chunks
# make one back-projection launch.
SLAB_VIEWS_PER_LAUNCH = 96


def profiled_counters(workload):
    """The committed rocprofv3 record of the back-projection kernel at
    2048^3: HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE passes
    (scaled by the calibration copy) and VALU instructions per launch, or
    None (each) if the kernel sources changed since they were taken."""
    import hashlib
    if workload != "bp2048" or not os.path.exists(TRAFFIC_RECORD):
        return None, None
    rec = json.load(open(TRAFFIC_RECORD))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None, None
    traffic = (rec["fetch_size_kib_per_dispatch"] * rec["copy_read_factor"] +
               rec["write_size_kib_per_dispatch"] * rec["copy_write_factor"]) * 1024.0
    valu = rec.get("sq_insts_valu_per_dispatch")
    return traffic, valu


def gups(updates: float, seconds: float) -> float:
    return updates / (seconds * 2.0 ** 30)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bp2048")
    ap.add_argument("--adjoint-views", type=int, default=256,
                    help="views of the adjoint timing, evenly spaced over the full circle "
                         "(a rate, reported per update)")
    ap.add_argument("--no-16bit", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 64^3, 512^3 and differentiable 256^3 legs of the default run")
    ap.add_argument("--no-sirt", action="store_true",
                    help="skip the SIRT leg (256^3, 360 views) of the default run")
    ap.add_argument("--no-filter", action="store_true",
                    help="skip the filtering leg (2048- and 4096-pixel rows) of the default run")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip the streamed 4096^2-slab leg of the default run")
    ap.add_argument("--ablation", action="store_true",
                    help="also time the back-projector without mirror pairs and without LDS "
                         "staging (2048^3, 64 views)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--oracle-configs", action="store_true",
                    help="also time the oracle on whole volumes: 512^3 from 512 views (~2 min on "
                         "16 threads) and one 256^3 volume from 360 views")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a buffer of this many MiB (a plain copy of known size, "
                         "whose HBM counters scale the kernel's)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def slab_pass(g, cfg, ang, produce, vol, scale, timing_cls, reconstruct_slab, torch):
    t = timing_cls()
    sl = cfg["slab"]
    reconstruct_slab(g, ang, produce, z0=sl["z0"], nz_local=sl["nz_local"], slab=sl["kind"],
                     chunk=cfg["B"], batch=SLAB_VIEWS_PER_LAUNCH, dtype=torch.float16,
                     kind=cfg["filter"], scale=scale, out=vol, timing=t)
    return t


def run_slab(steps, warmup, dev):
    """Streamed slab reconstruction; returns (bp_ms, wall_ms, launches) per
    pass (means over the timed passes) and the workload's geometry."""
    import numpy as np
    import torch

    import paper_1909_02724_amd as fdk
    import synth
    import synth.gpu as sg
    from paper_1909_02724_amd.pipeline import SlabTiming, reconstruct_slab

    cfg = synth.config("slab4096")
    g = cfg["geom"]
    ang = synth.angles(cfg["np"])
    sl = cfg["slab"]
    ell = synth.ellipsoids(cfg["seed"], cfg["n_ell"], g)
    ang_d = torch.as_tensor(ang, dtype=torch.float64, device=dev)
    ell_d = torch.as_tensor(np.ascontiguousarray(ell).reshape(-1), dtype=torch.float64, device=dev)
    sigma_d = sg.view_sigma(g, ang, ell, cfg["noise"], device=dev)
    bands = fdk.slab_rows(g, ang, z0=sl["z0"], nz_local=sl["nz_local"], slab=sl["kind"])
    log(f"slab4096: {g.nx}x{g.ny} x {sl['nz_local']} mirror-pair slab, {cfg['np']} views "
        f"of {g.nv}x{g.nu} in FP16 chunks of {cfg['B']}; row bands {bands}")

    # Inputs resident in HBM before timing: the noisy line integrals of every
    # view on the slab's row bands (2 x 289 rows of 4096 at 4096^2, 39 GB).
    store = [torch.empty((cfg["np"], nr, g.nu), dtype=torch.float32, device=dev)
             for _, nr in bands]
    for s0 in range(0, cfg["np"], 64):
        n = min(64, cfg["np"] - s0)
        for (v0, nr), st in zip(bands, store):
            sg.phantom_rows(g, ang_d[s0:s0 + n], ell_d, v0, st[s0:s0 + n], view_index0=s0,
                            seed=cfg["noise_seed"], sigma=sigma_d[s0:s0 + n])
    torch.cuda.synchronize()
    log(f"slab4096: band rows of all views generated ({sum(x.numel() for x in store) * 4 / 1e9:.1f} GB)")

    def produce(view0, n, bands, e_bands):
        return [st[view0:view0 + n] for st in store]

    scale = fdk.fdk_scale(g, ang)
    vol = torch.empty((sl["nz_local"], g.ny, g.nx), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        slab_pass(g, cfg, ang, produce, vol, scale, SlabTiming, reconstruct_slab, torch)
    torch.cuda.synchronize()
    bp, wall = [], []
    for k in range(steps):
        t = slab_pass(g, cfg, ang, produce, vol, scale, SlabTiming, reconstruct_slab, torch)
        bp.append(sum(t.bp_ms))
        wall.append(t.wall_ms)
        log(f"slab4096 pass {k}: back-projection {bp[-1]:.1f} ms over {len(t.bp_ms)} launches, "
            f"pipeline {wall[-1]:.1f} ms")
    n_launch = len(t.bp_ms)
    del vol, store
    torch.cuda.empty_cache()
    return sum(bp) / len(bp), sum(wall) / len(wall), n_launch, g, cfg


def run_sirt(dev, iters=10):
    """SIRT on the 256^3 / 360-view geometry: weights once, then `iters`
    iterations (one forward projection and one back-projection each),
    event-timed on the launch stream."""
    import torch

    import paper_1909_02724_amd as fdk
    import synth
    import synth.gpu as sg

    cfg = synth.config("diff256")
    g = cfg["geom"]
    ang = synth.angles(cfg["np"])
    ell = synth.ellipsoids(cfg["seed"], 16, g)
    p = sg.phantom_project(g, ang, ell, device=dev)
    stream = torch.cuda.current_stream(dev)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    row_inv, col_inv = fdk.sirt_weights(g, ang, device=dev)
    e1.record(stream)
    x = torch.zeros_like(col_inv)
    pt, vt = torch.empty_like(p), torch.empty_like(x)
    fdk.sirt_iteration(x, p, row_inv, col_inv, g, ang, proj_tmp=pt, vol_tmp=vt)  # warm
    torch.cuda.synchronize()
    e1b = torch.cuda.Event(enable_timing=True)
    e1b.record(stream)
    for _ in range(iters):
        fdk.sirt_iteration(x, p, row_inv, col_inv, g, ang, proj_tmp=pt, vol_tmp=vt)
    e2.record(stream)
    torch.cuda.synchronize()
    it_ms = e1b.elapsed_time(e2) / iters
    ups = 2.0 * g.nx * g.ny * g.nz * cfg["np"]
    log(f"sirt256: weights {e0.elapsed_time(e1):.1f} ms, {it_ms:.2f} ms per iteration "
        f"({gups(ups, it_ms / 1e3):.1f} GUPS over both passes)")
    return {"sirt256_iter_ms": round(it_ms, 3), "sirt256_gups": round(gups(ups, it_ms / 1e3), 1),
            "sirt256_weights_ms": round(e0.elapsed_time(e1), 2)}


def run_configs(dev):
    """The other workloads of the scan list, each timed with HIP events on
    the launch stream (inputs resident): the 64^3 FDK (filter and
    back-projection), the 512^3 back-projection from 512 views, and one
    training step (forward back-projection and matched backward) on the
    batch of four 256^3 volumes from 360 views."""
    import numpy as np
    import torch

    import paper_1909_02724_amd as fdk
    import synth
    import synth.gpu as sg

    stream = torch.cuda.current_stream(dev)
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # 64^3 FDK from 64 views of 64^2, Ram-Lak
    c = synth.config("fdk64")
    g, ang = c["geom"], synth.angles(c["np"])
    e = sg.phantom_project(g, ang, synth.ellipsoids(c["seed"], c["n_ell"], g), device=dev)
    q = torch.empty_like(e)
    vol = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=dev)
    sc = fdk.fdk_scale(g, ang)

    def fdk64():
        fdk.filter(e, g, ang, kind="ramlak", out=q)
        fdk.backproject(q, g, ang, out=vol, scale=sc)
    ms = timed(fdk64, 20)
    out["fdk64_ms"] = round(ms, 4)
    out["fdk64_gups"] = round(gups(float(g.nx) * g.ny * g.nz * c["np"], ms / 1e3), 2)
    # the same two launches replayed from a HIP graph (launch overhead removed)
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        fdk64()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fdk64()
    out["fdk64_graph_ms"] = round(timed(graph.replay, 50), 4)
    del graph
    # 512^3 back-projection from 512 views of 512^2
    c = synth.config("bp512")
    g, ang = c["geom"], synth.angles(c["np"])
    e = sg.phantom_project(g, ang, synth.ellipsoids(c["seed"], c["n_ell"], g), device=dev)
    q = fdk.filter(e, g, ang, kind=c["filter"])
    del e
    vol = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=dev)
    ms = timed(lambda: fdk.backproject(q, g, ang, out=vol), 3)
    out["bp512_ms"] = round(ms, 3)
    out["bp512_gups"] = round(gups(float(g.nx) * g.ny * g.nz * c["np"], ms / 1e3), 1)
    del q, vol
    # differentiable batch: 4 x 256^3 from 360 views of 384^2, forward + backward
    c = synth.config("diff256")
    g, ang = c["geom"], synth.angles(c["np"])
    rng = np.random.default_rng(c["seed"])
    qb = torch.from_numpy(rng.standard_normal((c["batch"], c["np"], g.nv, g.nu),
                                              dtype=np.float32)).to(dev).requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((c["batch"], g.nz, g.ny, g.nx),
                                             dtype=np.float32)).to(dev)
    scale = fdk.fdk_scale(g, ang)

    def step():
        qb.grad = None
        (fdk.fdk_backprojection(qb, g, ang, scale) * w).sum().backward()
    ms = timed(step, 3)
    out["diff256_step_ms"] = round(ms, 2)
    log(f"configs: fdk64 {out['fdk64_ms']} ms ({out['fdk64_gups']} GUPS; {out['fdk64_graph_ms']} ms "
        f"replayed from a graph), bp512 {out['bp512_ms']} ms "
        f"({out['bp512_gups']} GUPS), diff256 forward+backward {out['diff256_step_ms']} ms")
    return out


def run_filter(dev):
    """The filtering stage alone (cosine weight and Shepp-Logan ramp), HBM
    resident in and out, timed with HIP events on the launch stream: 256
    views of 2048^2 (FP32 to FP32, 4096-point FFTs) and the slab
    reconstruction's rows, 256 views x 578 rows of 4096 (FP32 to FP16,
    8192-point FFTs); the median of nine timed calls after three untimed
    ones. Algorithmic bytes: one read of each input pixel and one write of
    each output pixel."""
    import torch

    import paper_1909_02724_amd as fdk
    import synth

    stream = torch.cuda.current_stream(dev)
    out = {}
    for name, nu, nv, dt, ob in (("filter2048", 2048, 2048, torch.float32, 4),
                                 ("filter4096", 4096, 578, torch.float16, 2)):
        g = synth.Geom(nx=64, ny=64, nz=64, nu=nu, nv=nv, sod=1.0e3, sdd=1.5e3, du=1.0, dv=1.0)
        nviews = 256
        ang = synth.angles(nviews)
        e = torch.empty((nviews, nv, nu), dtype=torch.float32, device=dev).uniform_(0.0, 4.0)
        q = torch.empty((nviews, nv, nu), dtype=dt, device=dev)
        for _ in range(3):  # the first calls run at lower clocks
            fdk.filter(e, g, ang, kind="shepp-logan", out=q)
        torch.cuda.synchronize()
        times = []
        for _ in range(9):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fdk.filter(e, g, ang, kind="shepp-logan", out=q)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms = sorted(times)[len(times) // 2]
        gbs = float(nviews) * nv * nu * (4 + ob) / (ms / 1e3) / 1e9
        out[f"{name}_ms"] = round(ms, 3)
        out[f"{name}_GBps"] = round(gbs, 1)
        out[f"{name}_hbm_frac"] = round(gbs / (HBM_PEAK / 1e9), 4)
        log(f"{name}: {nviews} views of {nv}x{nu} in {ms:.2f} ms, {gbs:.0f} GB/s "
            f"({gbs / (HBM_PEAK / 1e9):.3f} of HBM peak)")
        del e, q
    torch.cuda.empty_cache()
    return out


def run_ablation(dev):
    """What each part of the kernel's design contributes, on the 2048^3
    geometry with 64 views of FP32 projections spread evenly over the circle
    (the kernels' speed varies with the view angle): the tiled kernel with
    mirror pairs (Theorem 1), the same without mirror pairs (a fractional
    principal-point offset leaves no pixel-aligned mirror, so every slice is
    back-projected on its own), and the direct variant (taps read from
    global memory, no LDS staging; the FDK_DIRECT flag)."""
    import torch

    import paper_1909_02724_amd as fdk
    import synth
    import synth.gpu as sg

    import numpy as np

    c = synth.config("bp2048")
    n = 64
    g0, ang = c["geom"], np.ascontiguousarray(synth.angles(c["np"])[:: c["np"] // n])
    q = sg.hash_fill(torch.empty((n, g0.nv, g0.nu), dtype=torch.float32, device=dev), 5)
    vol = torch.empty((g0.nz, g0.ny, g0.nx), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {}
    for key, g, direct in (("ablation_tiled_mirror_gups", g0, False),
                           ("ablation_tiled_no_mirror_gups", g0.replace(off_v=0.27), False),
                           ("ablation_direct_mirror_gups", g0, True)):
        fdk.backproject(q[:32], g, ang, out=vol, direct=direct)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fdk.backproject(q, g, ang, out=vol, direct=direct)
        b.record(stream)
        torch.cuda.synchronize()
        out[key] = round(gups(float(g.nx) * g.ny * g.nz * n, a.elapsed_time(b) / 1e3), 1)
        log(f"ablation: {key} = {out[key]}")
    del q, vol
    torch.cuda.empty_cache()
    return out


def oracle_configs(oracle, threads):
    """Whole-volume oracle back-projections of the smaller workloads (FP64,
    all threads): 512^3 from 512 views of 512^2 and one 256^3 volume from 360
    views of 384^2."""
    import numpy as np

    import synth
    out = {}
    for name in ("bp512", "diff256"):
        c = synth.config(name)
        g, ang = c["geom"], synth.angles(c["np"])
        q = np.random.default_rng(7).standard_normal((c["np"], g.nv, g.nu))
        t = time.time()
        oracle.backproject(g, ang, q)
        el = time.time() - t
        ups = float(g.nx) * g.ny * g.nz * c["np"]
        out[f"{name}_full_volume_s"] = round(el, 2)
        out[f"{name}_gups"] = round(gups(ups, el), 5)
        log(f"cpu oracle {name}: whole volume in {el:.1f} s ({gups(ups, el):.4f} GUPS, {threads} threads)")
    return out


def roofline_of(ms_step, launches, updates, g, views_per_launch, q_bytes, kernel, traffic,
                valu_insts=None, valu_ops=VALU_OPS_PER_UPDATE, lds_bytes=LDS_BYTES_PER_UPDATE,
                lds_rate=LDS_BYTES_PER_CLK):
    """The kernel against its roofs: VALU issue at the scheme's minimal op
    count per update, LDS bandwidth at its bytes per update (the measured
    ds_read peak), HBM at the algorithmic bytes (the volume read and written
    once per launch, each view read once). `peak` is the lower of the VALU
    and LDS roofs; `bound` stays "alu" (on-chip work, not HBM or MFMA) and
    `binding_roof` names which of the two sets the peak."""
    per_launch_s = ms_step / 1e3 / launches
    updates_per_launch = updates / launches
    achieved = gups(updates_per_launch, per_launch_s)
    valu_rate = N_CU * VALU_LANES_PER_CLK * CLOCK_HZ  # lane-ops per second
    valu_roof = valu_rate / valu_ops / 2 ** 30
    lds_roof = N_CU * lds_rate * CLOCK_HZ / lds_bytes / 2 ** 30
    peak = min(valu_roof, lds_roof)
    nz = updates / (float(g.nx) * g.ny * views_per_launch * launches)
    alg_bytes = updates_per_launch * (8.0 / views_per_launch +
                                      g.nu * g.nv * q_bytes / (g.nx * g.ny * nz))
    out = {
        "bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 1), "unit": "GUPS",
        "frac": round(achieved / peak, 4),
        "traffic": None if traffic is None else round(traffic),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "kernel": kernel, "launches_per_step": launches,
        "avg_launch_ms": round(per_launch_s * 1e3, 3),
        "binding_roof": "lds" if lds_roof < valu_roof else "valu",
        "valu_roof_gups": round(valu_roof, 1), "valu_ops_per_update_scheme": valu_ops,
        "valu_frac": round(achieved / valu_roof, 4),
        "lds_roof_gups": round(lds_roof, 1), "lds_bytes_per_update": lds_bytes,
        "lds_frac": round(achieved / lds_roof, 4),
        "hbm_algorithmic_bytes_per_launch": round(alg_bytes),
        "hbm_frac_algorithmic": round(alg_bytes / per_launch_s / HBM_PEAK, 4),
        "hbm_achieved_GBps": None if traffic is None else round(traffic / per_launch_s / 1e9, 1),
        "hbm_peak_GBps": HBM_PEAK / 1e9,
        "traffic_over_algorithmic": None if traffic is None else round(traffic / alg_bytes, 3),
    }
    if valu_insts is not None:
        # Measured VALU instructions per update at lane level (rocprofv3
        # SQ_INSTS_VALU x 64 lanes, full- and half-rate ops together) and
        # the issue time they would take at the full rate: a lower bound on
        # the VALU busy fraction at the achieved speed.
        ops = valu_insts * 64.0 / updates_per_launch
        out["valu_lane_ops_per_update_measured"] = round(ops, 3)
        out["valu_busy_frac_lower_bound"] = round(achieved * 2 ** 30 * ops / valu_rate, 4)
    return out


def main_slab(args):
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bp_ms, wall_ms, launches, g, cfg = run_slab(args.steps, args.warmup, dev)
    sl = cfg["slab"]
    updates = float(g.nx) * g.ny * sl["nz_local"] * cfg["np"]
    out = {
        "metric": METRIC, "value": round(gups(updates, bp_ms / 1e3), 2), "unit": "GUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(bp_ms, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
        "data": "synthetic: seeded 64-ellipsoid phantom with 1% Gaussian noise, line integrals of "
                "the slab's row bands resident in HBM, Shepp-Logan filtered per 16-view chunk "
                "on a second stream while the previous launch back-projects",
        "config": {"workload": f"slab4096: {g.nx}x{g.ny}x{sl['nz_local']} FP32 mirror-pair slab "
                               f"of a {g.nz}^3 volume, {cfg['np']} views of {g.nv}x{g.nu} FP16 "
                               f"filtered in chunks of {cfg['B']}, up to {SLAB_VIEWS_PER_LAUNCH} per launch",
                   "nx": g.nx, "ny": g.ny, "nz_local": sl["nz_local"], "n_views": cfg["np"],
                   "nu": g.nu, "nv": g.nv, "chunk_views": cfg["B"],
                   "views_per_launch": SLAB_VIEWS_PER_LAUNCH},
        "pipeline_gups": round(gups(updates, wall_ms / 1e3), 2),
        "pipeline_ms_per_step": round(wall_ms, 2),
        "roofline": roofline_of(bp_ms, launches, updates, g, cfg["np"] / launches, 2.0,
                                "bp_tiled_mirror_kernel<f16_t>", None),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path. The workload is "
              "one GPU's share; mirror-pair slabs of the volume shard across GPUs with no "
              "reduction, each GPU receiving every filtered view.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "slab4096":
        return main_slab(args)

    import numpy as np
    import torch

    import paper_1909_02724_amd as fdk
    import synth
    import synth.gpu as sg

    cfg = synth.config(args.workload)
    g = cfg["geom"]
    n_views = cfg["np"]
    ang = synth.angles(n_views)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    updates = float(g.nx) * g.ny * g.nz * n_views
    launches = math.ceil(n_views / BP_VIEWS_PER_LAUNCH)
    bp_vpl = n_views / launches  # views per launch, on average
    log(f"workload {args.workload}: {g.nx}x{g.ny}x{g.nz} volume, {n_views} views of {g.nv}x{g.nu}")
    if args.copy_calibration:
        n = args.copy_calibration * 2 ** 18
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.copy_calibration} MiB read, {args.copy_calibration} MiB written")
        del src, dst

    # ---- inputs: analytic phantom projections, filtered by the library ----
    t0 = time.time()
    ell = synth.ellipsoids(cfg["seed"], cfg["n_ell"], g)
    q32 = torch.empty((n_views, g.nv, g.nu), dtype=torch.float32, device=dev)
    chunk = 256  # the filtering leg's launch size too
    e = torch.empty((chunk, g.nv, g.nu), dtype=torch.float32, device=dev)
    for s in range(0, n_views, chunk):
        n = min(chunk, n_views - s)
        sg.phantom_project(g, ang[s:s + n], ell, out=e[:n])
        fdk.filter(e[:n], g, ang, view0=s, kind=cfg["filter"], out=q32[s:s + n])
    del e
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s")
    scale = fdk.fdk_scale(g, ang)
    vol = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=dev)

    step_ms = {}

    def timed_bp(q, steps, warmup, label):
        for _ in range(warmup):
            fdk.backproject(q, g, ang, out=vol, scale=scale)
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        wall0 = time.time()
        for k in range(steps):
            starts[k].record(stream)
            fdk.backproject(q, g, ang, out=vol, scale=scale)
            ends[k].record(stream)
        torch.cuda.synchronize()
        wall = time.time() - wall0
        ms = [starts[k].elapsed_time(ends[k]) for k in range(steps)]
        log(f"{label}: step ms {['%.1f' % m for m in ms]} (wall {wall:.2f} s)")
        step_ms[label] = ms
        return sum(ms) / len(ms)

    # Accuracy of each storage leg against the FP64 oracle: the same kernel
    # and launch shape on a subset of the views (3 launches of 96 consecutive
    # views at starting angles spread over the circle), sampled voxels.
    nb = BP_VIEWS_PER_LAUNCH
    n_acc = min(3 * nb, n_views)
    acc_views = np.concatenate([np.arange(s0, s0 + nb) for s0 in
                                np.linspace(0, n_views - nb, n_acc // nb).astype(int)])
    acc_ang = np.ascontiguousarray(ang[acc_views])
    acc_vox = synth.sample_voxels(211, g, 16384, columns=4)
    acc_idx = torch.from_numpy(acc_vox).to(dev)
    acc_got = {}

    def sample_subset(q, label):
        qs = q[torch.from_numpy(acc_views).to(dev)]
        fdk.backproject(qs, g, acc_ang, out=vol, scale=scale)
        acc_got[label] = vol[acc_idx[:, 2], acc_idx[:, 1], acc_idx[:, 0]].double().cpu().numpy()
        del qs

    # ---- FP32 storage: the headline figure ----
    ms32 = timed_bp(q32, args.steps, args.warmup, "fp32")
    gups32 = gups(updates, ms32 / 1e3)
    log(f"fp32: {gups32:.1f} GUPS")
    result_extra = {}
    if not args.no_cpu_baseline:
        sample_subset(q32, "fp32")

    if not args.no_16bit:
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            q16 = q32.to(dt)
            ms16 = timed_bp(q16, max(3, args.steps // 2), 1, name)
            result_extra[f"{name}_store_gups"] = round(gups(updates, ms16 / 1e3), 2)
            result_extra[f"{name}_ms_per_step"] = round(ms16, 2)
            result_extra[f"{name}_roofline"] = {
                k: v for k, v in roofline_of(ms16, launches, updates, g, bp_vpl, 2.0,
                                             f"bp_tiled_mirror_kernel<{name}_t>", None).items()
                if k not in ("traffic", "traffic_unit", "hbm_achieved_GBps",
                             "traffic_over_algorithmic")}
            if not args.no_cpu_baseline:
                sample_subset(q16, name)
            del q16
            torch.cuda.empty_cache()

    if acc_got:
        import oracle
        t_acc = time.time()
        ref = oracle.backproject(g, acc_ang, q32[torch.from_numpy(acc_views).to(dev)].cpu()
                                 .numpy().astype(np.float64), scale=scale, voxels=acc_vox)
        for label, got in acc_got.items():
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            result_extra[f"{label}_rel_l2_vs_oracle"] = float(f"{err:.3e}")
            log(f"{label}: rel-L2 {err:.3e} against the FP64 oracle (FP32 inputs), "
                f"{len(acc_vox)} sampled voxels x {n_acc} views")
        result_extra["rel_l2_sample"] = (f"{len(acc_vox)} voxels (seed 211, 4 full z-columns) x "
                                         f"{n_acc} views ({n_acc // nb} launches of {nb} spread "
                                         f"over the circle), oracle fed the FP32 projections")
        log(f"oracle comparison in {time.time() - t_acc:.1f} s")

    if not args.no_adjoint:
        nv_adj = min(args.adjoint_views, n_views)
        # Every (n_views / nv_adj)-th view: the timed views span the whole
        # circle, as the full set does (the cost varies with the angle).
        ang_adj = np.ascontiguousarray(ang[:: max(1, n_views // nv_adj)][:nv_adj])
        x = torch.empty_like(vol).normal_()
        qa = torch.empty((nv_adj, g.nv, g.nu), dtype=torch.float32, device=dev)
        fdk.forward_project(x, g, ang_adj, nviews=nv_adj, out=qa, scale=scale)
        torch.cuda.synchronize()
        reps = 5
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for k in range(reps):
            fdk.forward_project(x, g, ang_adj, nviews=nv_adj, out=qa, scale=scale)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        msl = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
        msa = float(np.median(msl))
        ua = float(g.nx) * g.ny * g.nz * nv_adj
        result_extra["adjoint_gups"] = round(gups(ua, msa / 1e3), 2)
        result_extra["adjoint_gups_mean"] = round(gups(ua, float(np.mean(msl)) / 1e3), 2)
        result_extra["adjoint_views_timed"] = nv_adj
        result_extra["adjoint_reps"] = reps
        result_extra["adjoint_roofline"] = {
            k: v for k, v in roofline_of(msa, math.ceil(nv_adj / ADJ_VIEWS_PER_LAUNCH), ua, g,
                                         ADJ_VIEWS_PER_LAUNCH, 4.0,
                                         "fp_tiled_kernel<true>", None,
                                         valu_ops=ADJ_VALU_OPS_PER_UPDATE,
                                         lds_bytes=ADJ_LDS_BYTES_PER_UPDATE,
                                         lds_rate=LDS_ATOMIC64_BYTES_PER_CLK).items()
            if not (k.startswith("hbm") or k.startswith("traffic"))}
        log(f"adjoint: {result_extra['adjoint_gups']} GUPS (median of {reps}) over {nv_adj} "
            f"views spread over the circle (ms {['%.1f' % m for m in msl]})")
        del x, qa

    # ---- roofline of the dominant kernel (the back-projection launches) ----
    traffic, valu_insts = profiled_counters(args.workload)
    roofline = roofline_of(ms32, launches, updates, g, bp_vpl, 4.0,
                           "bp_tiled_mirror_kernel<float>",
                           traffic, valu_insts)

    if not args.no_sirt and args.workload == "bp2048":
        result_extra.update(run_sirt(dev))

    if not args.no_configs and args.workload == "bp2048":
        result_extra.update(run_configs(dev))

    if not args.no_filter and args.workload == "bp2048":
        result_extra.update(run_filter(dev))

    if args.ablation and args.workload == "bp2048":
        result_extra.update(run_ablation(dev))

    if not args.no_slab and args.workload == "bp2048":
        del q32
        torch.cuda.empty_cache()
        bp_ms, wall_ms, nl, gs, cs = run_slab(1, 0, dev)
        su = float(gs.nx) * gs.ny * cs["slab"]["nz_local"] * cs["np"]
        result_extra["slab4096_f16_gups"] = round(gups(su, bp_ms / 1e3), 2)
        result_extra["slab4096_pipeline_gups"] = round(gups(su, wall_ms / 1e3), 2)
        result_extra["slab4096_bp_ms"] = round(bp_ms, 1)
        result_extra["slab4096_pipeline_ms"] = round(wall_ms, 1)

    # ---- the other legs against the same kernel's roofs ----
    valu_roof = roofline["valu_roof_gups"]
    for key in ("f16_store_gups", "bf16_store_gups", "bp512_gups", "slab4096_f16_gups"):
        if key in result_extra:
            result_extra[key.replace("_gups", "_valu_frac")] = round(result_extra[key] / valu_roof, 4)

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the workload ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(203)
        nv_cpu = 16
        qc = rng.standard_normal((nv_cpu, g.nv, g.nu))
        nvox = 4096
        vox = synth.sample_voxels(203, g, nvox)
        oracle.backproject(g, ang[:nv_cpu], qc, voxels=vox[:256])  # load, warm
        t = time.time()
        done = 0
        while time.time() - t < args.cpu_seconds:
            oracle.backproject(g, ang[:nv_cpu], qc, voxels=vox)
            done += nvox * nv_cpu
        el = time.time() - t
        threads = oracle.num_threads()
        # one thread, briefly, for the per-core rate
        oracle.set_num_threads(1)
        t1, done1 = time.time(), 0
        while time.time() - t1 < args.cpu_seconds / 3:
            oracle.backproject(g, ang[:nv_cpu], qc, voxels=vox[:1024])
            done1 += 1024 * nv_cpu
        el1 = time.time() - t1
        oracle.set_num_threads(threads)
        model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                      if ln.startswith("model name")), "unknown")
        # the 64^3 FDK's whole volume (64 views), all threads
        c1 = synth.config("fdk64")
        g1, a1 = c1["geom"], synth.angles(c1["np"])
        q1 = rng.standard_normal((c1["np"], g1.nv, g1.nu))
        t1 = time.time()
        oracle.backproject(g1, a1, q1)
        el_c1 = time.time() - t1
        rate = gups(done, el)
        cpu = {"value": round(rate, 5), "unit": "GUPS", "cores": threads, "kind": "oracle",
               "sample": f"{done} voxel-view updates ({nvox} random voxels of the "
                         f"{g.nx}x{g.ny}x{g.nz} volume x {nv_cpu} views of {g.nv}x{g.nu}, "
                         f"repeated for {el:.1f} s)",
               "single_thread_gups": round(gups(done1, el1), 5),
               "cpu_model": model, "host_cpus": os.cpu_count(),
               "extrapolated_full_step_s": round(updates / (rate * 2 ** 30), 0),
               "fdk64_full_volume_s": round(el_c1, 4)}
        if args.oracle_configs:
            cpu.update(oracle_configs(oracle, threads))
        log(f"cpu oracle: {cpu['value']} GUPS on {threads} threads, {cpu['single_thread_gups']} on one "
            f"({model}); a full step would take ~{cpu['extrapolated_full_step_s']:.0f} s")

    out = {
        "metric": METRIC, "value": round(gups32, 2), "unit": "GUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms32, 2),
        "ms_per_step_median": round(float(np.median(step_ms["fp32"])), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded 32-ellipsoid phantom, analytic line integrals, "
                "Shepp-Logan filtered on the GPU",
        "config": {"workload": f"{args.workload}: {g.nx}x{g.ny}x{g.nz} FP32 volume, "
                               f"{n_views} views of {g.nv}x{g.nu}, {launches} launches of at most "
                               f"{BP_VIEWS_PER_LAUNCH} views",
                   "nx": g.nx, "ny": g.ny, "nz": g.nz, "n_views": n_views, "nu": g.nu,
                   "nv": g.nv, "views_per_launch": round(bp_vpl, 2)},
        **result_extra,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
