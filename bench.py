#!/usr/bin/env python3
"""Back-projection benchmark: GUPS of the FDK back-projector on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload bp2048]

Workload (default): 2048^3 FP32 volume, 2048 views of 2048^2 pixels over a
full circle, views in launches of 32. A step is one complete back-projection
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

# Chip constants (MI355X, gfx950): 256 CUs at 2.4 GHz; a SIMD retires one
# 64-lane FP32 VALU instruction per 4 clocks, 4 SIMDs per CU -> 64 lane-ops/clk/CU.
N_CU, CLOCK_HZ, VALU_LANES_PER_CLK = 256, 2.4e9, 64
# LDS read bandwidth measured with lds_probe.hip on MI355X: 93.2 TB/s,
# 151.7 B/clk/CU at 2.4 GHz (above the 128 B/clk of the previous generation).
LDS_BYTES_PER_CLK = 151.7
HBM_PEAK = 8.0e12
# VALU work per voxel-view update of the mirrored, difference-staged scheme:
# per voxel pair v, truncation, fraction and tap address (4, shared); per
# voxel two u-interpolations (1 FMA each on the staged difference), one
# v-interpolation (2) and the weighted accumulate (1): (4 + 2 * 5) / 2 = 7.
VALU_OPS_PER_UPDATE = 7.0
LDS_BYTES_PER_UPDATE = 16.0  # 4 FP32 taps (value and u-difference of two rows)
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "bp_tiled_mirror_kernel_bp2048_traffic.json")


def profiled_traffic(workload):
    """HBM bytes per launch of the back-projection kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by the calibration copy),
    or None if the kernel sources changed since they were taken."""
    import hashlib
    if workload != "bp2048" or not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = json.load(open(TRAFFIC_RECORD))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None
    return (rec["fetch_size_kib_per_dispatch"] * rec["copy_read_factor"] +
            rec["write_size_kib_per_dispatch"] * rec["copy_write_factor"]) * 1024.0


def gups(updates: float, seconds: float) -> float:
    return updates / (seconds * 2.0 ** 30)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bp2048")
    ap.add_argument("--adjoint-views", type=int, default=256,
                    help="views of the adjoint timing (a rate, reported per update)")
    ap.add_argument("--no-16bit", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a buffer of this many MiB (a plain copy of known size, "
                         "whose HBM counters scale the kernel's)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(one GPU's share is the workload; see the design notes on sharding).",
              file=sys.stderr)
        sys.exit(2)

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
    launches = math.ceil(n_views / 32)
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
    chunk = 64
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
        return sum(ms) / len(ms)

    # ---- FP32 storage: the headline figure ----
    ms32 = timed_bp(q32, args.steps, args.warmup, "fp32")
    gups32 = gups(updates, ms32 / 1e3)
    log(f"fp32: {gups32:.1f} GUPS")
    result_extra = {}

    if not args.no_16bit:
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            q16 = q32.to(dt)
            ms16 = timed_bp(q16, max(1, args.steps // 2), 1, name)
            result_extra[f"{name}_store_gups"] = round(gups(updates, ms16 / 1e3), 2)
            result_extra[f"{name}_ms_per_step"] = round(ms16, 2)
            del q16
            torch.cuda.empty_cache()

    if not args.no_adjoint:
        nv_adj = min(args.adjoint_views, n_views)
        x = torch.empty_like(vol).normal_()
        qa = torch.empty((nv_adj, g.nv, g.nu), dtype=torch.float32, device=dev)
        fdk.forward_project(x, g, ang, nviews=nv_adj, out=qa, scale=scale)
        torch.cuda.synchronize()
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        fdk.forward_project(x, g, ang, nviews=nv_adj, out=qa, scale=scale)
        eb.record(stream)
        torch.cuda.synchronize()
        msa = ea.elapsed_time(eb)
        result_extra["adjoint_gups"] = round(gups(float(g.nx) * g.ny * g.nz * nv_adj, msa / 1e3), 2)
        result_extra["adjoint_views_timed"] = nv_adj
        log(f"adjoint: {result_extra['adjoint_gups']} GUPS over {nv_adj} views ({msa:.1f} ms)")
        del x, qa

    # ---- roofline of the dominant kernel (the back-projection launches) ----
    per_launch_s = ms32 / 1e3 / launches
    updates_per_launch = updates / launches
    achieved = gups(updates_per_launch, per_launch_s)
    valu_roof = N_CU * VALU_LANES_PER_CLK * CLOCK_HZ / VALU_OPS_PER_UPDATE / 2 ** 30
    lds_roof = N_CU * LDS_BYTES_PER_CLK * CLOCK_HZ / LDS_BYTES_PER_UPDATE / 2 ** 30
    peak = min(valu_roof, lds_roof)
    traffic = profiled_traffic(args.workload)
    roofline = {
        "bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 1), "unit": "GUPS",
        "frac": round(achieved / peak, 4),
        "traffic": None if traffic is None else round(traffic),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "kernel": "bp_tiled_mirror_kernel<float>", "launches_per_step": launches,
        "avg_launch_ms": round(per_launch_s * 1e3, 3),
        "valu_roof_gups": round(valu_roof, 1), "lds_roof_gups": round(lds_roof, 1),
        "hbm_algorithmic_bytes_per_launch": round(updates_per_launch * (
            8.0 / 32 + g.nu * g.nv * 4.0 / (g.nx * g.ny * g.nz))),
    }

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
        cpu = {"value": round(gups(done, el), 5), "unit": "GUPS", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{done} voxel-view updates ({nvox} random voxels of the "
                         f"{g.nx}x{g.ny}x{g.nz} volume x {nv_cpu} views of {g.nv}x{g.nu}, "
                         f"repeated for {el:.1f} s)"}
        log(f"cpu oracle: {cpu['value']} GUPS on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": round(gups32, 2), "unit": "GUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms32, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded 32-ellipsoid phantom, analytic line integrals, "
                "Shepp-Logan filtered on the GPU",
        "config": {"workload": f"{args.workload}: {g.nx}x{g.ny}x{g.nz} FP32 volume, "
                               f"{n_views} views of {g.nv}x{g.nu}, 32 views per launch",
                   "nx": g.nx, "ny": g.ny, "nz": g.nz, "n_views": n_views, "nu": g.nu,
                   "nv": g.nv, "views_per_launch": 32},
        **result_extra,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
