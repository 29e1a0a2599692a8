"""Streaming reconstruction of one volume slab: projections arrive in chunks
of views, each chunk is filtered on a producer stream and back-projected on
the caller's stream while the next chunk is being produced.

This is the single-GPU share of the paper's pipelined reconstruction
(Sec. 4: filtering overlapped with back-projection, volume split into
mirrored sub-volume pairs as in Fig. 5): only the detector rows the slab
reads (``slab_rows``) are produced and filtered, into two alternating
full-detector chunk buffers whose other rows stay zero. All arithmetic runs
in the HIP library; this module only orders work on streams.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Sequence

import numpy as np
import torch

from . import backproject, filter as filter_rows_op, slab_rows


@dataclass
class SlabTiming:
    """Event-timed pieces of a streamed reconstruction (milliseconds)."""
    bp_ms: list[float] = field(default_factory=list)  # each back-projection launch
    wall_ms: float = 0.0                                # first produce to last back-projection


# produce(view0, nviews, bands, e_bands): for each band (v0, nrows) fill
# e_bands[b][:nviews] (float32 (chunk, nrows, Nu)) with the raw line
# integrals of rows [v0, v0 + nrows) of views [view0, view0 + nviews). It is
# called with the producer stream current and must enqueue its work there.
Producer = Callable[[int, int, Sequence[tuple[int, int]], Sequence[torch.Tensor]], None]


def reconstruct_slab(geom, angles, produce: Producer, *, z0: int = 0,
                     nz_local: int | None = None, slab: str = "contiguous", chunk: int = 16,
                     dtype: torch.dtype = torch.float16, kind: str = "shepp-logan",
                     scale: float = 1.0, chunks: Sequence[int] | None = None,
                     out: torch.Tensor | None = None, device="cuda",
                     timing: SlabTiming | None = None) -> torch.Tensor:
    """FDK back-projection of a slab from views produced chunk by chunk.

    chunks: first view of each chunk (default: every `chunk` views over the
    whole scan); a chunk holds min(chunk, Np - view0) views. Returns the
    slab (nz_local, Ny, Nx) float32, accumulated over all chunks, in `out`
    if given. If `timing` is given, each back-projection launch and the
    whole pipeline are timed with events (the caller synchronises)."""
    ang = np.asarray(angles, np.float64)
    n_all = ang.size
    nz_local = geom.nz - z0 if nz_local is None else int(nz_local)
    if chunks is None:
        chunks = list(range(0, n_all, chunk))
    bands = slab_rows(geom, ang, z0=z0, nz_local=nz_local, slab=slab)
    main = torch.cuda.current_stream(device)
    if out is None:
        out = torch.empty((nz_local, geom.ny, geom.nx), dtype=torch.float32, device=device)
    qbuf = [torch.zeros((chunk, geom.nv, geom.nu), dtype=dtype, device=device) for _ in range(2)]
    ebuf = [[torch.empty((chunk, n, geom.nu), dtype=torch.float32, device=device)
             for _, n in bands] for _ in range(2)]
    prod = torch.cuda.Stream(device=device)
    prod.wait_stream(main)  # buffers were allocated and cleared on the caller's stream
    filled = [torch.cuda.Event() for _ in range(2)]
    consumed = [torch.cuda.Event() for _ in range(2)]
    used = [False, False]
    t0 = torch.cuda.Event(enable_timing=True) if timing is not None else None
    if t0 is not None:
        t0.record(main)
    pairs = []
    if not chunks or not bands:
        # nothing reaches the slab: it is zero
        backproject(qbuf[0][:0], geom, ang, out=out, z0=z0, nz_local=nz_local, slab=slab)
    for c, view0 in enumerate(chunks):
        n = min(chunk, n_all - view0)
        b = c % 2
        with torch.cuda.stream(prod):
            if used[b]:
                prod.wait_event(consumed[b])
            produce(view0, n, bands, [e[:n] for e in ebuf[b]])
            for (v0, nr), e in zip(bands, ebuf[b]):
                filter_rows_op(e[:n], geom, ang, view0=view0, kind=kind,
                               out=qbuf[b][:n, v0:v0 + nr], rows=(v0, nr))
            filled[b].record(prod)
        main.wait_event(filled[b])
        if timing is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(main)
        backproject(qbuf[b][:n], geom, ang, view0=view0, out=out, z0=z0, nz_local=nz_local,
                    slab=slab, scale=scale, accumulate=c > 0)
        if timing is not None:
            e1.record(main)
            pairs.append((e0, e1))
        consumed[b].record(main)
        used[b] = True
    if timing is not None:
        t1 = torch.cuda.Event(enable_timing=True)
        t1.record(main)
        t1.synchronize()
        timing.bp_ms = [a.elapsed_time(z) for a, z in pairs]
        timing.wall_ms = t0.elapsed_time(t1)
    return out
