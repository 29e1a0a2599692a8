"""Streaming reconstruction of one volume slab: projections arrive in chunks
of views, each chunk is filtered on a producer stream and back-projected on
the caller's stream while the next chunk is being produced.

This is the single-GPU share of the paper's pipelined reconstruction
(Sec. 4: filtering overlapped with back-projection, volume split into
mirrored sub-volume pairs as in Fig. 5): only the detector rows the slab
reads (``slab_rows``) are produced and filtered, into two alternating
full-detector buffers whose other rows stay zero. Contiguous chunks are
gathered into one back-projection launch of up to ``batch`` views (the
volume is read and written once per launch). All arithmetic runs in the HIP
library; this module only orders work on streams.
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


# produce(view0, nviews, bands, e_bands) supplies the raw line integrals of
# rows [v0, v0 + nrows) of views [view0, view0 + nviews) for each band
# (v0, nrows) in `bands`: either it fills e_bands[b] (float32
# (nviews, nrows, Nu) buffers) and returns None, or it returns one float32
# (nviews, nrows, Nu) tensor per band (rows contiguous, any view stride),
# e.g. views of projections already in device memory. It is called with the
# producer stream current and must enqueue its work there.
Producer = Callable[[int, int, Sequence[tuple[int, int]], Sequence[torch.Tensor]],
                    "Sequence[torch.Tensor] | None"]


def launch_groups(chunks: Sequence[int], chunk: int, batch: int, n_all: int):
    """Group chunk starts into back-projection launches: consecutive chunks
    that continue each other's views, up to `batch` views per launch."""
    groups: list[list[tuple[int, int]]] = []
    for v0 in chunks:
        n = min(chunk, n_all - v0)
        if n <= 0:
            raise ValueError(f"chunk start {v0} is outside the scan's {n_all} views")
        if groups:
            last = groups[-1]
            end = last[-1][0] + last[-1][1]
            if end == v0 and sum(m for _, m in last) + n <= batch:
                last.append((v0, n))
                continue
        groups.append([(v0, n)])
    return groups


def reconstruct_slab(geom, angles, produce: Producer, *, z0: int = 0,
                     nz_local: int | None = None, slab: str = "contiguous", chunk: int = 16,
                     batch: int = 96, dtype: torch.dtype = torch.float16,
                     kind: str = "shepp-logan", scale: float = 1.0,
                     chunks: Sequence[int] | None = None, out: torch.Tensor | None = None,
                     device="cuda", timing: SlabTiming | None = None) -> torch.Tensor:
    """FDK back-projection of a slab from views produced chunk by chunk.

    chunk: views produced and filtered at a time. batch: most views per
    back-projection launch (contiguous chunks are gathered). chunks: first
    view of each chunk (default: every `chunk` views over the whole scan);
    a chunk holds min(chunk, Np - view0) views. Returns the slab
    (nz_local, Ny, Nx) float32, accumulated over all chunks, in `out` if
    given. If `timing` is given, each back-projection launch and the whole
    pipeline are timed with events."""
    ang = np.asarray(angles, np.float64)
    n_all = ang.size
    nz_local = geom.nz - z0 if nz_local is None else int(nz_local)
    batch = max(int(batch), int(chunk))
    if chunks is None:
        chunks = list(range(0, n_all, chunk))
    groups = launch_groups(chunks, chunk, batch, n_all)
    bands = slab_rows(geom, ang, z0=z0, nz_local=nz_local, slab=slab)
    main = torch.cuda.current_stream(device)
    if out is None:
        out = torch.empty((nz_local, geom.ny, geom.nx), dtype=torch.float32, device=device)
    qbuf = [torch.zeros((batch, geom.nv, geom.nu), dtype=dtype, device=device) for _ in range(2)]
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
    if not groups or not bands:
        # nothing reaches the slab: it is zero
        backproject(qbuf[0][:0], geom, ang, out=out, z0=z0, nz_local=nz_local, slab=slab)
        groups = []
    for gi, grp in enumerate(groups):
        b = gi % 2
        with torch.cuda.stream(prod):
            if used[b]:
                prod.wait_event(consumed[b])
            at = 0
            for view0, n in grp:
                es = produce(view0, n, bands, [e[:n] for e in ebuf[b]])
                if es is None:
                    es = [e[:n] for e in ebuf[b]]
                for (v0, nr), e in zip(bands, es):
                    filter_rows_op(e, geom, ang, view0=view0, kind=kind,
                                   out=qbuf[b][at:at + n, v0:v0 + nr], rows=(v0, nr))
                at += n
            filled[b].record(prod)
        main.wait_event(filled[b])
        if timing is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(main)
        backproject(qbuf[b][:at], geom, ang, view0=grp[0][0], out=out, z0=z0,
                    nz_local=nz_local, slab=slab, scale=scale, accumulate=gi > 0)
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
