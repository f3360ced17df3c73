"""Volumes larger than one should keep resident: streamed through HBM in slabs along t.

Every output voxel of the method depends on samples at most `halo` voxels away along each
axis (floor(L/2) for the window plus floor(d/2) for the comparison of Eq. (5); 5 for the
surrogate's five 3^3 layers), so a slab of rows [s0, s1) is computed exactly from the rows
[s0 - halo, s1 + halo) clipped to the volume: reflection at a clipped face is the
volume's own.  The raw maps of every slab are kept in HBM (3 floats per voxel) and the
volume-wide FP64 statistics and Eq. (6) run once at the end.  Host-to-device copies of the
next slab run on a second stream while the current slab computes (double-buffered pinned
staging); max|V| for the zero-contrast rule is reduced slab by slab.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import sal, surrogate


def pinned(V: np.ndarray) -> torch.Tensor:
    """A page-locked host copy of the volume (allocated pinned, then filled)."""
    t = torch.empty(V.shape, dtype=torch.float32, pin_memory=True)
    t.numpy()[...] = V
    return t


def _slabs(n0: int, slab: int, halo: int, align: int = 1):
    """Output rows [s0, s1) and the rows [a, b) they depend on; a is a multiple of `align`
    (the window lattice of a strided context starts at row 0 of the volume)."""
    for s0 in range(0, n0, slab):
        s1 = min(n0, s0 + slab)
        yield s0, s1, max(0, s0 - halo) // align * align, min(n0, s1 + halo)


def raw_maps_streamed(V_host: torch.Tensor, compute, halo: int, slab: int = 64,
                      S_raw: Optional[torch.Tensor] = None, device="cuda",
                      keep: Optional[torch.Tensor] = None, ctx: Optional[sal.Saliency] = None,
                      align: int = 1):
    """Raw maps [3, n0, n1, n2] (device) of a pinned host volume; `compute(Vslab)` returns
    the raw maps [3, m, n1, n2] of a device slab [m, n1, n2].  With `keep` (device
    [n0, n1, n2]) the rows of every slab are also kept there as they pass.  max|V| is
    reduced slab by slab by the library (sal_absmax on `ctx`, or a plain FP32 context).
    Returns (S_raw, max|V|)."""
    n0, n1, n2 = V_host.shape
    dev = torch.device(device)
    if S_raw is None:
        S_raw = torch.empty((3, n0, n1, n2), dtype=torch.float32, device=dev)
    rows = min(n0, slab + 2 * halo + align - 1)
    bufs = [torch.empty((rows, n1, n2), dtype=torch.float32, device=dev) for _ in range(2)]
    comp = torch.cuda.current_stream(dev)
    copy = torch.cuda.Stream(dev)
    # The staging buffers come from the compute stream's pool and may reuse memory that work
    # still queued there reads (a map the caller has just dropped): the copy stream starts
    # after that work, and the buffers are marked as used by the copy stream.
    copy.wait_stream(comp)
    for b in bufs:
        b.record_stream(copy)
    done = [torch.cuda.Event(), torch.cuda.Event()]     # buffer free again
    ready = [torch.cuda.Event(), torch.cuda.Event()]    # buffer filled
    slabs = list(_slabs(n0, slab, halo, align))
    vmax = torch.zeros(1, dtype=torch.float32, device=dev)
    red = ctx if ctx is not None else sal.Saliency(L=8, device=dev.index or 0)

    def upload(i):
        _, _, a, b = slabs[i]
        k = i % 2
        with torch.cuda.stream(copy):
            if i >= 2:
                copy.wait_event(done[k])
            bufs[k][:b - a].copy_(V_host[a:b], non_blocking=True)
            ready[k].record(copy)

    upload(0)
    for i, (s0, s1, a, b) in enumerate(slabs):
        k = i % 2
        if i + 1 < len(slabs):
            upload(i + 1)
        comp.wait_event(ready[k])
        Vs = bufs[k][:b - a]
        out = compute(Vs)
        S_raw[:, s0:s1].copy_(out[:, s0 - a:s1 - a])
        if keep is not None:
            keep[s0:s1].copy_(Vs[s0 - a:s1 - a])
        sal.absmax(red, Vs[s0 - a:s1 - a], vmax, accumulate=i > 0)
        done[k].record(comp)
    return S_raw, float(vmax.item())


def plain_streamed(ctx: sal.Saliency, V_host: torch.Tensor, slab: int = 64):
    """The plain method on a host volume, slab by slab; returns (S, S_raw, stats).  With
    windows on the stride-s lattice each slab starts on a lattice row, and its halo also
    holds the next lattice point of the interpolation (s more rows)."""
    st = ctx.params.stride
    halo = ctx.L // 2 + ctx.params.d // 2 + (st if st > 1 else 0)

    def compute(Vs):
        o = torch.empty((3,) + tuple(Vs.shape), dtype=torch.float32, device=Vs.device)
        ctx.saliency(Vs, S_raw_out=o)
        return o

    S_raw, vmax = raw_maps_streamed(V_host, compute, halo, slab, ctx=ctx, align=st)
    stats = torch.zeros(8, dtype=torch.float64, device=S_raw.device)
    S = sal.normalize_combine(ctx, S_raw, None, stats_out=stats, vmax=vmax)
    return S, S_raw, stats


def slab_volumes(V_host: torch.Tensor, tile: int, halo: int, slab_rows: int = 4, device="cuda"):
    """For TileCheck.check_many without a resident volume: groups the tiles by runs of
    `slab_rows` tile rows along t and uploads, per group, the rows it covers plus `halo`
    (clipped to the volume), on the current stream."""
    n0, n1, n2 = V_host.shape
    nt12 = ((n1 + tile - 1) // tile) * ((n2 + tile - 1) // tile)

    def volumes(tis):
        rows = {}
        for ti in tis:
            rows.setdefault(ti // nt12 // slab_rows, []).append(ti)
        for g in sorted(rows):
            s0 = g * slab_rows * tile
            s1 = min(n0, s0 + slab_rows * tile)
            a, b = max(0, s0 - halo), min(n0, s1 + halo)
            Vs = V_host[a:b].to(device, non_blocking=True)
            yield Vs, (a, 0, 0), rows[g]
    return volumes


def surrogate_streamed(net: sal.Net, ctx_fallback: sal.Saliency, V_host: torch.Tensor,
                       slab: int = 64, tile: int = 32, frac: float = 0.02, bound: float = 0.02,
                       seed: int = 0, max_rounds: int = 8, per_round: int = 32, top_frac: float = 0.05,
                       keep_volume: bool = True):
    """Surrogate first, slab by slab (halo 5), then the seeded tile check, the check of the
    tiles with the highest predicted saliency and of the tiles holding each map's extremes,
    with the plain method (ctx_fallback, e.g. split-BF16) and exact replacement, in batched
    passes; then the FP64 normalisation and Eq. (6).  With keep_volume the slabs stay in HBM
    as they stream (one more float per voxel) and the checks read them there; otherwise
    the rows holding checked tiles are streamed again (halo floor(L/2) + r)."""
    dev = torch.device("cuda")
    keep = torch.empty(tuple(V_host.shape), dtype=torch.float32, device=dev) if keep_volume else None
    S_raw, vmax = raw_maps_streamed(V_host, net.infer, 5, slab, keep=keep, ctx=ctx_fallback)
    stats = torch.zeros(8, dtype=torch.float64, device=dev)
    S = sal.normalize_combine(ctx_fallback, S_raw, None, stats_out=stats, vmax=vmax)
    n_all = len(surrogate.tiles_of(tuple(V_host.shape), tile))
    sample = surrogate.seeded_tiles(n_all, frac, seed)
    halo = ctx_fallback.L // 2 + ctx_fallback.params.d // 2

    def crop(lo, hi):
        return V_host[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].contiguous().to(dev), lo

    if keep is not None:
        volumes = lambda tis: [(keep, (0, 0, 0), tis)]
    else:
        volumes = slab_volumes(V_host, tile, halo, device=dev)
    chk = surrogate.TileCheck(ctx_fallback, S_raw, stats, crop, tile, bound,
                              len(sample) + int(math.ceil(top_frac * n_all)) + 6 * per_round * max_rounds,
                              volumes=volumes)
    chk.check_many(sample)
    chk.check_top(top_frac)
    rounds = chk.verify_extremes(max_rounds, per_round)
    S = sal.normalize_combine(ctx_fallback, S_raw, None, S=S, stats_out=stats, vmax=vmax)
    return {"S": S, "S_raw": S_raw, "stats": stats, "tiles": chk.tiles, "tile_err": chk.errors(),
            "n_tiles": chk.n_tiles(), "extreme_rounds": rounds}
