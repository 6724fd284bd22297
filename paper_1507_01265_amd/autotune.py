"""Launch-plan tuner for batches of uneven grids.

Two decisions are made from measurements on the GPU:

* the launch shape (x-y region of a workgroup; its output tile is the region
  minus a 2-cell halo): every candidate shape is timed on the batch;
* the assignment of (grid, tile) blocks to the workgroups of the persistent
  kernel: blocks are placed by longest-processing-time-first (LPT) greedy
  scheduling onto the workgroup with the least accumulated cost.  The costs
  are per-block durations measured while all workgroups run together -- the
  paper's lesson that processing units sharing a chip must be benchmarked
  simultaneously, not one at a time (section 5.4) -- starting from a plan
  placed with the static cost (planes + pipeline priming).

The halo depth is fixed by the stencil (3 cells of psi^n per fused step).
"""
from __future__ import annotations

import dataclasses
import heapq
import time

import numpy as np
import torch

from . import _lib
from .batch import Batch

PRIMING = 4  # extra z-iterations of a march before its first output plane


def tiles_of(shape, tile):
    tx, ty, _ = _lib.mpdata_tile_info(tile)
    nz, ny, nx = shape
    return -(-nx // tx), -(-ny // ty)


def whole_tile_segments(shapes, tile):
    """One segment per (grid, tile) over all planes: rows (grid, tx, ty, 0, nz)."""
    segs = []
    for g, shp in enumerate(shapes):
        ntx, nty = tiles_of(shp, tile)
        for ty in range(nty):
            for tx in range(ntx):
                segs.append((g, tx, ty, 0, shp[0]))
    return np.array(segs, dtype=np.int32).reshape(-1, 5)


def lpt(costs, nwg):
    """Longest-processing-time-first: returns (owner of each item, loads)."""
    order = np.argsort(-np.asarray(costs, dtype=np.float64), kind="stable")
    heap = [(0.0, w) for w in range(nwg)]
    owner = np.empty(len(costs), dtype=np.int64)
    loads = np.zeros(nwg)
    for i in order:
        load, w = heapq.heappop(heap)
        owner[i] = w
        load += float(costs[i])
        loads[w] = load
        heapq.heappush(heap, (load, w))
    return owner, loads


def plan_from_owner(segs, owner, nwg):
    """Group segments by owning workgroup -> (seg, wg_begin)."""
    order = np.argsort(owner, kind="stable")
    seg = segs[order]
    counts = np.bincount(owner, minlength=nwg)
    wg_begin = np.zeros(nwg + 1, dtype=np.int32)
    wg_begin[1:] = np.cumsum(counts)
    return seg, wg_begin


@dataclasses.dataclass
class Tuned:
    tile: int
    plan: tuple            # (tile, seg, wg_begin) for Batch(plan=...)
    ms_per_step: float
    makespan_static: float
    makespan_measured: float
    log: list


def time_steps(batch, steps):
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(batch.stream)
    batch.step(steps)
    b.record(batch.stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def option_tiles():
    """Launch shapes built for the variable-sign option and the divergent-flow
    term: the 32x24 and 32x32 regions."""
    out = []
    for t in range(1, _lib.mpdata_tile_count() + 1):
        tx, ty, _ = _lib.mpdata_tile_info(t)
        if tx + 4 == 32 and ty + 4 in (24, 32):
            out.append(t)
    return out


def tune(grids, *, bc="periodic", nonos=True, eps=1e-15, tiles=None, steps=4, profiles=3,
         verbose=False, vsign=False, div=False):
    """Pick the launch shape and the block assignment for ``grids`` (list of
    5-tuples of device tensors).  The grids' psi is restored afterwards."""
    dtype = grids[0][0].dtype
    dt = _lib.MPDATA_FP32 if dtype == torch.float32 else _lib.MPDATA_FP64
    if tiles is None:
        tiles = (option_tiles() if (vsign or div)
                 else list(range(1, _lib.mpdata_tile_count() + 1)))
    opts = dict(bc=bc, nonos=nonos, eps=eps, vsign=vsign, div=div)
    shapes = [tuple(g[0].shape) for g in grids]
    saved = [g[0].clone() for g in grids]
    log = []
    best = None
    for tile in tiles:
        per, cus = _lib.mpdata_occupancy(dt, tile, _lib.MPDATA_BC_OPEN if bc == "open" else 0,
                                         int(bool(nonos)))
        nwg = per * cus
        segs = whole_tile_segments(shapes, tile)
        static = segs[:, 4] - segs[:, 3] + PRIMING
        owner, loads0 = lpt(static, nwg)
        plan0 = (tile, *plan_from_owner(segs, owner, nwg))
        b = Batch(grids, plan=plan0, **opts)
        b.step(2)
        ms0 = time_steps(b, steps)
        ticks = np.median(np.stack([b.profile_step() for _ in range(profiles)]), axis=0)
        b.close()
        # ticks come in the plan's segment order; map back to the tile list
        seg_sorted = plan0[1]
        key = {tuple(r): i for i, r in enumerate(segs.tolist())}
        measured = np.empty(len(segs))
        for r, t in zip(seg_sorted.tolist(), ticks):
            measured[key[tuple(r)]] = t
        owner1, loads1 = lpt(measured, nwg)
        plan1 = (tile, *plan_from_owner(segs, owner1, nwg))
        b = Batch(grids, plan=plan1, **opts)
        b.step(2)
        ms1 = time_steps(b, steps)
        b.close()
        entry = dict(tile=tile, nwg=nwg, nseg=len(segs), ms_static=ms0, ms_measured=ms1,
                     makespan_static_ticks=float(loads0.max()),
                     makespan_measured_ticks=float(loads1.max()),
                     mean_load_ticks=float(measured.sum() / nwg))
        log.append(entry)
        if verbose:
            print("tune", entry, flush=True)
        for ms, plan, mk in ((ms0, plan0, loads0.max()), (ms1, plan1, loads1.max())):
            if best is None or ms < best.ms_per_step:
                best = Tuned(tile, plan, ms, float(loads0.max()), float(loads1.max()), log)
    for g, s in zip(grids, saved):
        g[0].copy_(s)
    torch.cuda.synchronize()
    best.log = log
    return best
