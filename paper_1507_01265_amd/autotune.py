"""Launch-plan tuner for batches of uneven grids.

Two decisions are made from measurements on the GPU:

* the launch shape (x-y region of a workgroup; its output tile is the region
  minus a 2-cell halo): every candidate shape is timed on the batch, and
  for FP32 periodic batches a mixed plan gives each grid the one of the two
  768-thread regions (32x24, 24x32) whose tiles cost it less in the measured
  runs -- per-size-class shapes in one persistent launch;
* the assignment of (grid, tile) blocks to the workgroups of the persistent
  kernel: blocks are placed by longest-processing-time-first (LPT) greedy
  scheduling onto the workgroup with the least accumulated cost.  The costs
  are per-block durations measured while all workgroups run together -- the
  paper's lesson that processing units sharing a chip must be benchmarked
  simultaneously, not one at a time (section 5.4) -- starting from a plan
  placed with the static cost (planes + pipeline priming).  A third
  placement keeps every grid on one XCD (one L2).  All three are timed and
  the fastest kept: which one wins depends on the shape (measured).

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
XCDS = 8     # workgroup w of a launch runs on XCD w mod 8 (each XCD has its own L2)


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


def xcd_affine(segs, costs, nwg, ngrids):
    """Owner of each segment with every grid kept on one XCD: the grids are
    dealt to the XCDs by LPT of their total cost, then each XCD's segments
    by LPT over its workgroups (w mod XCDS == xcd), so a grid's tiles share
    one L2."""
    g = segs[:, 0]
    costs = np.asarray(costs, dtype=np.float64)
    grid_xcd, _ = lpt(np.bincount(g, weights=costs, minlength=ngrids), XCDS)
    owner = np.empty(len(segs), dtype=np.int64)
    for x in range(XCDS):
        idx = np.nonzero(grid_xcd[g] == x)[0]
        wgs = np.arange(x, nwg, XCDS)
        if len(idx):
            o, _ = lpt(costs[idx], len(wgs))
            owner[idx] = wgs[o]
    return owner


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
    tile: object           # a tile id, or "mixed" (per-grid shapes, plan[0] = 5)
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


MIXED_TILES = (5, 7)  # the 768-thread regions one mixed launch combines


def mixed_segments(shapes, choice):
    """Whole-tile segments with a sixth column, the shape of each grid
    (choice[g] in MIXED_TILES)."""
    rows = []
    for g, (shp, tile) in enumerate(zip(shapes, choice)):
        ntx, nty = tiles_of(shp, tile)
        for ty in range(nty):
            for tx in range(ntx):
                rows.append((g, tx, ty, 0, shp[0], tile))
    return np.array(rows, dtype=np.int32).reshape(-1, 6)


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
                 else [t for t in range(1, _lib.mpdata_tile_count() + 1)
                       if _lib.mpdata_tile_built(dt, t)])
    opts = dict(bc=bc, nonos=nonos, eps=eps, vsign=vsign, div=div)
    shapes = [tuple(g[0].shape) for g in grids]
    saved = [g[0].clone() for g in grids]
    log = []
    best = None
    per_tile = {}  # tile -> (segments, measured ticks per segment, nwg)
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
        per_tile[tile] = (segs, measured, nwg)
        owner1, loads1 = lpt(measured, nwg)
        plan1 = (tile, *plan_from_owner(segs, owner1, nwg))
        b = Batch(grids, plan=plan1, **opts)
        b.step(2)
        ms1 = time_steps(b, steps)
        b.close()
        # the static placement with every grid on one XCD (its own L2)
        ms2 = float("inf")
        if nwg % XCDS == 0:
            plan2 = (tile, *plan_from_owner(segs, xcd_affine(segs, static, nwg, len(grids)), nwg))
            b = Batch(grids, plan=plan2, **opts)
            b.step(2)
            ms2 = time_steps(b, steps)
            b.close()
        entry = dict(tile=tile, nwg=nwg, nseg=len(segs), ms_static=ms0, ms_measured=ms1,
                     ms_xcd=ms2,
                     makespan_static_ticks=float(loads0.max()),
                     makespan_measured_ticks=float(loads1.max()),
                     mean_load_ticks=float(measured.sum() / nwg))
        log.append(entry)
        if verbose:
            print("tune", entry, flush=True)
        cands = [(ms0, plan0), (ms1, plan1)] + ([(ms2, plan2)] if nwg % XCDS == 0 else [])
        for ms, plan in cands:
            if best is None or ms < best.ms_per_step:
                best = Tuned(tile, plan, ms, float(loads0.max()), float(loads1.max()), log)
    if (dtype == torch.float32 and bc == "periodic" and not vsign and not div
            and all(t in per_tile for t in MIXED_TILES)):
        # per-grid shapes: each grid takes the region whose tiles cost it
        # less, by the per-segment times measured with all workgroups busy
        cost = {}
        for t in MIXED_TILES:
            segs_t, meas_t, _ = per_tile[t]
            cost[t] = np.bincount(segs_t[:, 0], weights=meas_t, minlength=len(grids))
        choice = [min(MIXED_TILES, key=lambda t: cost[t][g]) for g in range(len(grids))]
        segs_m = mixed_segments(shapes, choice)
        key = {t: {tuple(r): m for r, m in zip(per_tile[t][0].tolist(), per_tile[t][1])}
               for t in MIXED_TILES}
        meas_m = np.array([key[r[5]][tuple(r[:5])] for r in segs_m.tolist()])
        nwg = per_tile[MIXED_TILES[0]][2]
        owner_m, loads_m = lpt(meas_m, nwg)
        plan_m = (MIXED_TILES[0], *plan_from_owner(segs_m, owner_m, nwg))
        b = Batch(grids, plan=plan_m, **opts)
        b.step(2)
        ms_m = time_steps(b, steps)
        b.close()
        entry = dict(tile="mixed", shapes={str(t): choice.count(t) for t in MIXED_TILES},
                     nwg=nwg, nseg=len(segs_m), ms_measured=ms_m,
                     makespan_measured_ticks=float(loads_m.max()))
        log.append(entry)
        if verbose:
            print("tune", entry, flush=True)
        if ms_m < best.ms_per_step:
            best = Tuned("mixed", plan_m, ms_m, float("nan"), float(loads_m.max()), log)
    for g, s in zip(grids, saved):
        g[0].copy_(s)
    torch.cuda.synchronize()
    best.log = log
    return best
