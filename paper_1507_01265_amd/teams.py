"""XCD teams: the paper's load-imbalancing method on one MI355X.

The paper (sections 3-5) splits one MPDATA domain between teams of cores,
builds each team's speed function -- the speed on a sub-domain of m frames,
measured while all teams run together -- checks Theorem 1's condition and,
where it fails, lets Algorithm 1 pick an uneven split.  Here the teams are
the 8 XCDs of the GPU (workgroup w of the persistent step kernel runs on XCD
w mod 8) and a team's sub-domain is a slab of m z-planes of one grid: all
x-y tiles over planes [z0, z0 + m), dealt whole to the team's workgroups.
Everything runs through the batch C ABI with caller-built plans; the
per-segment durations come from ``mpdata_batch_profile_step``; Theorem 1's
check and Algorithm 1 are the library's ``mpdata_fpm_*`` entry points.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib
from .autotune import tiles_of
from .batch import Batch

XCDS = 8
TICK_HZ = 100e6  # wall_clock64 rate of the segment durations


def slab_plan(shape, tile, nwg, slabs):
    """Plan for one grid of shape (nz, ny, nx): team i (workgroups w with
    w % XCDS == i) runs planes slabs[i] = (z0, z1) of every tile, whole tiles
    dealt round-robin over the team's workgroups.  Returns (tile, seg,
    wg_begin) for ``Batch(plan=...)``."""
    if len(slabs) != XCDS or nwg % XCDS:
        raise ValueError("one slab per XCD and a workgroup count divisible by the XCD count")
    ntx, nty = tiles_of(shape, tile)
    tiles = [(tx, ty) for ty in range(nty) for tx in range(ntx)]
    per_wg = [[] for _ in range(nwg)]
    for team, (z0, z1) in enumerate(slabs):
        if z1 <= z0:
            continue
        wgs = list(range(team, nwg, XCDS))
        for k, (tx, ty) in enumerate(tiles):
            per_wg[wgs[k % len(wgs)]].append((0, tx, ty, z0, z1))
    seg = np.array([s for w in per_wg for s in w], dtype=np.int32).reshape(-1, 5)
    wg_begin = np.zeros(nwg + 1, dtype=np.int32)
    wg_begin[1:] = np.cumsum([len(w) for w in per_wg])
    return tile, seg, wg_begin


def team_seconds(ticks, wg_begin):
    """Per-team time of one step: a workgroup runs its segments back to back,
    a team is done when its slowest workgroup is."""
    nwg = len(wg_begin) - 1
    per_wg = np.array([ticks[wg_begin[w]:wg_begin[w + 1]].sum() for w in range(nwg)])
    return np.array([per_wg[t::XCDS].max() for t in range(XCDS)]) / TICK_HZ


def even_slabs(nz):
    share = nz // XCDS
    return [(i * share, (i + 1) * share) for i in range(XCDS)]


def split_slabs(x_hi, x_lo):
    """Even-numbered teams x_hi planes, odd-numbered x_lo, in team order."""
    slabs, z = [], 0
    for t in range(XCDS):
        m = x_hi if t % 2 == 0 else x_lo
        slabs.append((z, z + m))
        z += m
    return slabs


def _grid(fields, dtype):
    np_dtype = np.float64 if dtype == torch.float64 else np.float32
    return tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np_dtype)).cuda()
                 for a in (fields.psi, fields.u1, fields.u2, fields.u3, fields.h))


def _occupancy_nwg(dtype, tile, bc):
    dt = _lib.MPDATA_FP64 if dtype == torch.float64 else _lib.MPDATA_FP32
    per, cus = _lib.mpdata_occupancy(dt, tile, bc, 1)
    return per * cus


@dataclasses.dataclass
class Run:
    slabs: list
    seconds_per_step: float      # HIP events over the timed steps
    team_seconds: np.ndarray     # per-team time of one step (median of profiled steps)


def run_plan(fields, dtype, tile, slabs, steps=20, profiles=5):
    """Time one grid under a slab plan: HIP events over ``steps`` steps and the
    per-team times of ``profiles`` profiled steps (median)."""
    grid = _grid(fields, dtype)
    nwg = _occupancy_nwg(dtype, tile, fields.bc)
    plan = slab_plan(fields.psi.shape, tile, nwg, slabs)
    b = Batch([grid], bc="open" if fields.bc else "periodic", plan=plan)
    try:
        b.step(2)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(b.stream)
        b.step(steps)
        a1.record(b.stream)
        torch.cuda.synchronize()
        sec = a0.elapsed_time(a1) / 1e3 / steps
        ticks = [b.profile_step() for _ in range(profiles)]
        teams = np.median(np.stack([team_seconds(np.asarray(t), plan[2]) for t in ticks]), axis=0)
    finally:
        b.close()
    return Run(slabs, sec, teams)


def speed_function(make_fields, ms, dtype, tile, profiles=5):
    """s(m) for each m in ms: a grid of XCDS*m planes split evenly, every team
    on m planes at once; the speed of team i is its cells over its time.
    Returns {m: (mean speed over teams, per-team speeds)} in cells/s."""
    out = {}
    for m in ms:
        f = make_fields(XCDS * m)
        nz, ny, nx = f.psi.shape
        r = run_plan(f, dtype, tile, even_slabs(nz), steps=4, profiles=profiles)
        speeds = nx * ny * m / r.team_seconds
        out[m] = (float(speeds.mean()), speeds.tolist())
    return out


def experiment(make_fields, nz, dtype, tile, deltas=None, steps=20):
    """The paper's procedure on the XCD teams for a grid of nz planes: speed
    functions, Theorem 1's check, Algorithm 1, and the measured step time of
    the even split, the chosen split and the splits dm in ``deltas``."""
    share = nz // XCDS
    if nz % XCDS or share < 2:
        raise ValueError("nz must be a multiple of 8 with at least 2 planes per team")
    ms = list(range(1, 2 * share))
    sf = speed_function(make_fields, ms, dtype, tile)
    table = [1.0] + [sf[m][0] for m in ms]
    violations, first = _lib.mpdata_fpm_check(table, 1)
    x_lo, x_hi, t_pred = _lib.mpdata_fpm_partition(table, nz, XCDS, 1)
    f = make_fields(nz)
    nx, ny = f.psi.shape[2], f.psi.shape[1]
    frame = nx * ny
    if deltas is None:
        deltas = sorted({0, x_hi - share, 1, 2, share // 2})
    rows = []
    for dm in deltas:
        if dm >= share:
            continue
        hi, lo = share + dm, share - dm
        r = run_plan(f, dtype, tile, split_slabs(hi, lo), steps=steps)
        predicted = max(hi * frame / sf[hi][0], lo * frame / sf[lo][0])
        rows.append({"dm": dm, "planes_even_teams": hi, "planes_odd_teams": lo,
                     "predicted_ms": predicted * 1e3, "measured_ms": r.seconds_per_step * 1e3,
                     "team_ms": (r.team_seconds * 1e3).tolist()})
    default_ms = None
    g = _grid(f, dtype)
    b = Batch([g], bc="open" if f.bc else "periodic", tile=tile)
    try:
        b.step(2)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(b.stream)
        b.step(steps)
        a1.record(b.stream)
        torch.cuda.synchronize()
        default_ms = a0.elapsed_time(a1) / steps
    finally:
        b.close()
    return {"speed_function": {m: sf[m][0] for m in ms},
            "speed_function_per_team": {m: sf[m][1] for m in ms},
            "theorem1_violations": violations, "theorem1_first_violation": first,
            "algorithm1": {"x_lo": x_lo, "x_hi": x_hi, "dm": x_hi - share,
                           "predicted_ms": t_pred * frame * 1e3},
            "splits": rows, "library_plan_ms": default_ms, "cells": frame * nz}
