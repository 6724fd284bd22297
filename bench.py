#!/usr/bin/env python3
"""Benchmark of the MPDATA time step on one MI355X.

One "step" is one MPDATA time step (donor-cell pass, pseudo-velocities,
limiter, corrective pass -- one launch of the fused kernel; with iord 3 a
second corrective pass in a second launch) over the whole grid.  The default workload is the 512x256x64 periodic solid-body-rotation
grid in FP64 (cone + slotted cube on a zero background, h in [0.8, 1.2]);
inputs are synthetic, seeded and resident in HBM before the timed region.

Prints ONE JSON line: cell-updates/s over exactly --steps timed steps after
--warmup untimed ones; the rooflines of the fused kernel at the launch time
measured with HIP events on the solver's stream -- HBM (algorithmic bytes per
launch against 8 TB/s) and VALU issue (busy SIMD-cycles per launch from the
committed counters of the same kernel source, against 1024 SIMDs x 2.4 GHz),
`roofline.bound` naming the one closer to saturation; the errors of a fresh
run of E steps against the FP64 oracle's E steps on the same inputs
(rel-Linf, rel-L2, mass drift); and that oracle run, timed on the host's
cores, as the CPU baseline.  The default workload adds an `fp32` object: the
same grid in FP32 + FP64 limiter, timed and checked the same way.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    # name: (generator, dtype, description)
    "rotation-fp64": ("rotation", "f64", "rotation 512x256x64 periodic FP64, limiter on, iord 2"),
    "rotation-fp32": ("rotation", "f32",
                      "rotation 512x256x64 periodic FP32 + FP64 limiter, limiter on, iord 2"),
    "streamfunction-fp32": ("streamfunction", "f32",
                            "streamfunction 1024x512x64 open FP32 + FP64 limiter, limiter on, iord 2"),
    "streamfunction-fp64": ("streamfunction", "f64",
                            "streamfunction 1024x512x64 open FP64, limiter on, iord 2"),
    "rotation-fp64-iord3": ("rotation", "f64",
                            "rotation 512x256x64 periodic FP64, limiter on, iord 3 (two corrective "
                            "passes: the fused step, then a second pass launch)"),
    "rotation-fp32-iord3": ("rotation", "f32",
                            "rotation 512x256x64 periodic FP32 + FP64 limiter, limiter on, iord 3"),
    "divergent-fp64": ("divergent", "f64",
                       "rotation 512x256x64 periodic FP64 with a compressible cosine part on every "
                       "axis (divergent flow), divergent-flow term on, limiter on, iord 2"),
    "rotation-tv-fp64": ("rotation", "f64",
                         "rotation 512x256x64 periodic FP64 whose angular rate changes every step "
                         "(8 cyclic time levels, rate x (1 + 0.1 sin(2 pi s/8))), the time-"
                         "variation term on, limiter on, iord 2"),
    "batched-fp32": ("batched", "f32",
                     "96 uneven periodic grids (nx, ny log-uniform in [32, 384], nz in [16, 64]), "
                     "FP32 + FP64 limiter, constant Courant per grid, one persistent launch per "
                     "step"),
    "teams-fp64": ("teams", "f64",
                   "rotation 512x256x64 periodic FP64 split into z-slabs over the 8 XCDs "
                   "(the paper's teams): speed functions measured with all teams running, "
                   "Theorem 1 check, Algorithm 1 split vs the even split"),
    "served": ("served", "mixed",
               "Poisson arrivals 200/s for 60 s, dims log-uniform [32,256]^2 x [16,64], steps "
               "uniform [10,200], 70% FP32 / 30% FP64, solid-body rotation, 200 GB HBM budget, "
               "continuous batching"),
}


def algorithmic_bytes(shape, word, tvel=False):
    """The five input arrays read once and psi written once per step:
    psi, h and psi_out are nx*ny*nz words; u1, u2, u3 carry one extra face
    along their own axis.  With Courant numbers that change in time the
    step also reads the three face arrays of its end level."""
    nz, ny, nx = shape
    n = nx * ny * nz
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    return word * (3 * n + (2 if tvel else 1) * faces)


# scheme options of a workload (iord 2, no divergent-flow term unless named here)
OPTIONS = {"rotation-fp64-iord3": {"iord": 3}, "rotation-fp32-iord3": {"iord": 3},
           "divergent-fp64": {"div": True}, "rotation-tv-fp64": {"tvel": True}}

# the cyclic time levels of rotation-tv-fp64: level s is the base rotation
# scaled by (1 + TV_AMP sin(2 pi s / TV_LEVELS)) (a product per face, the
# same bits on the host and the device; face n stays equal to face 0)
TV_LEVELS, TV_AMP = 8, 0.1


def tv_scale(s):
    import math
    return 1.0 + TV_AMP * math.sin(2 * math.pi * (s % TV_LEVELS) / TV_LEVELS)


def chain_bytes(shape, word, iord, nonos=True):
    """Bytes a step of iord > 2 moves by design: the fused step also writes
    its limited velocity (3 face arrays) and, with the limiter, psi1; each
    further pass reads its iterate, velocity, h and two bound arrays (psi1
    and psi^n after the fused step, the running bounds after that), and
    writes the next iterate, velocity and running bounds (the last pass
    writes psi only)."""
    nz, ny, nx = shape
    n = nx * ny * nz
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    b = 2 if nonos else 0
    head = 3 * n + faces + faces + (b // 2) * n
    mid = (2 + b) * n + faces + (1 + b) * n + faces
    last = (2 + b) * n + faces + n
    return word * (head + (iord - 3) * mid + last)


PROFILES = {"rotation-fp64": "step_kernel_rotation_512x256x64_fp64.md",
            "rotation-fp32": "step_kernel_rotation_512x256x64_fp32.md",
            "streamfunction-fp32": "step_kernel_streamfunction_1024x512x64_fp32.md",
            "streamfunction-fp64": "step_kernel_streamfunction_1024x512x64_fp64.md"}

# VALU issue peak: 256 CUs x 4 SIMDs, one issue cycle per SIMD per clock
SIMDS = 256 * 4
CLOCK_GHZ = 2.4


def step_compile_flags():
    """The compiler flags of the step kernel's source, as the build uses them."""
    from paper_1507_01265_amd import build
    extra = dict(build.SOURCES)["mpdata_step.hip"]
    return " ".join([*build.FLAGS, *extra])


def kernel_source_sha():
    """sha256 of what the step kernel is compiled from: the march and the
    kernel file, concatenated, followed by its compiler flags."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1507_01265_amd", "csrc")
    return hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                   for f in ("mpdata_march.h", "mpdata_step.hip"))
                          + step_compile_flags().encode()).hexdigest()


def profile_figures(workload):
    """Per-launch figures of the step kernel from the committed rocprofv3
    summary of this workload (lines "key: value"), or {} when there is none
    or the kernel source changed since the counters were taken:
    traffic_bytes_per_launch (FETCH_SIZE and WRITE_SIZE runs, each scaled by
    the same counter on a 512 MiB copy), valu_insts_per_launch
    (SQ_INSTS_VALU, wave instructions) and valu_quad_cycles_per_launch
    (SQ_ACTIVE_INST_VALU, quad-cycles a SIMD's VALU is busy, summed)."""
    name = PROFILES.get(workload)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return {}
    out = {}
    for k in ("traffic_bytes_per_launch", "valu_insts_per_launch", "valu_quad_cycles_per_launch"):
        if k in fields:
            out[k] = float(fields[k])
    return out


def measured_traffic(workload):
    """HBM bytes per launch from the committed profile, or None."""
    return profile_figures(workload).get("traffic_bytes_per_launch")


def roofline(workload, shape, word, ms_per_step, tvel=False):
    """Roofline objects of the step kernel at the measured launch time.

    HBM: algorithmic bytes per launch (5 reads + 1 write per cell) over the
    launch time against the 8 TB/s peak.  VALU: the SIMDs' VALU busy cycles
    per launch (SQ_ACTIVE_INST_VALU x 4, from the committed counters of the
    same kernel source) over the launch time against 1024 SIMDs x 2.4 GHz;
    lane instructions per output cell-step from SQ_INSTS_VALU x 64.
    `bound` names the roof closer to saturation; both are reported."""
    abytes = algorithmic_bytes(shape, word, tvel)
    t = ms_per_step / 1e3
    achieved = abytes / t / 1e9
    prof = profile_figures(workload)
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": prof.get("traffic_bytes_per_launch"),
           "algorithmic_bytes_per_launch": abytes}
    if "valu_quad_cycles_per_launch" not in prof:
        return hbm, None
    nz, ny, nx = shape
    cyc = 4.0 * prof["valu_quad_cycles_per_launch"]
    valu = {"achieved": cyc / t / 1e12, "peak": SIMDS * CLOCK_GHZ / 1e3,
            "unit": "T VALU-busy SIMD-cycles/s", "frac": cyc / t / (SIMDS * CLOCK_GHZ * 1e9),
            "lane_insts_per_cell_step": prof.get("valu_insts_per_launch", 0.0) * 64 / (nx * ny * nz)}
    if valu["frac"] > hbm["frac"]:
        main = {"bound": "alu", "achieved": valu["achieved"], "peak": valu["peak"],
                "unit": valu["unit"], "frac": valu["frac"], "traffic": hbm["traffic"],
                "hbm": {k: hbm[k] for k in ("achieved", "peak", "unit", "frac",
                                            "algorithmic_bytes_per_launch")}}
        return main, valu
    return hbm, valu


def make_fields(kind):
    from paper_1507_01265_amd import inputs
    if kind == "divergent":
        return inputs.divergent_rotation()
    return inputs.rotation() if kind == "rotation" else inputs.streamfunction()


def tv_levels_device(s):
    """The TV_LEVELS cyclic time levels of a solver's Courant numbers, built
    on the device from the bound (level 0) arrays."""
    base = (s.u1, s.u2, s.u3)
    return [tuple(a * tv_scale(k) for a in base) for k in range(TV_LEVELS)]


class _TvStepper:
    """s.step(n) for a solver whose Courant numbers change every step: the
    next n cyclic levels through mpdata_step_tv."""

    def __init__(self, s):
        self.s, self.levels, self.k = s, tv_levels_device(s), 0

    def __call__(self, n):
        if n:
            self.s.step_tv([self.levels[(self.k + i + 1) % TV_LEVELS] for i in range(n)])
            self.k = (self.k + n) % TV_LEVELS


def time_gpu(fields, dtype_tag, steps, warmup, tile=0, iord=2, div=False, ci_target=0.0,
             max_reps=50, tvel=False, before_warmup=None):
    import numpy as np
    import torch
    from paper_1507_01265_amd.solver import Solver

    tdt = torch.float64 if dtype_tag == "f64" else torch.float32
    f = fields if dtype_tag == "f64" else fields.astype(np.float32)
    s = Solver.from_numpy(f, dtype=tdt, device="cuda", tile=tile, iord=iord, div=div, tvel=tvel)
    stream = s.stream
    step = _TvStepper(s) if tvel else s.step
    m0 = s.mass()
    if before_warmup is not None:
        # other GPU work, run between this solver's set-up (host work, the
        # GPU idle) and its warm-up, so that the timed steps do not start
        # while the clocks still ramp up from idle
        before_warmup()
    if warmup:
        step(warmup)
    torch.cuda.synchronize()
    # the timed region is exactly `steps` steps; events between chunks of 8
    # (one replayed graph each) give per-chunk times for the spread
    chunks = [8] * (steps // 8) + ([steps % 8] if steps % 8 else [])
    events = [torch.cuda.Event(enable_timing=True) for _ in range(len(chunks) + 1)]
    events[0].record(stream)
    for c, ev in zip(chunks, events[1:]):
        step(c)
        ev.record(stream)
    torch.cuda.synchronize()
    ms = events[0].elapsed_time(events[-1])
    per_step = [events[i].elapsed_time(events[i + 1]) / c for i, c in enumerate(chunks) if c == 8]
    m1 = s.mass()
    psi_min = float(s.psi.min().item())
    # after the timed region: the same `steps` steps repeated until the 95 %
    # Student-t half-width of the repetition means is within ci_target of
    # their mean (at least 3, at most max_reps repetitions)
    reps = []
    while ci_target > 0 and len(reps) < max_reps:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / steps)
        r = spread(reps)
        if len(reps) >= 3 and r["ci95_rel"] <= ci_target:
            break
    s.close()
    return {"ms": ms, "mass0": m0, "mass1": m1, "psi_min": psi_min, "per_step_ms": per_step,
            "rep_ms": reps}


def spread(samples, unit="chunks_of_8_steps"):
    """Median and 95 % Student-t half-width of the mean of step-time samples
    (None with fewer than two)."""
    import numpy as np
    from scipy import stats
    x = np.asarray(samples, dtype=float)
    if x.size < 2:
        return None
    half = float(stats.t.ppf(0.975, x.size - 1) * x.std(ddof=1) / np.sqrt(x.size))
    return {"median_ms": float(np.median(x)), "mean_ms": float(x.mean()), "ci95_half_ms": half,
            "ci95_rel": half / float(x.mean()), unit: int(x.size)}


def cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def error_run(fields, dtype_tag, steps, iord=2, div=False, tvel=False):
    """A fresh run of `steps` steps on the GPU from the workload's initial
    state: psi after the run (the device tensor; the caller copies it to the
    host later, so that the GPU is not left idle meanwhile) and the relative
    mass drift."""
    import numpy as np
    import torch
    from paper_1507_01265_amd.solver import Solver
    tdt = torch.float64 if dtype_tag == "f64" else torch.float32
    f = fields if dtype_tag == "f64" else fields.astype(np.float32)
    s = Solver.from_numpy(f, dtype=tdt, device="cuda", iord=iord, div=div, tvel=tvel)
    m0 = s.mass()
    (_TvStepper(s) if tvel else s.step)(steps)
    m1 = s.mass()
    out = s.psi
    s.close()
    return out, (m1 - m0) / m0


def oracle_steps(fields, steps, iord=2, div=False, tvel=False):
    """The FP64 oracle stepped `steps` times on the host (its inputs: the
    workload's FP64 fields, or their FP32 roundings for an FP32 result);
    returns psi and the seconds it took."""
    import oracle
    f = fields
    t0 = time.perf_counter()
    if tvel:
        lev = lambda k: tuple(a * tv_scale(k) for a in (f.u1, f.u2, f.u3))
        psi, a = f.psi, lev(0)
        for k in range(steps):
            b = lev(k + 1)
            psi = oracle.step_tv(psi, *a, *b, f.h, bc=f.bc, iord=iord, div=div)
            a = b
    else:
        psi = oracle.run(f.psi, f.u1, f.u2, f.u3, f.h, steps, bc=f.bc, iord=iord, div=div)
    return psi, time.perf_counter() - t0


def errors(got, want, drift, steps):
    """Relative errors of a GPU result against the oracle on the same
    inputs: max-norm and 2-norm over the field's own norm, and the GPU
    run's relative mass drift (on an open grid that is the net boundary
    flux, not an error)."""
    import numpy as np
    d = got - want
    return {"rel_linf": float(np.abs(d).max() / np.abs(want).max()),
            "rel_l2": float(np.linalg.norm(d.ravel()) / np.linalg.norm(want.ravel())),
            "mass_drift": float(drift), "steps": int(steps), "against": "FP64 oracle, same inputs"}


def time_region(fn, stream):
    import torch
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def bench_batched(args):
    """96 uneven grids, FP32, K steps: one persistent launch per step over
    all grids (library plan and tuned plan) against the same grids advanced
    one after another through the single-grid path."""
    import numpy as np
    import torch
    from paper_1507_01265_amd import autotune, inputs
    from paper_1507_01265_amd.batch import Batch
    from paper_1507_01265_amd.solver import Solver

    print("# generating 96 grids", file=sys.stderr, flush=True)
    fs = [f.astype(np.float32) for f in inputs.batched_grids(96)]
    grids = [tuple(torch.from_numpy(a).cuda() for a in (f.psi, f.u1, f.u2, f.u3, f.h)) for f in fs]
    cells = sum(g[0].numel() for g in grids)
    saved = [g[0].clone() for g in grids]
    K, W = args.steps, args.warmup

    def restore():
        for g, s0 in zip(grids, saved):
            g[0].copy_(s0)

    out = {}
    print("# batched, library plan", file=sys.stderr, flush=True)
    b = Batch(grids)
    b.step(W)
    ms_default = time_region(lambda: b.step(K), b.stream)
    b.close()
    restore()
    print("# tuning", file=sys.stderr, flush=True)
    tuned = autotune.tune(grids, steps=4, profiles=3)
    for e in tuned.log:
        print("# tune", json.dumps(e), file=sys.stderr, flush=True)
    b = Batch(grids, plan=tuned.plan)
    b.step(W)
    restore()
    ms_tuned = time_region(lambda: b.step(K), b.stream)
    torch.cuda.synchronize()
    result_tuned = [g[0].clone() for g in grids]
    b.close()
    restore()
    print("# single-grid path, one grid after another", file=sys.stderr, flush=True)
    solvers = [Solver(*g, tile=5) for g in grids]
    for s_ in solvers:
        s_.step(W)
    restore()
    stream = solvers[0].stream

    def seq():
        for s_ in solvers:
            s_.step(K)
    ms_single = time_region(seq, stream)
    same = all(torch.equal(g[0], r) for g, r in zip(grids, result_tuned))
    for s_ in solvers:
        s_.close()
    best = min(ms_default, ms_tuned)
    out.update(ms=best, cells=cells, steps=K,
               extra={"ms_library_plan": ms_default, "ms_tuned_plan": ms_tuned,
                      "ms_single_grid_sequence": ms_single,
                      "speedup_vs_single_grid": ms_single / best,
                      "tuned_tile": tuned.tile, "tuner_log": tuned.log,
                      "bitwise_equal_to_single_grid": bool(same),
                      "grids": len(grids)})
    return out


def bench_served(args):
    """Poisson arrivals replayed in real time against the continuous-batching
    server; the plain single-grid path serving the first arrivals one after
    another gives the comparison."""
    import numpy as np
    import torch
    from paper_1507_01265_amd import inputs, serve
    from paper_1507_01265_amd.solver import Solver

    reqs = inputs.served_requests(rate=args.rate, duration=args.duration, seed=5000)
    print(f"# serving {len(reqs)} requests over {args.duration} s", file=sys.stderr, flush=True)
    warm = serve.Server(200e9)
    warm.run(inputs.served_requests(rate=50, duration=0.2, seed=1), realtime=False)
    warm.close()
    srv = serve.Server(args.budget)
    done = srv.run(reqs, realtime=True, log_every=10.0)
    summ = serve.summarize(done, srv.elapsed)
    stats = dict(srv.stats)
    srv.close()
    # plain single-grid path: the first requests, one at a time, back to back
    sample = reqs[:200]
    t0 = time.perf_counter()
    cu = 0
    for r in sample:
        f = inputs.rotation_request_device(r)
        s_ = Solver(*f)
        s_.step(r.steps)
        out = s_.psi.cpu()
        s_.close()
        cu += r.cells * r.steps
    single_rate = cu / (time.perf_counter() - t0)
    return {"summary": summ, "stats": stats, "single_grid_cell_updates_per_s": single_rate,
            "single_grid_sample": len(sample)}


def bench_teams(args):
    """The paper's load-imbalancing procedure with the XCDs as teams, on the
    512x256x64 FP64 rotation grid: value = cell-updates/s of the split
    Algorithm 1 picks (the even split when Theorem 1's condition holds)."""
    import numpy as np
    import torch
    from paper_1507_01265_amd import inputs, teams

    full = inputs.rotation(shape=(8 * 15, 256, 512))  # one field, sliced per plane count

    def make(nz):
        f = full
        return inputs.Fields(f.psi[:nz], f.u1[:nz], f.u2[:nz], f.u3[:nz + 1], f.h[:nz], f.bc)

    print("# teams: speed functions, Algorithm 1, splits", file=sys.stderr, flush=True)
    ex = teams.experiment(make, 64, torch.float64, args.tile or 5, steps=args.steps)
    chosen = [r for r in ex["splits"] if r["dm"] == ex["algorithm1"]["dm"]][0]
    even = [r for r in ex["splits"] if r["dm"] == 0][0]
    return {"metric": "MPDATA cell-updates/s per step", "value": ex["cells"] / (chosen["measured_ms"] / 1e3),
            "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 2,
            "ms_per_step": chosen["measured_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator, resident in HBM)",
            "config": {"workload": WORKLOADS["teams-fp64"][2], "teams": teams.XCDS, "tile": args.tile or 5},
            "even_split_ms": even["measured_ms"], "speedup_vs_even": even["measured_ms"] / chosen["measured_ms"],
            "teams": ex}


# steps of the workload's configured run (the error check runs at most
# this many)
RUN_STEPS = {"rotation": 100, "divergent": 100, "streamfunction": 50}


def error_steps(args, kind):
    return args.error_steps or RUN_STEPS.get(kind, args.steps)


def single_grid(args, workload, fields, sub=False, before_warmup=None):
    """Times exactly --steps steps after --warmup on one grid; returns the
    JSON object of the result (the bench line's fields, or a sub-object)."""
    kind, dtag, desc = WORKLOADS[workload]
    nz, ny, nx = fields.shape
    cells = nx * ny * nz
    word = 8 if dtag == "f64" else 4
    print(f"# {workload}: timing {args.steps} steps after {args.warmup} warmup", file=sys.stderr,
          flush=True)
    iord = OPTIONS.get(workload, {}).get("iord", 2)
    div = OPTIONS.get(workload, {}).get("div", False)
    tvel = OPTIONS.get(workload, {}).get("tvel", False)
    g = time_gpu(fields, dtag, args.steps, args.warmup, args.tile, iord, div, args.ci_target,
                 tvel=tvel, before_warmup=before_warmup)
    ms_per_step = g["ms"] / args.steps
    value = cells * args.steps / (g["ms"] / 1e3)
    roof, valu = roofline(workload, fields.shape, word, ms_per_step, tvel)

    from paper_1507_01265_amd import _lib
    tile = args.tile or _lib.mpdata_default_tile(
        _lib.MPDATA_FP64 if dtag == "f64" else _lib.MPDATA_FP32, int(fields.bc))
    tx, ty, threads = _lib.mpdata_tile_info(tile)
    config = {"workload": desc, "nx": nx, "ny": ny, "nz": nz,
              "bc": "periodic" if fields.bc == 0 else "open", "iord": iord, "nonos": True,
              "divergent_flow_term": div, "time_variation_term": tvel,
              "tile": tile, "output_tile": f"{tx}x{ty}", "threads_per_workgroup": threads}
    head = {"value": value, "unit": "cell-updates/s", "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "dtype": dtag, "config": config} if sub else {
        "metric": "MPDATA cell-updates/s per step",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtag,
        "data": "synthetic (seeded generator, resident in HBM)",
        "config": config}
    return {
        **head,
        "roofline": roof,
        **({"valu": valu} if valu else {}),
        **({"chain": {"launches_per_step": iord - 1,
                      "bytes_per_step_by_design": chain_bytes(fields.shape, word, iord),
                      "achieved_by_design_GBs": chain_bytes(fields.shape, word, iord)
                      / (ms_per_step / 1e3) / 1e9}} if iord > 2 else {}),
        "step_time_spread": spread(g["per_step_ms"]),
        **({"repeated": {**spread(g["rep_ms"], f"repetitions_of_{args.steps}_steps"),
                         "ci_target": args.ci_target}} if len(g["rep_ms"]) >= 2 else {}),
        "mass_drift": (g["mass1"] - g["mass0"]) / g["mass0"],
        "psi_min": g["psi_min"],
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the first few dozen steps after start run ~5 % slow (clocks ramping):
    # 200 untimed steps (~35 ms of FP64 work) put the timed region in steady state
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="rotation-fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=0, help="launch shape id (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the error check against the oracle (and with it the CPU baseline)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="rotation-fp64: do not also time the FP32 grid")
    ap.add_argument("--no-batched", action="store_true",
                    help="rotation-fp64: do not also time the 96-grid batched workload")
    ap.add_argument("--error-steps", type=int, default=0,
                    help="steps of the error check (0 = the workload's configured run: 100 "
                         "rotation, 50 streamfunction)")
    ap.add_argument("--ci-target", type=float, default=0.01,
                    help="after the timed steps, repeat them until the 95%% Student-t half-width "
                         "is within this fraction of the mean (at most 50 times; 0 = off)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0 = the OpenMP default)")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="served: seconds of arrivals")
    ap.add_argument("--budget", type=float, default=200e9, help="served: HBM budget in bytes")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB device buffer once (a copy kernel of "
                         "known size for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one MI355X: the MPDATA path is built and timed on a single "
              f"GPU (asked for --gpus {args.gpus}); multi-GPU sharding is design-only.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    kind, dtag, desc = WORKLOADS[args.workload]
    if kind == "batched":
        r = bench_batched(args)
        line = {"metric": "MPDATA cell-updates/s per step", "value": r["cells"] * r["steps"] / (r["ms"] / 1e3),
                "unit": "cell-updates/s", "n_gpus": 1, "steps": r["steps"], "warmup": args.warmup,
                "ms_per_step": r["ms"] / r["steps"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded generator, resident in HBM)",
                "config": {"workload": desc, "cells": r["cells"]}}
        line.update(r["extra"])
        print(json.dumps(line), flush=True)
        return
    if kind == "teams":
        r = bench_teams(args)
        print(json.dumps(r), flush=True)
        return
    if kind == "served":
        r = bench_served(args)
        sm = r["summary"]
        line = {"metric": "MPDATA cell-updates/s (served), p50/p99 latency", "value": sm["cell_updates_per_s"],
                "unit": "cell-updates/s", "n_gpus": 1, "steps": None, "warmup": None,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "mixed f32/f64",
                "data": "synthetic (seeded Poisson arrivals, fields built on the device)",
                "config": {"workload": desc, "rate": args.rate, "duration_s": args.duration,
                           "budget_bytes": args.budget},
                "p50_ms": sm["p50_ms"], "p99_ms": sm["p99_ms"], "served": sm, "server": r["stats"],
                "single_grid_cell_updates_per_s": r["single_grid_cell_updates_per_s"],
                "single_grid_sample_requests": r["single_grid_sample"]}
        print(json.dumps(line), flush=True)
        return
    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    fields = make_fields(kind)
    nz, ny, nx = fields.shape
    cells = nx * ny * nz
    iord = OPTIONS.get(args.workload, {}).get("iord", 2)
    div = OPTIONS.get(args.workload, {}).get("div", False)
    tvel = OPTIONS.get(args.workload, {}).get("tvel", False)
    # the default workload also times the same grid in FP32 (the metric names
    # both precisions) and the batched workload (96 uneven FP32 grids, one
    # persistent launch per step, against the same grids run one after
    # another through the single-grid path)
    precisions = [args.workload] + (["rotation-fp32"] if args.workload == "rotation-fp64"
                                    and not args.no_fp32 else [])
    # errors of a fresh run of E steps (the workload's configured run)
    # against the oracle's E steps on the same inputs; the FP64 oracle run is
    # also the CPU baseline sample.  The oracle runs first, on the host.
    E = error_steps(args, kind)
    want = {}
    if not args.no_errors:
        import oracle
        if args.cpu_threads:
            oracle.set_threads(args.cpu_threads)
        for wl in precisions:
            dtag = WORKLOADS[wl][1]
            print(f"# oracle: {wl}, {E} steps", file=sys.stderr, flush=True)
            f64 = fields if dtag == "f64" else fields.astype("float32").as_f64()
            want[wl] = oracle_steps(f64, E, iord, div, tvel)
    # Everything else runs on the GPU after the headline grid is set up and
    # before its warm-up: the FP32 grid (its error run before its own
    # warm-up), the batched workload and last the GPU run the headline's
    # errors are taken from.  A new run needs about 100 steps (20 ms) of the
    # same kernel before its step time settles (measured in FP64: the first
    # 100 steps after a set-up or an idle GPU take 182-197 us, later ones
    # 167 us, whatever ran before), so an error run of the configured length
    # right before the warm-up leaves the timed steps in steady state.
    extra, got = {}, {}

    def error_gpu(wl):
        if not args.no_errors:
            print(f"# errors: {wl}, {E} steps on the GPU", file=sys.stderr, flush=True)
            got[wl] = error_run(fields, WORKLOADS[wl][1], E, iord, div, tvel)

    def others():
        if "rotation-fp32" in precisions:
            extra["fp32"] = single_grid(args, "rotation-fp32", fields, sub=True,
                                        before_warmup=lambda: error_gpu("rotation-fp32"))
        if args.workload == "rotation-fp64" and not args.no_batched:
            r = bench_batched(args)
            extra["batched"] = {
                "value": r["cells"] * r["steps"] / (r["ms"] / 1e3), "unit": "cell-updates/s",
                "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms"] / r["steps"],
                "dtype": "f32",
                "config": {"workload": WORKLOADS["batched-fp32"][2], "cells": r["cells"]},
                **{k: v for k, v in r["extra"].items() if k != "tuner_log"}}
        error_gpu(args.workload)
    line = single_grid(args, args.workload, fields, before_warmup=others)
    line.update(extra)
    for wl in precisions if not args.no_errors else []:
        obj = line if wl == args.workload else line["fp32"]
        (g, drift), (w, el) = got[wl], want[wl]
        obj["errors"] = errors(g.cpu().numpy().astype("float64"), w, drift, E)
        if obj is line and not args.no_cpu_baseline:
            line["cpu_baseline"] = {
                "value": cells * E / el, "unit": "cell-updates/s", "cores": oracle.threads(),
                "kind": "oracle",
                "sample": f"{nx}x{ny}x{nz} {args.workload} inputs, {E} FP64 steps of the "
                          f"whole grid (the run the errors are taken against), {el:.1f} s",
                "cpu_model": cpu_model()}
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 2 * n * 8
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
