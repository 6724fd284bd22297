#!/usr/bin/env python3
"""Benchmark of the MPDATA time step on one MI355X.

One "step" is one MPDATA time step (donor-cell pass, pseudo-velocities,
limiter, corrective pass -- one launch of the fused kernel) over the whole
grid.  The default workload is the 512x256x64 periodic solid-body-rotation
grid in FP64 (cone + slotted cube on a zero background, h in [0.8, 1.2]);
inputs are synthetic, seeded and resident in HBM before the timed region.

Prints ONE JSON line: cell-updates/s over exactly --steps timed steps after
--warmup untimed ones, the HBM roofline of the fused kernel (algorithmic
bytes per launch / average launch time from HIP events on the solver's
stream), and the FP64 CPU oracle timed on a bounded sample of the same
workload on the host's cores.
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
}


def algorithmic_bytes(shape, word):
    """The five input arrays read once and psi written once per step:
    psi, h and psi_out are nx*ny*nz words; u1, u2, u3 carry one extra face
    along their own axis."""
    nz, ny, nx = shape
    n = nx * ny * nz
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    return word * (3 * n + faces)


def make_fields(kind):
    from paper_1507_01265_amd import inputs
    return inputs.rotation() if kind == "rotation" else inputs.streamfunction()


def time_gpu(fields, dtype_tag, steps, warmup, tile=0):
    import numpy as np
    import torch
    from paper_1507_01265_amd.solver import Solver

    tdt = torch.float64 if dtype_tag == "f64" else torch.float32
    f = fields if dtype_tag == "f64" else fields.astype(np.float32)
    s = Solver.from_numpy(f, dtype=tdt, device="cuda", tile=tile)
    stream = s.stream
    m0 = s.mass()
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    s.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    m1 = s.mass()
    psi_min = float(s.psi.min().item())
    s.close()
    return {"ms": ms, "mass0": m0, "mass1": m1, "psi_min": psi_min}


def cpu_baseline(fields, budget_s=12.0, max_steps=40):
    """The FP64 oracle as it stands, stepped on the host until the budget is
    spent (at least 2 steps)."""
    import oracle
    f = fields
    psi = f.psi
    steps = 0
    t0 = time.perf_counter()
    while True:
        psi = oracle.step(psi, f.u1, f.u2, f.u3, f.h, bc=f.bc)
        steps += 1
        el = time.perf_counter() - t0
        if (steps >= 2 and el >= budget_s) or steps >= max_steps:
            break
    return steps, el


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rotation-fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=0, help="launch shape id (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
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
    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    fields = make_fields(kind)
    nz, ny, nx = fields.shape
    cells = nx * ny * nz
    word = 8 if dtag == "f64" else 4

    print(f"# timing {args.steps} steps after {args.warmup} warmup", file=sys.stderr, flush=True)
    g = time_gpu(fields, dtag, args.steps, args.warmup, args.tile)
    ms_per_step = g["ms"] / args.steps
    value = cells * args.steps / (g["ms"] / 1e3)
    abytes = algorithmic_bytes(fields.shape, word)
    achieved = abytes / (ms_per_step / 1e3) / 1e9

    line = {
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
        "config": {"workload": desc, "nx": nx, "ny": ny, "nz": nz,
                   "bc": "periodic" if fields.bc == 0 else "open", "iord": 2, "nonos": True,
                   "tile": args.tile},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": abytes},
        "mass_drift": (g["mass1"] - g["mass0"]) / g["mass0"],
        "psi_min": g["psi_min"],
    }
    if not args.no_cpu_baseline:
        import oracle
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        f64 = fields if dtag == "f64" else fields.astype("float32").as_f64()
        steps, el = cpu_baseline(f64, args.cpu_budget)
        line["cpu_baseline"] = {"value": cells * steps / el, "unit": "cell-updates/s",
                                "cores": oracle.threads(), "kind": "oracle",
                                "sample": f"{nx}x{ny}x{nz} {args.workload} inputs, {steps} FP64 "
                                          f"steps of the whole grid, {el:.1f} s"}
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
