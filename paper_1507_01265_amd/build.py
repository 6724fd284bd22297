"""Build of libmpdata.so (hipcc, gfx950) in the package directory.

``python -m paper_1507_01265_amd.build`` compiles every HIP source of the
library.  The flags: gfx950 code only; packed FP32 instructions disabled; FMA
contraction on (within expressions only in the step kernels; the
compensated sums of the mass reduction switch it off locally); the step
kernels are compiled without NaN semantics.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpdata.so")
# Scheduling of the march kernels: the compiler's AMDGPU register-pressure
# trackers leave fewer spills at the 168-VGPR limit of three waves per SIMD
# (the time-dependent FP64 step: 8 VGPRs instead of 29, 15 % faster; the open
# FP64 step: 8 instead of 36), and the strategy that keeps memory clauses
# together makes the FP64 steps 1.5-2 % faster (measured; FP32 unchanged,
# the ILP strategy slower).
SCHED = ["-mllvm", "-amdgpu-use-amdgpu-trackers=1",
         "-mllvm", "-amdgpu-sched-strategy=max-memory-clause"]
# (source, extra flags): the step kernels assume finite inputs (no NaN
# semantics, so min/max need no operand canonicalisation) and contract a
# product and a sum into an FMA only within one expression
# (-ffp-contract=on): the march is unrolled into several copies of one
# iteration, and contraction across statements could round the same cell
# differently in different copies, so that launch plans (which decide the
# copy a plane lands in) would change bits.  The mass and validation kernels
# keep IEEE semantics because they detect NaN/Inf.
SOURCES = [("mpdata_step.hip", ["-fno-honor-nans", "-ffp-contract=on", *SCHED]),
           ("mpdata_pass.hip", ["-fno-honor-nans", "-ffp-contract=on", *SCHED]),
           ("mpdata_reduce.hip", []), ("mpdata_abi.hip", [])]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=fast",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libmpdata.so."""
    objs, procs = [], []
    for src, extra in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
