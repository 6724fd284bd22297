"""Parity bars of the GPU tests against the FP64 oracle.

FP64: rel-Linf <= 1e-12 (max|gpu - oracle| / max|oracle|).

FP32 (FP32 storage and bulk arithmetic, the limiter's sums and divides in
FP64): the oracle runs in FP64 on the same FP32-rounded inputs.  A step
commits a few units of FP32 rounding (2^-24, about 6e-8) per stage; the
scheme damps rather than accumulates them, and the observed errors stay
below about 1e-6 rel-Linf even after 100 steps.  The bar is a fixed one,
about ten times the observed error, for runs of at most 100 steps:
rel-Linf <= 1e-5 and rel-L2 <= 2e-6; on periodic grids the relative mass
drift is at most 1e-6.
"""
import numpy as np

FP64_LINF = 1e-12
FP32_LINF = 1e-5
FP32_L2 = 2e-6
FP32_DRIFT = 1e-6


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def check_fp32(got, want, label=""):
    """Asserts the FP32 bar and returns (rel-Linf, rel-L2)."""
    e_inf, e_2 = rel_linf(got, want), rel_l2(got, want)
    print(f"fp32 {label} rel-Linf {e_inf:.3e} rel-L2 {e_2:.3e}", flush=True)
    assert e_inf <= FP32_LINF and e_2 <= FP32_L2, (label, e_inf, e_2)
    return e_inf, e_2


def check_fp64(got, want, label=""):
    e = rel_linf(got, want)
    print(f"fp64 {label} rel-Linf {e:.3e}", flush=True)
    assert e <= FP64_LINF, (label, e)
    return e
