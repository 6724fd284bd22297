"""FP64 CPU oracle of one MPDATA time step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library
(``paper_1507_01265_amd``) never imports it, and this package imports
nothing from the product.

The arithmetic lives in ``mpdata_oracle.c`` (plain C, whole-array stages in
the order of the scheme, no fusion); this module is argument marshalling
through ``ctypes`` plus the build of that file with gcc.  What the step
computes and every reading taken where the paper is silent is stated at the
top of ``mpdata_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpdata_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC = 0
BC_OPEN = 1


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("bc", ctypes.c_int),
        ("iord", ctypes.c_int),
        ("nonos", ctypes.c_int),
        ("vsign", ctypes.c_int),
        ("div", ctypes.c_int),
        ("eps", ctypes.c_double),
    ]


class _Stages(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("psi1", "v1", "v2", "v3", "mx", "mn", "beta_up", "beta_dn")]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (FMA contraction off, OpenMP on)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_step.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp,
                                 ctypes.POINTER(_Stages)]
        lib.orc_step.restype = ctypes.c_int
        lib.orc_step_tv.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                    ctypes.POINTER(_Stages)]
        lib.orc_step_tv.restype = ctypes.c_int
        lib.orc_run.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, ctypes.c_int]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_mass.argtypes = [ctypes.c_long, dp, dp]
        lib.orc_mass.restype = ctypes.c_double
        lib.orc_open_inflow.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp]
        lib.orc_open_inflow.restype = ctypes.c_double
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a, shape, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"{name}: shape {a.shape}, expected {shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(shape, bc, iord, nonos, eps, vsign=False, div=False):
    nz, ny, nx = shape
    return _Params(nx, ny, nz, int(bc), int(iord), int(bool(nonos)), int(bool(vsign)),
                   int(bool(div)), float(eps))


def _inputs(psi, u1, u2, u3, h):
    psi = np.asarray(psi)
    if psi.ndim != 3:
        raise ValueError("psi must be 3-D [nz][ny][nx]")
    nz, ny, nx = psi.shape
    return (_f64(psi, (nz, ny, nx), "psi"), _f64(u1, (nz, ny, nx + 1), "u1"),
            _f64(u2, (nz, ny + 1, nx), "u2"), _f64(u3, (nz + 1, ny, nx), "u3"),
            _f64(h, (nz, ny, nx), "h"))


def step(psi, u1, u2, u3, h, *, bc=BC_PERIODIC, iord=2, nonos=True, eps=1e-15,
         stages=False, vsign=False, div=False):
    """One step; returns psi at n+1 (and a dict of stage arrays if asked).
    vsign: the variable-sign option (|psi1| in the pseudo-velocity ratios);
    div: the divergent-flow term of the pseudo-velocity."""
    psi, u1, u2, u3, h = _inputs(psi, u1, u2, u3, h)
    p = _params(psi.shape, bc, iord, nonos, eps, vsign, div)
    out = np.empty_like(psi)
    st = None
    arrays = {}
    if stages:
        nz, ny, nx = psi.shape
        arrays = {"psi1": np.zeros_like(psi), "v1": np.zeros((nz, ny, nx + 1)),
                  "v2": np.zeros((nz, ny + 1, nx)), "v3": np.zeros((nz + 1, ny, nx)),
                  "mx": np.zeros_like(psi), "mn": np.zeros_like(psi),
                  "beta_up": np.zeros_like(psi), "beta_dn": np.zeros_like(psi)}
        st = _Stages(*[arrays[k].ctypes.data for k in
                       ("psi1", "v1", "v2", "v3", "mx", "mn", "beta_up", "beta_dn")])
    rc = _load().orc_step(ctypes.byref(p), _ptr(psi), _ptr(u1), _ptr(u2), _ptr(u3),
                          _ptr(h), _ptr(out), ctypes.byref(st) if st else None)
    if rc:
        raise ValueError(f"oracle step failed ({rc})")
    return (out, arrays) if stages else out


def step_tv(psi, u1, u2, u3, w1, w2, w3, h, *, bc=BC_PERIODIC, iord=2, nonos=True, eps=1e-15,
            vsign=False, div=False):
    """One step with Courant numbers that change in time: u1..u3 at the
    start of the step, w1..w3 at its end (the time-variation term of the
    first corrective pass, see mpdata_oracle.c)."""
    psi, u1, u2, u3, h = _inputs(psi, u1, u2, u3, h)
    nz, ny, nx = psi.shape
    w1 = _f64(w1, (nz, ny, nx + 1), "w1")
    w2 = _f64(w2, (nz, ny + 1, nx), "w2")
    w3 = _f64(w3, (nz + 1, ny, nx), "w3")
    p = _params(psi.shape, bc, iord, nonos, eps, vsign, div)
    out = np.empty_like(psi)
    rc = _load().orc_step_tv(ctypes.byref(p), _ptr(psi), _ptr(u1), _ptr(u2), _ptr(u3),
                             _ptr(w1), _ptr(w2), _ptr(w3), _ptr(h), _ptr(out), None)
    if rc:
        raise ValueError(f"oracle step failed ({rc})")
    return out


def run_tv(psi, levels, h, *, bc=BC_PERIODIC, iord=2, nonos=True, eps=1e-15, vsign=False,
           div=False, term=True):
    """len(levels) - 1 steps; levels[s] = (u1, u2, u3) at time level s.  Step
    s runs from level s to level s + 1 (with term=False each step holds the
    Courant numbers of its start, the plain scheme)."""
    out = np.ascontiguousarray(psi, dtype=np.float64).copy()
    for s in range(len(levels) - 1):
        a, b = levels[s], levels[s + 1]
        if term:
            out = step_tv(out, *a, *b, h, bc=bc, iord=iord, nonos=nonos, eps=eps, vsign=vsign,
                          div=div)
        else:
            out = step(out, *a, h, bc=bc, iord=iord, nonos=nonos, eps=eps, vsign=vsign, div=div)
    return out


def run(psi, u1, u2, u3, h, nsteps, *, bc=BC_PERIODIC, iord=2, nonos=True, eps=1e-15,
        vsign=False, div=False):
    """nsteps steps; returns a new array."""
    psi, u1, u2, u3, h = _inputs(psi, u1, u2, u3, h)
    psi = psi.copy()
    p = _params(psi.shape, bc, iord, nonos, eps, vsign, div)
    rc = _load().orc_run(ctypes.byref(p), _ptr(psi), _ptr(u1), _ptr(u2), _ptr(u3),
                         _ptr(h), int(nsteps))
    if rc:
        raise ValueError(f"oracle run failed ({rc})")
    return psi


def mass(psi, h):
    """Compensated sum of h*psi (Dot2)."""
    psi = np.ascontiguousarray(psi, dtype=np.float64).ravel()
    h = np.ascontiguousarray(h, dtype=np.float64).ravel()
    if psi.shape != h.shape:
        raise ValueError("psi and h differ in size")
    return float(_load().orc_mass(psi.size, _ptr(h), _ptr(psi)))


def open_inflow(psi, u1, u2, u3):
    """Net first-order inflow through the faces of an open domain."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    nz, ny, nx = psi.shape
    u1 = _f64(u1, (nz, ny, nx + 1), "u1")
    u2 = _f64(u2, (nz, ny + 1, nx), "u2")
    u3 = _f64(u3, (nz + 1, ny, nx), "u3")
    p = _params(psi.shape, BC_OPEN, 2, True, 1e-15)
    return float(_load().orc_open_inflow(ctypes.byref(p), _ptr(psi), _ptr(u1), _ptr(u2),
                                         _ptr(u3)))


def threads() -> int:
    """OpenMP threads the oracle's stage loops use."""
    return int(_load().orc_threads())


def set_threads(n: int) -> int:
    """Runs the stage loops on n OpenMP threads (results do not depend on
    it); returns the number now in effect."""
    if n < 1:
        raise ValueError("threads must be >= 1")
    return int(_load().orc_set_threads(int(n)))
