"""Single-grid MPDATA solver on torch device tensors (plumbing only).

torch provides the device memory (the caller's field tensors and the
workspace) and the stream; every step of the computation runs in
libmpdata's HIP kernels through the C ABI.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

BC = {"periodic": _lib.MPDATA_BC_PERIODIC, "open": _lib.MPDATA_BC_OPEN,
      _lib.MPDATA_BC_PERIODIC: _lib.MPDATA_BC_PERIODIC, _lib.MPDATA_BC_OPEN: _lib.MPDATA_BC_OPEN}
DTYPES = {torch.float64: _lib.MPDATA_FP64, torch.float32: _lib.MPDATA_FP32}


def _check_runtime():
    mapped = _lib.hip_runtimes_mapped()
    if len(mapped) > 1:
        raise RuntimeError(f"more than one HIP runtime mapped: {mapped}")


def make_params(shape, dtype=torch.float64, bc="periodic", iord=2, nonos=True, eps=1e-15, tile=0,
                graph=True, vsign=False, div=False, tvel=False):
    nz, ny, nx = shape
    flags = ((0 if graph else _lib.MPDATA_FLAG_NO_GRAPH) | (_lib.MPDATA_FLAG_VSIGN if vsign else 0)
             | (_lib.MPDATA_FLAG_DIV if div else 0) | (_lib.MPDATA_FLAG_TVEL if tvel else 0))
    return _lib.mpdata_params(nx, ny, nz, DTYPES[dtype], BC[bc], iord, int(bool(nonos)), tile,
                              flags, 0, eps)


class Solver:
    """``Solver(psi, u1, u2, u3, h, bc=..., iord=2, nonos=True, vsign=False)``.

    vsign: fields of variable sign (|psi1| in the pseudo-velocity ratios).
    div: the divergent-flow term of the pseudo-velocity (flows that are not
    divergence-free).
    tvel: Courant numbers that change in time (``step_tv``).

    psi: [nz][ny][nx] device tensor (float64 or float32), updated in place by
    ``step``; u1 [nz][ny][nx+1], u2 [nz][ny+1][nx], u3 [nz+1][ny][nx], h like
    psi.  The tensors are borrowed for the solver's lifetime.
    """

    def __init__(self, psi, u1, u2, u3, h, *, bc="periodic", iord=2, nonos=True, eps=1e-15,
                 tile=0, graph=True, stream=None, vsign=False, div=False, tvel=False):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpdata needs a GPU")
        _lib.load()
        _check_runtime()
        if psi.dim() != 3:
            raise ValueError("psi must be 3-D [nz][ny][nx]")
        nz, ny, nx = psi.shape
        want = {"psi": (nz, ny, nx), "u1": (nz, ny, nx + 1), "u2": (nz, ny + 1, nx),
                "u3": (nz + 1, ny, nx), "h": (nz, ny, nx)}
        for name, t in zip(want, (psi, u1, u2, u3, h)):
            if tuple(t.shape) != want[name]:
                raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {want[name]}")
            if not t.is_cuda or not t.is_contiguous() or t.dtype != psi.dtype:
                raise ValueError(f"{name}: needs a contiguous {psi.dtype} device tensor")
        self.params = make_params(psi.shape, psi.dtype, bc, iord, nonos, eps, tile, graph, vsign,
                                  div, tvel)
        self.stream = stream if stream is not None else torch.cuda.current_stream(psi.device)
        ws_bytes = _lib.mpdata_workspace_bytes(self.params)
        if ws_bytes == 0:
            raise ValueError("invalid parameters: " + str(dict(nx=nx, ny=ny, nz=nz, bc=bc,
                                                               iord=iord, nonos=nonos)))
        # allocated on the stream the steps run on, so the caching allocator
        # does not hand it out while they are queued
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=psi.device)
        self.psi, self.u1, self.u2, self.u3, self.h = psi, u1, u2, u3, h
        self._ctx = None
        self._ctx = _lib.mpdata_create(self.params, psi.data_ptr(), u1.data_ptr(), u2.data_ptr(),
                                       u3.data_ptr(), h.data_ptr(), self.workspace.data_ptr(),
                                       ws_bytes, self.stream.cuda_stream)

    @classmethod
    def from_numpy(cls, fields, dtype=torch.float64, device="cuda", **kw):
        """Upload an ``inputs.Fields`` (or 5-tuple of arrays) and build a solver."""
        arrs = (fields.psi, fields.u1, fields.u2, fields.u3, fields.h) if hasattr(fields, "psi") \
            else fields
        np_dtype = np.float64 if dtype == torch.float64 else np.float32
        ts = [torch.from_numpy(np.ascontiguousarray(a, dtype=np_dtype)).to(device) for a in arrs]
        if hasattr(fields, "bc") and "bc" not in kw:
            kw["bc"] = fields.bc
        return cls(*ts, **kw)

    def step(self, nsteps: int = 1):
        _lib.mpdata_step(self._ctx, int(nsteps))

    def step_tv(self, levels):
        """len(levels) steps with Courant numbers that change in time:
        levels[s] = (u1, u2, u3), device tensors shaped like the solver's,
        at the end of step s (the bound velocity is the start of step 0).
        The last level becomes the bound velocity (kept referenced here)."""
        if not levels:
            return
        for lv in levels:
            for name, t, ref in zip(("u1", "u2", "u3"), lv, (self.u1, self.u2, self.u3)):
                if (tuple(t.shape) != tuple(ref.shape) or t.dtype != ref.dtype or not t.is_cuda
                        or not t.is_contiguous()):
                    raise ValueError(f"level {name}: needs a contiguous {ref.dtype} device tensor "
                                     f"of shape {tuple(ref.shape)}")
        _lib.mpdata_step_tv(self._ctx, [lv[0].data_ptr() for lv in levels],
                            [lv[1].data_ptr() for lv in levels], [lv[2].data_ptr() for lv in levels])
        # the allocator must not hand a level's memory out before the steps
        # that read it have run on the solver's stream
        for lv in levels:
            for t in lv:
                t.record_stream(self.stream)
        self.u1, self.u2, self.u3 = levels[-1]

    def mass(self) -> float:
        return _lib.mpdata_mass(self._ctx)

    def sync(self):
        _lib.mpdata_sync(self._ctx)

    def set_psi(self, src):
        _lib.mpdata_set_psi(self._ctx, src.data_ptr())

    def get_psi(self, dst):
        _lib.mpdata_get_psi(self._ctx, dst.data_ptr())

    @property
    def steps_done(self) -> int:
        return _lib.mpdata_steps_done(self._ctx)

    def close(self):
        if self._ctx is not None:
            _lib.mpdata_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
