"""Batches of uneven MPDATA grids advanced by one persistent launch per step.

torch provides the device memory and the stream; the C ABI
(``mpdata_batch_*``) does the work.  All grids of a batch share dtype,
boundary mode, limiter switch and eps; their sizes differ.  A plan -- which
workgroup of the persistent kernel runs which (grid, tile, z-range) segment
-- comes from the library (``plan=None``) or from :mod:`.autotune`.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .solver import BC, DTYPES, _check_runtime


class Batch:
    """``Batch(grids, ...)`` with ``grids`` a list of 5-tuples of device
    tensors ``(psi, u1, u2, u3, h)`` (shapes as for :class:`Solver`).
    ``vsign`` and ``div`` select the variable-sign option and the
    divergent-flow term for every grid (built for the 32x24 and 32x32
    launch shapes)."""

    def __init__(self, grids, *, bc="periodic", nonos=True, eps=1e-15, tile=0, plan=None,
                 graph=True, stream=None, vsign=False, div=False):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpdata needs a GPU")
        _lib.load()
        _check_runtime()
        if not grids:
            raise ValueError("empty batch")
        dtype = grids[0][0].dtype
        flags = ((0 if graph else _lib.MPDATA_FLAG_NO_GRAPH)
                 | (_lib.MPDATA_FLAG_VSIGN if vsign else 0) | (_lib.MPDATA_FLAG_DIV if div else 0))
        self.params = []
        for i, (psi, u1, u2, u3, h) in enumerate(grids):
            nz, ny, nx = psi.shape
            want = [(nz, ny, nx), (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx)]
            for t, w in zip((psi, u1, u2, u3, h), want):
                if tuple(t.shape) != w or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"grid {i}: expected contiguous {dtype} device tensors {want}")
            self.params.append(_lib.mpdata_params(nx, ny, nz, DTYPES[dtype], BC[bc], 2,
                                                  int(bool(nonos)), tile, flags, 0, eps))
        self.grids = grids
        self.dtype = dtype
        self.bc, self.nonos, self.eps = bc, nonos, eps
        self.vsign, self.div = vsign, div
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        keep = None
        cplan = None
        max_seg = max_wg = 0
        if plan is not None:
            tile_p, seg, wg_begin = plan
            cplan, keep = _lib.make_plan(tile_p, seg, wg_begin)
            max_seg, max_wg = cplan.nseg, cplan.nwg
        ws_bytes = _lib.mpdata_batch_workspace_bytes(self.params, max_seg, max_wg)
        if ws_bytes == 0:
            raise ValueError("invalid batch parameters")
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=grids[0][0].device)
        self._b = None
        self._b = _lib.mpdata_batch_create(
            self.params, [g[0].data_ptr() for g in grids], [g[1].data_ptr() for g in grids],
            [g[2].data_ptr() for g in grids], [g[3].data_ptr() for g in grids],
            [g[4].data_ptr() for g in grids], self.workspace.data_ptr(), ws_bytes,
            self.stream.cuda_stream, cplan)
        del keep
        if plan is not None:
            self.tile, self.nseg = plan[0], cplan.nseg
        else:
            self.tile = tile if tile else _lib.mpdata_default_tile(DTYPES[dtype], BC[bc])
            self.nseg, _ = _lib.mpdata_batch_default_plan_size(self.params, self.tile)

    @classmethod
    def from_numpy(cls, fields_list, dtype=torch.float32, device="cuda", **kw):
        np_dtype = np.float64 if dtype == torch.float64 else np.float32
        grids = []
        for f in fields_list:
            grids.append(tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np_dtype)).to(device)
                               for a in (f.psi, f.u1, f.u2, f.u3, f.h)))
        if "bc" not in kw:
            kw["bc"] = fields_list[0].bc
        return cls(grids, **kw)

    def step(self, nsteps: int = 1):
        _lib.mpdata_batch_step(self._b, int(nsteps))

    def profile_step(self):
        """One step of every grid; returns the wall-clock ticks (100 MHz) of
        every segment of the plan, measured with all workgroups running."""
        return _lib.mpdata_batch_profile_step(self._b, self.nseg)

    def mass(self, i: int) -> float:
        return _lib.mpdata_batch_mass(self._b, i)

    def sync(self):
        _lib.mpdata_batch_sync(self._b)

    def psi(self, i: int):
        return self.grids[i][0]

    @property
    def cells(self) -> int:
        return sum(g[0].numel() for g in self.grids)

    def close(self):
        if self._b is not None:
            _lib.mpdata_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
