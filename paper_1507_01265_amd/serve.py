"""Continuous-batching server of MPDATA solves.

Requests (a grid, a step count, a precision) arrive over time.  The server
keeps their fields resident in HBM and advances every resident request
together: each tick advances all of them by ``k = min(k_max, fewest steps
left)`` steps with one persistent launch per step and precision (the pools of
the C ABI, whose plan is rebuilt for the current members).  A request is
admitted -- its fields built in device memory on a side stream, validated and
added to the pool of its precision -- as soon as the HBM it needs fits in the
budget, so newcomers join at the next tick while others are in flight.  A
request is retired when its steps are done: its result is copied to the host,
its memory returned to the budget.  Latency = result on the host - arrival.

Results do not depend on the company a request keeps: every cell of a grid
is computed by the same operations whatever the plan, so a request served
alone and in a mix gives the same bits.

A request that fails (refused at admission, a step that cannot be enqueued,
a result that is not finite) is retired as failed with its reason; its slot
and budget are released and the loop carries on with the others.
"""
from __future__ import annotations

import collections
import dataclasses
import sys
import time

import numpy as np
import torch

from . import _lib
from .inputs import Request, rotation_request_device
from .solver import BC, DTYPES, _check_runtime


class Pool:
    """Thin owner of an ``mpdata_pool`` (members share dtype, bc, limiter)."""

    def __init__(self, dtype, *, bc="periodic", nonos=True, eps=1e-15, tile=0, max_grids=512,
                 max_segments=1 << 16, stream=None, device="cuda"):
        _lib.load()
        _check_runtime()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        shared = _lib.mpdata_params(1, 1, 1, DTYPES[dtype], BC[bc], 2, int(bool(nonos)), tile, 0,
                                    0, eps)
        ws = _lib.mpdata_pool_workspace_bytes(max_grids, max_segments)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        self._p = None
        self._p = _lib.mpdata_pool_create(shared, max_grids, max_segments,
                                          self.workspace.data_ptr(), ws, self.stream.cuda_stream)
        self.dtype = dtype

    def add(self, fields, scratch, validate_stream=None) -> int:
        psi, u1, u2, u3, h = fields
        nz, ny, nx = psi.shape
        vs = validate_stream.cuda_stream if validate_stream is not None else None
        return _lib.mpdata_pool_add(self._p, nx, ny, nz, psi.data_ptr(), scratch.data_ptr(),
                                    u1.data_ptr(), u2.data_ptr(), u3.data_ptr(), h.data_ptr(), vs)

    def remove(self, slot):
        _lib.mpdata_pool_remove(self._p, slot)

    def step(self, n):
        _lib.mpdata_pool_step(self._p, int(n))

    @property
    def size(self):
        return _lib.mpdata_pool_size(self._p)

    def close(self):
        if self._p is not None:
            _lib.mpdata_pool_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_bytes(req: Request) -> int:
    """HBM a request holds while resident: two psi buffers, u1, u2, u3, h."""
    nz, ny, nx = req.shape
    word = 4 if req.fp32 else 8
    n = nx * ny * nz
    return word * (2 * n + (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1) + n)


@dataclasses.dataclass
class Done:
    """A retired request.  ``error`` is None for a request served to the
    end; otherwise it says why the request failed (its result is None)."""
    rid: int
    arrival: float
    admitted: float
    finished: float
    cells: int
    steps: int
    fp32: bool
    result: np.ndarray | None = None
    error: str | None = None


class Scheduler:
    """Admission and tick sizing of continuous batching, independent of the
    device: FIFO admission under an HBM budget, ticks of
    ``min(k_max, fewest steps left)`` steps over the members present when the
    tick starts."""

    def __init__(self, budget_bytes: float, k_max: int = 8, size_of=request_bytes):
        self.budget = float(budget_bytes)
        self.k_max = int(k_max)
        self.size_of = size_of
        self.queue = collections.deque()
        self.left = {}          # rid -> steps left (members only)
        self.reqs = {}
        self.used = 0.0
        self.peak = 0.0
        self.waits = 0

    def arrive(self, req):
        if self.size_of(req) > self.budget:
            raise ValueError(f"request {req.rid} needs {self.size_of(req)} B > budget {self.budget}")
        self.queue.append(req)

    def admit(self):
        """Requests to admit now (FIFO while they fit)."""
        out = []
        while self.queue:
            need = self.size_of(self.queue[0])
            if self.used + need > self.budget:
                self.waits += 1
                break
            req = self.queue.popleft()
            self.used += need
            self.peak = max(self.peak, self.used)
            self.left[req.rid] = req.steps
            self.reqs[req.rid] = req
            out.append(req)
        return out

    def tick(self):
        """(k, members) of the next tick, or (0, []) with no members."""
        if not self.left:
            return 0, []
        return min(self.k_max, min(self.left.values())), list(self.left)

    def advance(self, members, k):
        """Members advanced by k steps; returns the finished requests (their
        budget is released)."""
        fin = []
        for rid in members:
            self.left[rid] -= k
            if self.left[rid] <= 0:
                del self.left[rid]
                req = self.reqs.pop(rid)
                self.used -= self.size_of(req)
                fin.append(req)
        return fin

    def drop(self, rid):
        """Takes a failed member out before its steps are done and releases
        its budget (no-op for a rid that is not a member)."""
        req = self.reqs.pop(rid, None)
        if req is None:
            return None
        del self.left[rid]
        self.used -= self.size_of(req)
        return req

    @property
    def idle(self):
        return not self.left and not self.queue


class GpuExecutor:
    """The device side of the server: one pool per precision on the compute
    stream; a newcomer's fields are built on a side stream and validated
    there when it joins its pool."""

    def __init__(self, device="cuda", nonos=True):
        self.device = device
        self.compute = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()
        self.pools = {True: Pool(torch.float32, nonos=nonos, stream=self.compute),
                      False: Pool(torch.float64, nonos=nonos, stream=self.compute)}

    def add(self, req):
        """Resident fields of a request, joined to its pool (raises if the
        library refuses them)."""
        with torch.cuda.stream(self.side):
            fields = rotation_request_device(req, self.device)
            scratch = torch.empty_like(fields[0])
        slot = self.pools[req.fp32].add(fields, scratch, validate_stream=self.side)
        return dict(fields=fields, scratch=scratch, slot=slot, fp32=req.fp32)

    def launch(self, k):
        """Enqueues k steps of every non-empty pool; returns (event,
        {fp32: error}) for the pools whose step could not be enqueued."""
        failed = {}
        for fp32, pool in self.pools.items():
            if pool.size:
                try:
                    pool.step(k)
                except _lib.MpdataError as e:
                    failed[fp32] = f"step: {e}"
        ev = torch.cuda.Event()
        ev.record(self.compute)
        return ev, failed

    def wait(self, ev):
        ev.synchronize()

    def result(self, handle):
        """The state of a member on the host."""
        return handle["fields"][0].cpu().numpy()

    def remove(self, handle):
        self.pools[handle["fp32"]].remove(handle["slot"])

    def close(self):
        for p in self.pools.values():
            p.close()


class Server:
    """Continuous batching of a :class:`Scheduler` over an executor (by
    default :class:`GpuExecutor`).

    A request that fails -- its fields refused when it joins, its pool's
    step not enqueued, or a result that is not finite or cannot be read back
    at retirement -- is retired as failed (``Done.error``): its slot and its
    budget are released and every other request carries on."""

    def __init__(self, budget_bytes: float, *, k_max: int = 8, keep_results=False,
                 device="cuda", nonos=True, executor=None):
        self.sched = Scheduler(budget_bytes, k_max)
        self.keep = keep_results
        self.ex = executor if executor is not None else GpuExecutor(device, nonos)
        self.stats = collections.Counter()

    def close(self):
        self.ex.close()

    def run(self, requests, *, realtime=True, log_every=0.0):
        """Serve ``requests``.  With ``realtime`` the arrivals are replayed
        against the wall clock; otherwise all requests are present at time 0
        (a saturation run).  Returns the list of :class:`Done` in completion
        order (failed requests included)."""
        sched, ex = self.sched, self.ex
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        members = {}           # rid -> dict(handle, admitted)
        done = []
        t0 = time.perf_counter()
        last_log = t0
        now = lambda: time.perf_counter() - t0

        def fail(req, admitted, why):
            self.stats["failed"] += 1
            done.append(Done(req.rid, req.arrival, admitted, now(), req.cells, req.steps,
                             req.fp32, None, why))

        def arrivals_and_admission():
            t = now() if realtime else float("inf")
            while pending and pending[0].arrival <= t:
                sched.arrive(pending.popleft())
            for req in sched.admit():
                try:
                    handle = ex.add(req)
                except Exception as e:       # refused: the others carry on
                    sched.drop(req.rid)
                    fail(req, now(), f"add: {e}")
                    continue
                if members:
                    self.stats["joined_busy"] += 1   # others are resident
                members[req.rid] = dict(handle=handle, admitted=now())

        def retire(req, why=None):
            m = members.pop(req.rid)
            out = None
            if why is None:
                try:
                    out = ex.result(m["handle"])
                    if not np.isfinite(out).all():
                        why = "result holds NaN or Inf"
                except Exception as e:
                    why = f"result: {e}"
            try:
                ex.remove(m["handle"])
            except Exception as e:
                why = why or f"remove: {e}"
            if why is not None:
                fail(req, m["admitted"], why)
            else:
                done.append(Done(req.rid, req.arrival, m["admitted"], now(), req.cells,
                                 req.steps, req.fp32, out if self.keep else None))

        while pending or not sched.idle:
            arrivals_and_admission()
            k, tick_members = sched.tick()
            if k == 0:
                if pending and realtime:
                    time.sleep(max(0.0, pending[0].arrival - now()))
                continue
            ev, failed = ex.launch(k)
            self.stats["ticks"] += 1
            self.stats["steps"] += k
            if failed:
                # members of a pool whose step was not enqueued leave as failed
                for rid in [r for r in tick_members if sched.reqs[r].fp32 in failed]:
                    req = sched.drop(rid)
                    retire(req, failed[req.fp32])
                tick_members = [r for r in tick_members if r in sched.left]
            arrivals_and_admission()          # newcomers join the next tick
            ex.wait(ev)
            for req in sched.advance(tick_members, k):
                retire(req)
            if log_every and time.perf_counter() - last_log > log_every:
                last_log = time.perf_counter()
                print(f"# serve t={now():.1f}s done={len(done)} members={len(members)} "
                      f"queued={len(sched.queue)} pending={len(pending)}", file=sys.stderr,
                      flush=True)
        self.elapsed = now()
        self.stats["admission_waits"] = sched.waits
        self.stats["peak_bytes"] = int(sched.peak)
        return done


def summarize(done, elapsed=None):
    """Latency percentiles and throughput of the requests served to the end
    (failed ones are counted apart)."""
    ok = [d for d in done if d.error is None]
    lat = np.array([d.finished - d.arrival for d in ok]) * 1e3
    cells = sum(d.cells * d.steps for d in ok)
    span = elapsed if elapsed is not None else (max(d.finished for d in done) -
                                                min(d.arrival for d in done))
    return {"requests": len(ok), "failed": len(done) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "cell_updates": cells, "seconds": span,
            "cell_updates_per_s": cells / span}
