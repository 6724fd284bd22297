"""Continuous-batching scheduler logic on the CPU, driven by a fake executor
with a simulated clock (no device work)."""
import collections

import numpy as np
import pytest

from paper_1507_01265_amd.inputs import Request, served_requests
from paper_1507_01265_amd.serve import Scheduler, request_bytes


def simulate(reqs, budget, k_max, step_time):
    """Event loop of the server with a simulated clock: a tick of k steps over
    members of total cells C takes k * step_time(C) seconds."""
    sched = Scheduler(budget, k_max)
    pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
    t = 0.0
    progress = collections.Counter()
    finished_at = {}
    ticks = 0
    while pending or not sched.idle:
        while pending and pending[0].arrival <= t:
            sched.arrive(pending.popleft())
        sched.admit()
        assert sched.used <= sched.budget
        k, members = sched.tick()
        if k == 0:
            t = pending[0].arrival
            continue
        cells = sum(sched.reqs[r].cells for r in members)
        t += k * step_time(cells)
        ticks += 1
        for r in members:
            progress[r] += k
        for req in sched.advance(members, k):
            finished_at[req.rid] = t
    return finished_at, progress, ticks, sched


def test_every_request_gets_exactly_its_steps():
    reqs = served_requests(rate=200, duration=2.0, seed=5000)
    fin, progress, ticks, sched = simulate(reqs, 200e9, 8, lambda c: 1e-9 * c + 20e-6)
    assert len(fin) == len(reqs)
    for r in reqs:
        assert progress[r.rid] == r.steps
        assert fin[r.rid] >= r.arrival
    assert sched.used == 0


def test_budget_is_never_exceeded_and_queueing_happens():
    reqs = served_requests(rate=200, duration=1.0, seed=5001)
    big = max(request_bytes(r) for r in reqs)
    budget = 3 * big
    fin, progress, ticks, sched = simulate(reqs, budget, 8, lambda c: 2e-9 * c + 20e-6)
    assert len(fin) == len(reqs)
    assert sched.peak <= budget
    assert sched.waits > 0


def test_fifo_admission_order():
    mk = lambda i, t, n: Request(i, t, (8, 32, 32), n, True, 1, i)
    reqs = [mk(0, 0.0, 50), mk(1, 0.0, 10), mk(2, 0.0, 10)]
    budget = request_bytes(reqs[0])   # one at a time
    fin, progress, ticks, sched = simulate(reqs, budget, 8, lambda c: 1e-6)
    assert fin[0] < fin[1] < fin[2]


def test_ticks_never_overshoot_and_newcomers_join():
    mk = lambda i, t, n: Request(i, t, (8, 16, 16), n, False, 1, i)
    reqs = [mk(0, 0.0, 13), mk(1, 1e-6, 3), mk(2, 2e-6, 20)]
    fin, progress, ticks, sched = simulate(reqs, 1e12, 8, lambda c: 1e-6)
    assert [progress[i] for i in range(3)] == [13, 3, 20]
    # request 1 (3 steps) joins while 0 is running and finishes first
    assert fin[1] < fin[0] < fin[2]


def test_oversized_request_is_refused():
    r = Request(0, 0.0, (64, 256, 256), 10, False, 1, 0)
    with pytest.raises(ValueError):
        Scheduler(request_bytes(r) - 1).arrive(r)


def test_served_workload_recipe():
    reqs = served_requests(rate=200, duration=60.0, seed=5000)
    assert 11000 < len(reqs) < 13000
    fp32 = np.mean([r.fp32 for r in reqs])
    assert 0.66 < fp32 < 0.74
    steps = [r.steps for r in reqs]
    assert min(steps) >= 10 and max(steps) <= 200
    dims = np.array([r.shape for r in reqs])
    assert dims[:, 0].min() >= 16 and dims[:, 0].max() <= 64
    assert dims[:, 1:].min() >= 32 and dims[:, 1:].max() <= 256


# ------------------------------------------------ failure path of the server

class FakeExecutor:
    """Executor of the server on the CPU: a member's state is its step count.
    Raises on add for the rids in bad_add, returns a non-finite result for
    the rids in bad_result and refuses the step of one precision at tick
    number bad_tick."""

    def __init__(self, bad_add=(), bad_result=(), bad_tick=None, bad_fp32=True):
        self.bad_add, self.bad_result = set(bad_add), set(bad_result)
        self.bad_tick, self.bad_fp32 = bad_tick, bad_fp32
        self.members = {}
        self.ticks = 0
        self.removed = []

    def add(self, req):
        if req.rid in self.bad_add:
            raise ValueError("h must be finite and > 0")
        self.members[req.rid] = {"rid": req.rid, "fp32": req.fp32, "steps": 0}
        return self.members[req.rid]

    def launch(self, k):
        self.ticks += 1
        failed = {}
        for fp32 in (True, False):
            if self.ticks == self.bad_tick and fp32 == self.bad_fp32:
                failed[fp32] = "step: launch refused"
                continue
            for m in self.members.values():
                if m["fp32"] == fp32:
                    m["steps"] += k
        return None, failed

    def wait(self, ev):
        pass

    def result(self, h):
        out = np.full(4, float(h["steps"]))
        if h["rid"] in self.bad_result:
            out[1] = np.nan
        return out

    def remove(self, h):
        self.removed.append(h["rid"])
        del self.members[h["rid"]]

    def close(self):
        pass


def _serve_fake(reqs, ex, budget=1e12):
    from paper_1507_01265_amd.serve import Server
    srv = Server(budget, keep_results=True, executor=ex)
    done = srv.run(reqs, realtime=False)
    return {d.rid: d for d in done}, srv


def _mixed_reqs(n):
    return [Request(i, 0.0, (4, 8, 8), 5 + 3 * i, i % 2 == 0, 1, i) for i in range(n)]


def test_failed_admission_and_result_release_their_slot_and_budget():
    reqs = _mixed_reqs(8)
    ex = FakeExecutor(bad_add={2}, bad_result={5})
    done, srv = _serve_fake(reqs, ex, budget=3 * request_bytes(reqs[0]))
    assert set(done) == {r.rid for r in reqs}          # every request is retired
    assert "add" in done[2].error and done[2].result is None
    assert "NaN" in done[5].error and done[5].result is None
    for r in reqs:
        if r.rid not in (2, 5):
            assert done[r.rid].error is None
            assert done[r.rid].result[0] == r.steps      # exactly its steps
    assert srv.sched.used == 0 and srv.sched.idle
    assert not ex.members                                # every slot released
    assert 5 in ex.removed and 2 not in ex.removed
    assert srv.stats["failed"] == 2


def test_failed_step_retires_that_pool_only():
    reqs = _mixed_reqs(6)
    ex = FakeExecutor(bad_tick=2, bad_fp32=True)
    done, srv = _serve_fake(reqs, ex)
    fp32 = {r.rid for r in reqs if r.fp32}
    # the FP32 members present at the second tick fail, the FP64 ones finish
    failed = {rid for rid, d in done.items() if d.error is not None}
    assert failed and failed <= fp32
    assert all("launch refused" in done[r].error for r in failed)
    for r in reqs:
        if not r.fp32:
            assert done[r.rid].error is None and done[r.rid].result[0] == r.steps
    assert srv.sched.used == 0 and not ex.members


def test_summary_counts_failures_apart():
    from paper_1507_01265_amd.serve import Done, summarize
    done = [Done(0, 0.0, 0.0, 0.010, 100, 10, True),
            Done(1, 0.0, 0.0, 0.020, 100, 10, True),
            Done(2, 0.0, 0.0, 0.001, 100, 10, True, None, "add: refused")]
    s = summarize(done, 1.0)
    assert s["requests"] == 2 and s["failed"] == 1
    assert s["cell_updates"] == 2000
