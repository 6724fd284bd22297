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
