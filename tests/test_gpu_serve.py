"""Serving: continuous batching gives each request the same bits as serving
it alone, matches the oracle, and respects the HBM budget."""
import numpy as np
import pytest
from bars import FP32_LINF, FP64_LINF

from paper_1507_01265_amd.inputs import Request, rotation_request_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        shape = (int(rng.integers(4, 24)), int(rng.integers(8, 80)), int(rng.integers(8, 80)))
        out.append(Request(i, float(i) * 1e-3, shape, int(rng.integers(1, 30)),
                           bool(rng.uniform() < 0.6), 1 if rng.uniform() < 0.5 else -1,
                           int(rng.integers(0, 2 ** 31))))
    return out


def _serve(reqs, budget=1e12, realtime=False):
    from paper_1507_01265_amd.serve import Server
    srv = Server(budget, keep_results=True)
    done = srv.run(reqs, realtime=realtime)
    stats = dict(srv.stats)
    srv.close()
    return {d.rid: d for d in done}, stats


def test_alone_equals_in_mix():
    reqs = _requests(16, 1)
    mix, stats = _serve(reqs)
    assert len(mix) == len(reqs) and stats["ticks"] > 1
    for r in reqs:
        alone, _ = _serve([Request(r.rid, 0.0, r.shape, r.steps, r.fp32, r.sense, r.field_seed)])
        np.testing.assert_array_equal(mix[r.rid].result, alone[r.rid].result)


def test_served_results_match_oracle(orc):
    reqs = _requests(6, 2)
    mix, _ = _serve(reqs)
    for r in reqs:
        psi, u1, u2, u3, h = [t.double().cpu().numpy() for t in rotation_request_device(r)]
        want = orc.run(psi, u1, u2, u3, h, r.steps)
        got = mix[r.rid].result.astype(np.float64)
        tol = FP32_LINF if r.fp32 else FP64_LINF
        assert np.abs(got - want).max() <= tol * np.abs(want).max(), r


def test_small_budget_queues_but_completes():
    from paper_1507_01265_amd.serve import request_bytes
    reqs = _requests(12, 3)
    budget = 2 * max(request_bytes(r) for r in reqs)
    mix, stats = _serve(reqs, budget=budget)
    assert len(mix) == len(reqs)
    assert stats["peak_bytes"] <= budget
    assert stats["admission_waits"] > 0


def test_realtime_arrivals():
    reqs = _requests(10, 4)
    for i, r in enumerate(reqs):
        r.arrival = 0.005 * i
    mix, stats = _serve(reqs, realtime=True)
    assert len(mix) == len(reqs)
    for r in reqs:
        assert mix[r.rid].finished >= r.arrival


def test_late_joiners_equal_alone_and_match_oracle(orc):
    """A budget of two of the largest requests: most requests join a pool
    while others are resident and mid-run (the plan is uploaded again under
    the already-built replay graph of 8 steps; every request runs >= 8
    steps).  Each result equals the request served alone, bit for bit, and
    the oracle within the precision's bar."""
    from paper_1507_01265_amd.serve import request_bytes
    rng = np.random.default_rng(7)
    reqs = []
    for i in range(10):
        shape = (int(rng.integers(4, 20)), int(rng.integers(8, 64)), int(rng.integers(8, 64)))
        reqs.append(Request(i, 0.0, shape, int(rng.integers(8, 41)), i % 3 != 0,
                            1 if i % 2 else -1, int(rng.integers(0, 2 ** 31))))
    budget = 2 * max(request_bytes(r) for r in reqs)
    mix, stats = _serve(reqs, budget=budget)
    assert len(mix) == len(reqs) and all(d.error is None for d in mix.values())
    assert stats["admission_waits"] > 0 and stats["joined_busy"] >= 3
    for r in reqs:
        alone, _ = _serve([Request(r.rid, 0.0, r.shape, r.steps, r.fp32, r.sense, r.field_seed)])
        np.testing.assert_array_equal(mix[r.rid].result, alone[r.rid].result)
        psi, u1, u2, u3, h = [t.double().cpu().numpy() for t in rotation_request_device(r)]
        want = orc.run(psi, u1, u2, u3, h, r.steps)
        got = mix[r.rid].result.astype(np.float64)
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= (FP32_LINF if r.fp32 else FP64_LINF), (r, err)
