"""XCD-team slab plans on the GPU: any split computes the same step as the
single-grid path, and the per-team timing is well formed."""
import numpy as np
import pytest
import torch

from paper_1507_01265_amd import inputs, teams
from paper_1507_01265_amd.batch import Batch
from paper_1507_01265_amd.solver import Solver

pytestmark = pytest.mark.gpu


def _make(nz):
    return inputs.rotation(shape=(nz, 64, 96))


@pytest.mark.parametrize("split", [(2, 2), (3, 1), (4, 0)])
def test_slab_plans_match_single_grid_bitwise(split):
    f = _make(32)
    hi, lo = split
    slabs = teams.split_slabs(hi * 2, lo * 2) if lo else \
        [(0, 8), (8, 16), (16, 16), (16, 24), (24, 24), (24, 32), (32, 32), (32, 32)]
    grid = teams._grid(f, torch.float64)
    nwg = teams._occupancy_nwg(torch.float64, 5, f.bc)
    plan = teams.slab_plan(f.psi.shape, 5, nwg, slabs)
    b = Batch([grid], plan=plan)
    b.step(3)
    b.sync()
    got = grid[0].cpu().numpy()
    b.close()
    s = Solver.from_numpy(f, dtype=torch.float64, tile=5)
    s.step(3)
    s.sync()
    want = s.psi.cpu().numpy()
    s.close()
    assert np.array_equal(got, want)


def test_team_times_and_speed_function_are_positive():
    sf = teams.speed_function(_make, [1, 2], torch.float64, 5, profiles=2)
    for m, (mean, per_team) in sf.items():
        assert mean > 0 and len(per_team) == teams.XCDS and min(per_team) > 0
