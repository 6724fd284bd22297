"""Host logic of the batch tuner: segments, LPT and the placements it times
(no GPU)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1507_01265_amd import autotune  # noqa: E402


def _shapes():
    rng = np.random.default_rng(7)
    return [(int(rng.integers(16, 65)), int(rng.integers(32, 385)), int(rng.integers(32, 385)))
            for _ in range(40)]


def test_whole_tile_segments_cover_every_tile_once():
    shapes = _shapes()
    for tile in (2, 5):
        segs = autotune.whole_tile_segments(shapes, tile)
        for g, shp in enumerate(shapes):
            ntx, nty = autotune.tiles_of(shp, tile)
            mine = segs[segs[:, 0] == g]
            assert len(mine) == ntx * nty
            assert len({(r[1], r[2]) for r in mine.tolist()}) == ntx * nty
            assert (mine[:, 3] == 0).all() and (mine[:, 4] == shp[0]).all()


def test_lpt_is_within_the_greedy_bound():
    rng = np.random.default_rng(3)
    costs = rng.uniform(1, 10, 500)
    owner, loads = autotune.lpt(costs, 37)
    assert np.allclose(np.bincount(owner, weights=costs, minlength=37), loads)
    # greedy list scheduling: makespan <= mean load + largest item; LPT
    # also within 4/3 of the lower bound max(mean, largest item) here
    assert loads.max() <= costs.sum() / 37 + costs.max()
    assert loads.max() <= 4 / 3 * max(costs.sum() / 37, costs.max())


def test_xcd_affine_keeps_each_grid_on_one_xcd():
    shapes = _shapes()
    segs = autotune.whole_tile_segments(shapes, 5)
    cost = (segs[:, 4] - segs[:, 3] + autotune.PRIMING).astype(float)
    nwg = 256
    owner = autotune.xcd_affine(segs, cost, nwg, len(shapes))
    assert owner.min() >= 0 and owner.max() < nwg
    for g in range(len(shapes)):
        assert len(set((owner[segs[:, 0] == g] % autotune.XCDS).tolist())) == 1
    # the XCDs carry about the same work (LPT over whole grids)
    per_xcd = np.bincount(owner % autotune.XCDS, weights=cost, minlength=autotune.XCDS)
    assert per_xcd.max() <= per_xcd.mean() + max(np.bincount(segs[:, 0], weights=cost))
    seg, wg_begin = autotune.plan_from_owner(segs, owner, nwg)
    assert len(seg) == len(segs) and wg_begin[0] == 0 and wg_begin[-1] == len(segs)
    assert (np.diff(wg_begin) >= 0).all()


def test_mixed_segments_name_one_shape_per_grid():
    shapes = _shapes()
    choice = [autotune.MIXED_TILES[g % 2] for g in range(len(shapes))]
    segs = autotune.mixed_segments(shapes, choice)
    assert segs.shape[1] == 6
    for g, t in enumerate(choice):
        mine = segs[segs[:, 0] == g]
        assert (mine[:, 5] == t).all()
        ntx, nty = autotune.tiles_of(shapes[g], t)
        assert len(mine) == ntx * nty
