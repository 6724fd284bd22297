"""Slab plans of the XCD-team experiment (host logic, no GPU)."""
import numpy as np
import pytest

from paper_1507_01265_amd import teams


@pytest.mark.parametrize("slabs", [teams.even_slabs(64), teams.split_slabs(10, 6),
                                   teams.split_slabs(15, 1)])
def test_slab_plan_covers_every_tile_plane_once_within_teams(slabs):
    shape = (64, 256, 512)
    tile, seg, wg_begin = teams.slab_plan(shape, 5, 256, slabs)
    ntx, nty = teams.tiles_of(shape, tile)
    cover = np.zeros((nty, ntx, 64), dtype=int)
    for w in range(256):
        team = w % teams.XCDS
        for g, tx, ty, z0, z1 in seg[wg_begin[w]:wg_begin[w + 1]]:
            assert g == 0 and (z0, z1) == tuple(slabs[team])
            cover[ty, tx, z0:z1] += 1
    assert (cover == 1).all()


def test_split_slabs_alternate_and_sum():
    s = teams.split_slabs(11, 5)
    assert [z1 - z0 for z0, z1 in s] == [11, 5] * 4 and s[-1][1] == 64
    assert all(a[1] == b[0] for a, b in zip(s, s[1:]))


def test_team_seconds_takes_the_slowest_workgroup_per_team():
    wg_begin = np.arange(0, 17)            # 16 workgroups, one segment each
    ticks = np.arange(1, 17, dtype=float) * 1e6
    t = teams.team_seconds(ticks, wg_begin)
    # team i = workgroups i and i + 8: the later one is slower
    assert np.allclose(t, (np.arange(8) + 9) * 1e6 / teams.TICK_HZ)
