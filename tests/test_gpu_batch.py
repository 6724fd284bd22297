"""Batches of uneven grids (one persistent launch per step) against the
oracle and against the single-grid path, plus the plan checks."""
import numpy as np
import pytest

from paper_1507_01265_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _grids(n, seed, dtype=np.float64, bc=0):
    out = []
    rng = np.random.default_rng(seed)
    for g in range(n):
        shape = (int(rng.integers(1, 20)), int(rng.integers(1, 70)), int(rng.integers(1, 90)))
        out.append(inputs.random_smooth(seed + g, shape, bc=bc, cmax=0.15).astype(dtype))
    return out


def _single(f, steps, dtype):
    from paper_1507_01265_amd.solver import Solver
    s = Solver.from_numpy(f, dtype=dtype)
    s.step(steps)
    s.sync()
    out = s.psi.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_batch_matches_oracle_and_single_grid(orc, bc):
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(7, 300, bc=bc)
    b = Batch.from_numpy(fs, dtype=torch.float64, bc=bc)
    b.step(5)
    b.sync()
    for i, f in enumerate(fs):
        got = b.psi(i).cpu().numpy()
        want = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 5, bc=bc)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), i
        np.testing.assert_array_equal(got, _single(f, 5, torch.float64))
    b.close()


def test_batch_fp32_every_tile_same_bits():
    from paper_1507_01265_amd import _lib
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(5, 400, dtype=np.float32)
    ref = [_single(f, 3, torch.float32) for f in fs]
    for tile in range(1, _lib.mpdata_tile_count() + 1):
        b = Batch.from_numpy(fs, dtype=torch.float32, tile=tile)
        b.step(3)
        b.sync()
        for i in range(len(fs)):
            np.testing.assert_array_equal(b.psi(i).cpu().numpy(), ref[i])
        b.close()


def test_custom_plan_and_profile():
    """A tuner-style plan (LPT over whole tiles) gives the same bits as the
    default plan, and per-segment timing returns one positive value each."""
    from paper_1507_01265_amd import autotune
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(6, 500, dtype=np.float32)
    ref = [_single(f, 4, torch.float32) for f in fs]
    tile = 5
    segs = autotune.whole_tile_segments([f.psi.shape for f in fs], tile)
    owner, _ = autotune.lpt(segs[:, 4] - segs[:, 3] + 4, 37)
    plan = (tile, *autotune.plan_from_owner(segs, owner, 37))
    b = Batch.from_numpy(fs, dtype=torch.float32, plan=plan)
    ticks = b.profile_step()
    assert ticks.shape == (len(segs),) and (ticks > 0).all()
    b.step(3)
    b.sync()
    for i in range(len(fs)):
        np.testing.assert_array_equal(b.psi(i).cpu().numpy(), ref[i])
    b.close()


def test_plan_validation():
    from paper_1507_01265_amd import _lib, autotune
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(3, 600, dtype=np.float32)
    tile = 5
    segs = autotune.whole_tile_segments([f.psi.shape for f in fs], tile)
    bad = segs[:-1]                                  # one tile left out
    with pytest.raises(_lib.MpdataError, match="not covered"):
        Batch.from_numpy(fs, dtype=torch.float32, plan=(tile, bad, np.array([0, len(bad)])))
    dup = np.concatenate([segs, segs[:1]])            # one tile twice
    with pytest.raises(_lib.MpdataError, match="twice"):
        Batch.from_numpy(fs, dtype=torch.float32, plan=(tile, dup, np.array([0, len(dup)])))


def test_mixed_batch_is_rejected():
    from paper_1507_01265_amd import _lib
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(2, 700)
    g = [tuple(torch.from_numpy(a).cuda() for a in (f.psi, f.u1, f.u2, f.u3, f.h)) for f in fs]
    g[1] = tuple(t.float() for t in g[1])
    with pytest.raises(ValueError):
        Batch(g)


def test_graph_and_plain_launches_agree():
    from paper_1507_01265_amd.solver import Solver
    f = inputs.random_smooth(801, (10, 40, 60), cmax=0.15)
    outs = []
    for graph in (True, False):
        s = Solver.from_numpy(f, graph=graph)
        s.step(19)                                  # 2 graph replays + 3 launches
        s.sync()
        outs.append(s.psi.cpu().numpy())
        s.close()
    np.testing.assert_array_equal(outs[0], outs[1])


def test_autotune_small_batch():
    from paper_1507_01265_amd import autotune
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(8, 900, dtype=np.float32)
    g = [tuple(torch.from_numpy(a).cuda() for a in (f.psi, f.u1, f.u2, f.u3, f.h)) for f in fs]
    before = [x[0].clone() for x in g]
    tuned = autotune.tune(g, tiles=[2, 5], steps=2, profiles=2)
    for x, y in zip(g, before):
        assert torch.equal(x[0], y)
    b = Batch(g, plan=tuned.plan)
    b.step(2)
    b.sync()
    for i, f in enumerate(fs):
        np.testing.assert_array_equal(b.psi(i).cpu().numpy(), _single(f, 2, torch.float32))
    b.close()


@pytest.mark.parametrize("opts", [dict(div=True), dict(vsign=True, div=True)])
def test_batch_with_options_matches_single_grid(orc, opts):
    """The variable-sign option and the divergent-flow term in a batch (one
    launch for all grids) equal the single-grid path bit for bit and the
    oracle to 1e-12; the tuner keeps to the shapes built for them."""
    import dataclasses
    from paper_1507_01265_amd import autotune
    from paper_1507_01265_amd.batch import Batch
    from paper_1507_01265_amd.solver import Solver
    fs = _grids(5, 950)
    if opts.get("vsign"):
        fs = [dataclasses.replace(f, psi=f.psi - 1.0) for f in fs]
    g = [tuple(torch.from_numpy(a).cuda() for a in (f.psi, f.u1, f.u2, f.u3, f.h)) for f in fs]
    tuned = autotune.tune(g, steps=1, profiles=1, **opts)
    assert tuned.plan[0] in autotune.option_tiles()
    b = Batch(g, plan=tuned.plan, **opts)
    b.step(3)
    b.sync()
    for i, f in enumerate(fs):
        got = b.psi(i).cpu().numpy()
        s = Solver.from_numpy(f, dtype=torch.float64, **opts)
        s.step(3)
        s.sync()
        np.testing.assert_array_equal(got, s.psi.cpu().numpy())
        s.close()
        want = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 3, **opts)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), i
    b.close()


def test_mixed_shapes_in_one_launch_same_bits():
    """Per-grid launch shapes in one persistent launch (32x24 and 24x32
    regions, a sixth plan column): every grid equals its single-grid run bit
    for bit, whichever shape it takes; a grid whose segments name two shapes,
    or a shape outside the family, is rejected."""
    from paper_1507_01265_amd import _lib, autotune
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(6, 1200, dtype=np.float32)
    ref = [_single(f, 3, torch.float32) for f in fs]
    shapes = [f.psi.shape for f in fs]
    for choice in ([5, 7, 5, 7, 7, 5], [7] * 6):
        segs = autotune.mixed_segments(shapes, choice)
        owner, _ = autotune.lpt(segs[:, 4] - segs[:, 3], 41)
        plan = (5, *autotune.plan_from_owner(segs, owner, 41))
        b = Batch.from_numpy(fs, dtype=torch.float32, plan=plan)
        b.step(3)
        b.sync()
        for i in range(len(fs)):
            np.testing.assert_array_equal(b.psi(i).cpu().numpy(), ref[i])
        ticks = b.profile_step()
        assert len(ticks) == len(segs) and (ticks > 0).all()
        b.close()
    segs = autotune.mixed_segments(shapes, [5] * 6)
    bad = segs.copy()
    bad[0, 5] = 7  # grid 0 in two shapes
    with pytest.raises(_lib.MpdataError):
        Batch.from_numpy(fs, dtype=torch.float32, plan=(5, bad, np.array([0, len(bad)])))
    bad = segs.copy()
    bad[:, 5] = 2  # not a shape of the family
    with pytest.raises(_lib.MpdataError):
        Batch.from_numpy(fs, dtype=torch.float32, plan=(5, bad, np.array([0, len(bad)])))
    with pytest.raises(_lib.MpdataError):  # FP64 has no mixed launch
        Batch.from_numpy(_grids(6, 1200), dtype=torch.float64, plan=(5, segs, np.array([0, len(segs)])))


def test_autotune_per_grid_shapes():
    """With both 768-thread regions measured, the tuner also times the mixed
    plan; whichever plan wins gives the single-grid bits."""
    from paper_1507_01265_amd import autotune
    from paper_1507_01265_amd.batch import Batch
    fs = _grids(8, 1300, dtype=np.float32)
    g = [tuple(torch.from_numpy(a).cuda() for a in (f.psi, f.u1, f.u2, f.u3, f.h)) for f in fs]
    tuned = autotune.tune(g, tiles=[5, 7], steps=2, profiles=2)
    assert any(e["tile"] == "mixed" for e in tuned.log)
    b = Batch(g, plan=tuned.plan)
    b.step(2)
    b.sync()
    for i, f in enumerate(fs):
        np.testing.assert_array_equal(b.psi(i).cpu().numpy(), _single(f, 2, torch.float32))
    b.close()
