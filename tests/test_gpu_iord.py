"""More than one corrective pass (iord > 2) on the GPU against the oracle.

The step is a chain of launches (the fused step, then one launch per further
pass); these tests run it through the C ABI.  Bars as for one corrective
pass (tests/bars.py): FP64 rel-Linf <= 1e-12; FP32 rel-Linf <= 1e-5 and
rel-L2 <= 2e-6.
"""
import dataclasses

import numpy as np
import pytest
from bars import check_fp32

from paper_1507_01265_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1507_01265_amd import _lib
    _lib.load()


def gpu_run(fields, steps, dtype=torch.float64, **kw):
    from paper_1507_01265_amd.solver import Solver
    s = Solver.from_numpy(fields, dtype=dtype, **kw)
    s.step(steps)
    s.sync()
    out = s.psi.cpu().numpy().astype(np.float64)
    s.close()
    return out


def oracle_run(orc, f, steps, **kw):
    return orc.run(f.psi, f.u1, f.u2, f.u3, f.h, steps, bc=f.bc, **kw)


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.mark.parametrize("iord", [3, 4, 5])
@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
@pytest.mark.parametrize("nonos", [True, False], ids=["nonos", "unlimited"])
def test_parity_fp64(orc, iord, bc, nonos):
    """70x45x13 (ragged tiles on every axis), variable h, random Courant
    numbers, 3 steps (both step parities and the final copy back); iord 4
    and 5 run one and two middle passes (both buffer sets)."""
    f = inputs.random_smooth(201, (13, 45, 70), bc=bc, cmax=0.15)
    print(f"iord {iord} bc {bc} nonos {nonos}", flush=True)
    want = oracle_run(orc, f, 3, iord=iord, nonos=nonos)
    got = gpu_run(f, 3, iord=iord, nonos=nonos)
    err = rel_linf(got, want)
    print(f"  rel-Linf {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_parity_fp32(orc, bc):
    f = inputs.random_smooth(202, (13, 45, 70), bc=bc, cmax=0.15).astype(np.float32)
    n, iord = 4, 3
    want = oracle_run(orc, f.as_f64(), n, iord=iord)
    got = gpu_run(f, n, dtype=torch.float32, iord=iord)
    check_fp32(got, want, f"iord {iord} bc {bc}")


@pytest.mark.parametrize("nonos", [True, False], ids=["nonos", "unlimited"])
def test_parity_variable_sign(orc, nonos):
    f = inputs.random_smooth(203, (13, 45, 70))
    f = dataclasses.replace(f, psi=f.psi - 1.0)
    assert f.psi.min() < 0.0 < f.psi.max()
    want = oracle_run(orc, f, 3, iord=3, nonos=nonos, vsign=True)
    got = gpu_run(f, 3, iord=3, nonos=nonos, vsign=True)
    assert rel_linf(got, want) <= 1e-12


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 40), (1, 33, 1), (29, 1, 1), (1, 20, 35)])
@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_degenerate_shapes(orc, shape, bc):
    f = inputs.random_smooth(204, shape, bc=bc, cmax=0.15)
    want = oracle_run(orc, f, 3, iord=4)
    got = gpu_run(f, 3, iord=4)
    assert rel_linf(got, want) <= 1e-12


def test_courant_one_shift_bitwise():
    """|C| = 1 along x: every pass after the first has a zero velocity
    field, so the step is an exact one-cell roll."""
    rng = np.random.default_rng(205)
    shape = (9, 30, 37)
    psi = rng.uniform(1.0, 2.0, shape)
    u1, u2, u3 = inputs.constant_courant(shape, (1.0, 0.0, 0.0))
    f = inputs.Fields(psi=psi, u1=u1, u2=u2, u3=u3, h=np.ones(shape), bc=0)
    got = gpu_run(f, 2, iord=3)
    np.testing.assert_array_equal(got, np.roll(psi, 2, axis=2))


def test_constant_field_and_mass():
    """psi = 1 under solid-body rotation stays 1 bit for bit; a smooth field
    keeps its mass to rounding."""
    f = inputs.rotation(seed=6, shape=(12, 40, 56))
    ones = dataclasses.replace(f, psi=np.ones_like(f.psi))
    np.testing.assert_array_equal(gpu_run(ones, 2, iord=4), ones.psi)
    from paper_1507_01265_amd.solver import Solver
    g = inputs.random_smooth(206, (12, 40, 56), cmax=0.15)
    s = Solver.from_numpy(g, dtype=torch.float64, iord=3)
    m0 = s.mass()
    s.step(5)
    m1 = s.mass()
    s.close()
    assert abs(m1 - m0) / m0 < 1e-13


def test_iord_needs_the_default_launch_shape():
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(207, (8, 16, 16))
    with pytest.raises((_lib.MpdataError, ValueError)):
        gpu_run(f, 1, iord=3, tile=4)


@pytest.mark.slow
def test_full_size_rotation_fp64(orc):
    """512x256x64 rotation, iord 3, 2 steps."""
    f = inputs.rotation()
    want = oracle_run(orc, f, 2, iord=3)
    got = gpu_run(f, 2, iord=3)
    assert rel_linf(got, want) <= 1e-12
    assert got.min() >= -1e-15


@pytest.mark.parametrize("iord", [3, 4])
def test_graph_and_plain_launches_agree(iord):
    """19 steps: two replays of the 8-step graph of pass chains plus three
    plain steps, against 19 plain steps -- bit for bit."""
    f = inputs.random_smooth(208, (13, 45, 70), cmax=0.15)
    a = gpu_run(f, 19, iord=iord)
    b = gpu_run(f, 19, iord=iord, graph=False)
    np.testing.assert_array_equal(a, b)
