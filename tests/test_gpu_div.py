"""The divergent-flow term (MPDATA_FLAG_DIV) on the GPU against the oracle.

random_smooth draws independent face Courant numbers, so its flows are
divergent and the term is active.  Bars as for the plain step
(tests/bars.py): FP64 rel-Linf <= 1e-12; FP32 rel-Linf <= 1e-5 and rel-L2
<= 2e-6.
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


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
@pytest.mark.parametrize("nonos", [True, False], ids=["nonos", "unlimited"])
def test_parity_fp64(orc, bc, nonos):
    """70x45x13 ragged, variable h, divergent random Courant numbers, 4 steps;
    the term changes the result (checked against the oracle without it)."""
    f = inputs.random_smooth(301, (13, 45, 70), bc=bc, cmax=0.15)
    print(f"div bc {bc} nonos {nonos}", flush=True)
    want = oracle_run(orc, f, 4, nonos=nonos, div=True)
    got = gpu_run(f, 4, nonos=nonos, div=True)
    assert rel_linf(got, want) <= 1e-12
    assert rel_linf(oracle_run(orc, f, 4, nonos=nonos), want) > 1e-6


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_parity_fp32(orc, bc):
    f = inputs.random_smooth(302, (13, 45, 70), bc=bc, cmax=0.15).astype(np.float32)
    n = 4
    want = oracle_run(orc, f.as_f64(), n, div=True)
    got = gpu_run(f, n, dtype=torch.float32, div=True)
    check_fp32(got, want, f"div bc {bc}")


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
@pytest.mark.parametrize("iord", [3, 4])
def test_parity_with_more_passes(orc, bc, iord):
    """In a later pass the term acts on the divergence of the previous
    pass's antidiffusive velocity."""
    f = inputs.random_smooth(303, (13, 45, 70), bc=bc, cmax=0.15)
    want = oracle_run(orc, f, 3, iord=iord, div=True)
    got = gpu_run(f, 3, iord=iord, div=True)
    assert rel_linf(got, want) <= 1e-12


def test_parity_with_variable_sign(orc):
    f = inputs.random_smooth(304, (13, 45, 70), cmax=0.15)
    f = dataclasses.replace(f, psi=f.psi - 1.0)
    want = oracle_run(orc, f, 3, div=True, vsign=True)
    got = gpu_run(f, 3, div=True, vsign=True)
    assert rel_linf(got, want) <= 1e-12


@pytest.mark.parametrize("kind", ["rotation", "streamfunction"])
def test_term_vanishes_on_solenoidal_flows(kind):
    """Discretely divergence-free Courant numbers: every cell divergence is an
    exact zero, so the result is bitwise that of the plain step."""
    if kind == "rotation":
        f = inputs.rotation(seed=7, shape=(12, 40, 56))
    else:
        f = inputs.random_smooth(305, (12, 40, 56), bc=1, divergence_free=True, cmax=0.4)
    np.testing.assert_array_equal(gpu_run(f, 3, div=True), gpu_run(f, 3))


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 40), (1, 33, 1), (29, 1, 1)])
def test_degenerate_shapes(orc, shape):
    f = inputs.random_smooth(306, shape, cmax=0.15)
    want = oracle_run(orc, f, 3, div=True)
    got = gpu_run(f, 3, div=True)
    assert rel_linf(got, want) <= 1e-12


def test_flag_needs_a_default_launch_shape():
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(307, (8, 16, 16))
    with pytest.raises((_lib.MpdataError, ValueError)):
        gpu_run(f, 1, tile=4, div=True)


@pytest.mark.slow
def test_full_size_divergent_fp64(orc):
    """512x256x64 with divergent random Courant numbers, 2 steps."""
    f = inputs.random_smooth(308, (64, 256, 512), cmax=0.15)
    want = oracle_run(orc, f, 2, div=True)
    got = gpu_run(f, 2, div=True)
    assert rel_linf(got, want) <= 1e-12


def test_parity_benchmark_flow(orc):
    """The benchmark's divergent rotation flow at 128x64x16, 4 steps."""
    f = inputs.divergent_rotation(shape=(16, 64, 128))
    want = oracle_run(orc, f, 4, div=True)
    got = gpu_run(f, 4, div=True)
    assert rel_linf(got, want) <= 1e-12
