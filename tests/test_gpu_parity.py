"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

The bars (FP64 rel-Linf <= 1e-12; FP32 rel-Linf <= 1e-5 and rel-L2 <= 2e-6
against the FP64 oracle on the same FP32-rounded inputs, for runs of at most
100 steps) are stated and derived in tests/bars.py.
"""
import numpy as np
import pytest
from bars import FP32_DRIFT, check_fp32, check_fp64

from paper_1507_01265_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1507_01265_amd import _lib
    _lib.load()


def _solver(fields, dtype=torch.float64, **kw):
    from paper_1507_01265_amd.solver import Solver
    return Solver.from_numpy(fields, dtype=dtype, **kw)


def gpu_run(fields, steps, dtype=torch.float64, **kw):
    s = _solver(fields, dtype=dtype, **kw)
    s.step(steps)
    s.sync()
    out = s.psi.cpu().numpy().astype(np.float64)
    s.close()
    return out


def rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def oracle_run(orc, f, steps, **kw):
    return orc.run(f.psi, f.u1, f.u2, f.u3, f.h, steps, bc=f.bc, **kw)


# ------------------------------------------------------------------ FP64

def test_parity_small_config(orc):
    """32x32x16 periodic, constant Courant (0.3,0.2,0.1), 10 steps, limiter on."""
    f = inputs.parity_small()
    want = oracle_run(orc, f, 10)
    got = gpu_run(f, 10)
    err = rel_linf(got, want)
    print(f"parity_small rel-Linf {err:.3e} max|diff| {np.abs(got - want).max():.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
@pytest.mark.parametrize("nonos", [True, False], ids=["nonos", "unlimited"])
def test_parity_every_tile_ragged(orc, bc, nonos):
    """70x45x13 (several tiles and ragged tails on every axis), variable h,
    random face Courant numbers: every launch shape matches the oracle and
    all shapes agree bit for bit."""
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(101, (13, 45, 70), bc=bc, cmax=0.15)
    want = oracle_run(orc, f, 4, nonos=nonos)
    first = None
    for tile in range(1, _lib.mpdata_tile_count() + 1):
        if not _lib.mpdata_tile_built(_lib.MPDATA_FP64, tile):
            continue  # tile 7 (24x32) is built for FP32 only
        print(f"tile {tile} bc {bc} nonos {nonos}", flush=True)
        got = gpu_run(f, 4, nonos=nonos, tile=tile)
        assert rel_linf(got, want) <= 1e-12, (tile, rel_linf(got, want))
        if first is None:
            first = got
        else:
            np.testing.assert_array_equal(got, first)


@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_parity_divergence_free_with_zero_background(orc, bc):
    """Streamfunction flow on a zero background with a sharp block: exercises
    A = 0/eps, the limiter at zero bounds and the open-boundary budget."""
    f = inputs.random_smooth(103, (10, 40, 66), bc=bc, divergence_free=True, cmax=0.45)
    psi = np.zeros_like(f.psi)
    psi[2:8, 10:30, 20:50] = 1.0
    f.psi = psi
    want = oracle_run(orc, f, 6)
    got = gpu_run(f, 6)
    assert rel_linf(got, want) <= 1e-12
    assert got.min() >= -1e-15


def test_parity_donor_cell_only(orc):
    f = inputs.random_smooth(105, (9, 21, 37), cmax=0.15)
    for bc in (0, 1):
        f.bc = bc
        want = oracle_run(orc, f, 3, iord=1, nonos=False)
        got = gpu_run(f, 3, iord=1, nonos=False)
        assert rel_linf(got, want) <= 1e-12


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 9), (7, 1, 1), (1, 6, 1), (2, 5, 3),
                                   (3, 1, 66), (1, 17, 2), (5, 3, 61)])
@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_degenerate_shapes(orc, shape, bc):
    f = inputs.random_smooth(107, shape, bc=bc, cmax=0.15)
    want = oracle_run(orc, f, 3)
    got = gpu_run(f, 3)
    assert rel_linf(got, want) <= 1e-12


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 5, 3), (3, 1, 66), (4, 17, 9), (5, 30, 41),
                                   (6, 23, 33)])
@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_degenerate_shapes_fp32(orc, shape, bc):
    """FP32 marches run a segment's first two iterations and its last one
    reduced; columns of 1 to 6 planes take every arrangement of those
    iterations (the iteration count z1 - z0 + 5 in each residue mod 3), with
    the limiter and without it, against the oracle on the same FP32 inputs."""
    g = inputs.random_smooth(131 + shape[0], shape, bc=bc, cmax=0.15).astype(np.float32)
    for nonos in (True, False):
        want = oracle_run(orc, g.as_f64(), 3, nonos=nonos)
        got = gpu_run(g, 3, dtype=torch.float32, nonos=nonos)
        check_fp32(got, want, f"{shape} nonos={nonos}")


@pytest.mark.parametrize("steps", [0, 1, 3])
def test_step_counts(orc, steps):
    """Odd counts end with a copy from the workspace; 0 is a no-op."""
    f = inputs.random_smooth(109, (6, 12, 20), cmax=0.15)
    want = oracle_run(orc, f, steps)
    got = gpu_run(f, steps)
    assert rel_linf(got, want) <= 1e-12


def test_courant_one_shift_is_exact():
    f = inputs.random_smooth(111, (5, 9, 13))
    f.psi = 1.0 + np.random.default_rng(1).uniform(0, 1, f.psi.shape) * 0.999
    f.u1, f.u2, f.u3 = inputs.constant_courant(f.psi.shape, (1.0, 0.0, 0.0))
    f.h = np.ones_like(f.psi)
    got = gpu_run(f, 1)
    np.testing.assert_array_equal(got, np.roll(f.psi, 1, axis=2))


def test_constant_field_preserved():
    f = inputs.random_smooth(113, (8, 30, 40), divergence_free=True, cmax=0.45)
    f.psi = np.ones_like(f.psi)
    got = gpu_run(f, 5)
    np.testing.assert_array_equal(got, f.psi)


# ------------------------------------------------------------------ mass

def test_mass_matches_oracle(orc):
    f = inputs.random_smooth(115, (16, 40, 72), cmax=0.15)
    s = _solver(f)
    m0 = s.mass()
    assert abs(m0 - orc.mass(f.psi, f.h)) <= 2e-16 * abs(m0)
    s.step(6)
    m1 = s.mass()
    want = orc.mass(s.psi.cpu().numpy(), f.h)
    assert abs(m1 - want) <= 2e-16 * abs(want)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)       # periodic: conserved
    s.close()


def test_mass_fp32_is_compensated(orc):
    f = inputs.random_smooth(117, (16, 40, 72), cmax=0.15).astype(np.float32)
    s = _solver(f, dtype=torch.float32)
    m = s.mass()
    want = orc.mass(f.psi.astype(np.float64), f.h.astype(np.float64))
    assert abs(m - want) <= 2e-16 * abs(want)
    s.close()


def test_mass_reports_nonfinite():
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(119, (4, 8, 8))
    f.psi[1, 2, 3] = np.nan
    s = _solver(f)
    with pytest.raises(_lib.MpdataError) as e:
        s.mass()
    assert e.value.code == _lib.MPDATA_ENONFINITE
    s.close()


# ------------------------------------------------------------ validation

def test_create_rejects_mismatched_periodic_faces():
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(121, (4, 8, 8))
    f.u2[2, -1, 3] += 0.01
    with pytest.raises(_lib.MpdataError, match="face"):
        _solver(f)


def test_create_rejects_nonpositive_density():
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(123, (4, 8, 8))
    f.h[0, 0, 0] = 0.0
    with pytest.raises(_lib.MpdataError, match="h must"):
        _solver(f)


# ------------------------------------------------ determinism and restart

def test_deterministic_and_restartable():
    f = inputs.random_smooth(125, (12, 33, 47), cmax=0.15)
    a = gpu_run(f, 10)
    b = gpu_run(f, 10)
    np.testing.assert_array_equal(a, b)
    s = _solver(f)
    s.step(5)
    saved = torch.empty_like(s.psi)
    s.get_psi(saved)
    s.step(3)                       # diverge, then restore
    s.set_psi(saved)
    s.step(5)
    s.sync()
    np.testing.assert_array_equal(s.psi.cpu().numpy(), a)
    s.close()


# ------------------------------------------------------------------ FP32

@pytest.mark.parametrize("bc", [0, 1], ids=["periodic", "open"])
def test_fp32_against_fp64_oracle(orc, bc):
    steps = 8
    f = inputs.random_smooth(127, (12, 50, 70), bc=bc, cmax=0.15).astype(np.float32)
    want = oracle_run(orc, f.as_f64(), steps)
    got = gpu_run(f, steps, dtype=torch.float32)
    check_fp32(got, want, f"bc={bc}")


def test_fp32_every_tile_agrees(orc):
    from paper_1507_01265_amd import _lib
    f = inputs.random_smooth(129, (7, 45, 70), cmax=0.15).astype(np.float32)
    first = None
    for tile in range(1, _lib.mpdata_tile_count() + 1):
        got = gpu_run(f, 3, dtype=torch.float32, tile=tile)
        if first is None:
            first = got
        np.testing.assert_array_equal(got, first)


# ------------------------------------------------------------ full sizes

# ------------------------------------------------- variable-sign option

def _mixed_sign(seed, shape, bc=0):
    import dataclasses
    f = inputs.random_smooth(seed, shape, bc=bc)
    return dataclasses.replace(f, psi=f.psi - 1.0)


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("nonos", [True, False])
def test_vsign_parity_fp64(orc, bc, nonos):
    """|psi1| in the ratios on a sign-changing field, ragged tiles, 4 steps."""
    f = _mixed_sign(31, (13, 45, 70), bc)
    assert f.psi.min() < 0.0 < f.psi.max()
    want = oracle_run(orc, f, 4, nonos=nonos, vsign=True)
    got = gpu_run(f, 4, nonos=nonos, vsign=True)
    assert rel_linf(got, want) <= 1e-12


@pytest.mark.parametrize("bc", [0, 1])
def test_vsign_parity_fp32(orc, bc):
    f = _mixed_sign(32, (13, 45, 70), bc).astype(np.float32)
    n = 4
    want = oracle_run(orc, f.as_f64(), n, vsign=True)
    got = gpu_run(f, n, dtype=torch.float32, vsign=True)
    check_fp32(got, want)


def test_vsign_is_the_default_scheme_on_positive_fields():
    f = inputs.random_smooth(33, (13, 45, 70))
    assert f.psi.min() > 0.3
    assert np.array_equal(gpu_run(f, 3, vsign=True), gpu_run(f, 3))


def test_vsign_odd_symmetry_bitwise():
    import dataclasses
    f = _mixed_sign(34, (13, 45, 70))
    a = gpu_run(f, 3, nonos=False, vsign=True)
    b = gpu_run(dataclasses.replace(f, psi=-f.psi), 3, nonos=False, vsign=True)
    assert np.array_equal(b, -a)


def test_vsign_needs_a_default_launch_shape():
    from paper_1507_01265_amd import _lib
    f = _mixed_sign(35, (8, 16, 16))
    with pytest.raises((_lib.MpdataError, ValueError)):
        gpu_run(f, 1, tile=4, vsign=True)


@pytest.mark.slow
def test_full_size_rotation_fp64(orc):
    """512x256x64, the rotation workload at full size, 2 steps."""
    f = inputs.rotation()
    want = oracle_run(orc, f, 2)
    got = gpu_run(f, 2)
    assert rel_linf(got, want) <= 1e-12
    assert got.min() >= -1e-15


@pytest.mark.slow
def test_full_size_rotation_fp64_100_steps(orc):
    """512x256x64 rotation, the benchmark's 100 steps: the scheme's rounding
    differences must not grow past the FP64 bound over a whole run."""
    f = inputs.rotation()
    want = oracle_run(orc, f, 100)
    got = gpu_run(f, 100)
    assert rel_linf(got, want) <= 1e-12
    assert got.min() >= -1e-15


@pytest.mark.slow
def test_full_size_rotation_fp32_100_steps(orc):
    """512x256x64 rotation in FP32 + FP64 limiter, the benchmark's 100 steps,
    against the FP64 oracle within the FP32 bar; the zero background stays
    non-negative and the mass drift stays within the FP32 bar."""
    f = inputs.rotation().astype(np.float32)
    n = 100
    want = oracle_run(orc, f.as_f64(), n)
    s = _solver(f, dtype=torch.float32)
    m0 = s.mass()
    s.step(n)
    m1 = s.mass()
    got = s.psi.cpu().numpy().astype(np.float64)
    s.close()
    drift = (m1 - m0) / m0
    check_fp32(got, want, f"rotation 100 steps min {got.min():.3e} drift {drift:.3e}")
    assert got.min() >= 0.0
    assert abs(drift) <= FP32_DRIFT


@pytest.mark.slow
def test_full_size_streamfunction_fp32_50_steps(orc):
    """1024x512x64 open domain, FP32 + FP64 limiter, the configured 50 steps,
    against the FP64 oracle; the open-boundary mass budget holds on the GPU
    side: the change of the mass over the run equals the net donor-cell
    inflow through the six boundary faces summed over the steps (the
    corrective fluxes there are zero)."""
    f = inputs.streamfunction().astype(np.float32)
    n = 50
    want = oracle_run(orc, f.as_f64(), n)
    s = _solver(f, dtype=torch.float32, graph=False)
    u = [t.astype(np.float64) for t in (f.u1, f.u2, f.u3)]
    m0 = s.mass()
    inflow = 0.0
    for _ in range(n):
        psi_n = s.psi.cpu().numpy().astype(np.float64)
        inflow += orc.open_inflow(psi_n, *u)
        s.step(1)
    m1 = s.mass()
    got = s.psi.cpu().numpy().astype(np.float64)
    s.close()
    check_fp32(got, want, "streamfunction 50 steps")
    budget = abs((m1 - m0) - inflow) / abs(m0)
    print(f"mass change {(m1 - m0) / m0:.3e}, budget residual {budget:.3e}", flush=True)
    assert budget <= 1e-7


@pytest.mark.parametrize("e2", [41, -44], ids=["x2^41", "x2^-44"])
@pytest.mark.parametrize("vsign", [False, True], ids=["plain", "vsign"])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_scaled_field_parity(orc, dtype, vsign, e2):
    """A field scaled by 2^41 (about 2e12) or 2^-44 (about 6e-14): the
    pseudo-velocity's single division over a product of three ratio
    denominators must stay in range (in FP32 each transverse pair is scaled
    by a power of two first).  Positive field, and a sign-changing one with
    the variable-sign option; the oracle runs on the same rounded inputs."""
    import dataclasses
    shape = (13, 45, 70)
    f = _mixed_sign(41, shape) if vsign else inputs.random_smooth(41, shape, cmax=0.15)
    f = dataclasses.replace(f, psi=f.psi * 2.0 ** e2)
    n = 4
    if dtype == "fp64":
        check_fp64(gpu_run(f, n, vsign=vsign), oracle_run(orc, f, n, vsign=vsign), f"2^{e2}")
    else:
        g = f.astype(np.float32)
        want = oracle_run(orc, g.as_f64(), n, vsign=vsign)
        check_fp32(gpu_run(g, n, dtype=torch.float32, vsign=vsign), want, f"2^{e2}")


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_thin_row_of_small_values_on_zero_background(orc, dtype):
    """psi = 0 except one x-row of values near 1e-9: on the row's x-faces
    the transverse ratio sums hold eps alone, so the product of the three
    ratio denominators is about h psi eps^2 (below the smallest normal
    float); the pseudo-velocity must still match the oracle's separate
    ratios."""
    import dataclasses
    f = inputs.random_smooth(42, (9, 21, 64), cmax=0.15)
    psi = np.zeros_like(f.psi)
    x = np.arange(64)
    psi[4, 10, :] = 1e-9 * (1.5 + np.sin(2 * np.pi * x / 64))
    f = dataclasses.replace(f, psi=psi)
    n = 3
    if dtype == "fp64":
        check_fp64(gpu_run(f, n), oracle_run(orc, f, n), "thin row")
    else:
        g = f.astype(np.float32)
        check_fp32(gpu_run(g, n, dtype=torch.float32), oracle_run(orc, g.as_f64(), n), "thin row")


@pytest.mark.slow
def test_full_size_streamfunction_fp64(orc):
    """1024x512x64 open domain in FP64 (the open FP64 kernel), 2 steps."""
    f = inputs.streamfunction()
    want = oracle_run(orc, f, 2)
    got = gpu_run(f, 2)
    assert rel_linf(got, want) <= 1e-12


@pytest.mark.slow
def test_full_size_streamfunction_fp32(orc):
    """1024x512x64 open domain, FP32 + FP64 limiter, 1 step at full size."""
    f = inputs.streamfunction().astype(np.float32)
    want = oracle_run(orc, f.as_f64(), 1)
    got = gpu_run(f, 1, dtype=torch.float32)
    check_fp32(got, want, "streamfunction 1 step")


@pytest.mark.parametrize("bc", [0, 1])
def test_negative_field_parity_fp64(orc, bc):
    """A field below zero everywhere, without the variable-sign option and
    without the limiter (which assumes psi >= 0): every ratio denominator is
    negative and far from zero, so the common denominator of the
    pseudo-velocity is negative and must divide like a positive one."""
    import dataclasses
    f = inputs.random_smooth(36, (13, 45, 70), bc=bc, cmax=0.15)
    f = dataclasses.replace(f, psi=-f.psi)
    assert f.psi.max() < -0.3
    want = oracle_run(orc, f, 4, nonos=False)
    got = gpu_run(f, 4, nonos=False)
    assert rel_linf(got, want) <= 1e-12


def test_negative_field_parity_fp32(orc):
    import dataclasses
    f = inputs.random_smooth(37, (13, 45, 70), cmax=0.15)
    f = dataclasses.replace(f, psi=-f.psi).astype(np.float32)
    n = 4
    want = oracle_run(orc, f.as_f64(), n, nonos=False)
    got = gpu_run(f, n, dtype=torch.float32, nonos=False)
    check_fp32(got, want)


def _interior_tiles(shape, rx, ry):
    """Tiles of an open grid whose region and ring lie inside the x-y domain
    with a cell to spare (they run the periodic x-y addressing)."""
    nz, ny, nx = shape
    tx_n, ty_n = (nx + rx - 5) // (rx - 4), (ny + ry - 5) // (ry - 4)
    return sum(1 for tx in range(tx_n) for ty in range(ty_n)
               if tx * (rx - 4) >= 3 and tx * (rx - 4) + rx <= nx + 1
               and ty * (ry - 4) >= 3 and ty * (ry - 4) + ry <= ny + 1)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_open_grid_interior_and_edge_tiles(orc, dtype):
    """130x100x9 open grid: interior tiles (periodic x-y addressing) and edge
    tiles (clamped addressing, redirected neighbours) side by side in the
    default launch shape of each precision, with each option."""
    shape = (9, 100, 130)
    f = inputs.random_smooth(38, shape, bc=1, cmax=0.15)
    rx, ry = (32, 24) if dtype == "fp64" else (32, 32)
    assert _interior_tiles(shape, rx, ry) >= 2
    # plain, with the divergent-flow term, and with the variable-sign option
    # on a field that crosses zero
    cases = [(f, 4, {}), (f, 2, {"div": True}), (_mixed_sign(39, shape, 1), 2, {"vsign": True})]
    for g, n, opts in cases:
        print(f"{dtype} {opts}", flush=True)
        if dtype == "fp64":
            want = oracle_run(orc, g, n, **opts)
            assert rel_linf(gpu_run(g, n, **opts), want) <= 1e-12
        else:
            g = g.astype(np.float32)
            want = oracle_run(orc, g.as_f64(), n, **opts)
            got = gpu_run(g, n, dtype=torch.float32, **opts)
            check_fp32(got, want)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_open_column_cut_into_shares(orc, dtype):
    """One 20x20 tile with 200 planes: the plan cuts the column into
    contiguous shares of about 25 planes, so most segments start (and prime
    their pipeline) on planes away from the open top and bottom, where the
    march runs without the z-boundary handling; options and more passes
    too."""
    f = inputs.random_smooth(40, (200, 20, 20), bc=1, cmax=0.15)
    for n, opts in ((3, {}), (2, {"div": True}), (2, {"iord": 3})):
        print(f"{dtype} {opts}", flush=True)
        if dtype == "fp64":
            want = oracle_run(orc, f, n, **opts)
            assert rel_linf(gpu_run(f, n, **opts), want) <= 1e-12
        else:
            g = f.astype(np.float32)
            want = oracle_run(orc, g.as_f64(), n, **opts)
            got = gpu_run(g, n, dtype=torch.float32, **opts)
            check_fp32(got, want, str(opts))
