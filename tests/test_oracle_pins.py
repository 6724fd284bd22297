"""Pins of the FP64 CPU oracle against facts fixed by the mathematics.

Nothing here compares the oracle with itself: every expected value comes
from hand arithmetic, a closed form, an exact rational sum, an invariant of
the scheme or its known order of accuracy.  Together they are chosen so that
a plausible slip in any stage -- a dropped term, a wrong sign or index, a
transposed operand -- fails at least one of them (the mutation test in
``test_oracle_mutations.py`` plants such slips and checks that they do).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1507_01265_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53  # unit roundoff of binary64


def _line(psi0, c=0.5):
    n = len(psi0)
    psi = np.array(psi0, dtype=np.float64).reshape(1, 1, n)
    u1 = np.full((1, 1, n + 1), c)
    return psi, u1, np.zeros((1, 2, n)), np.zeros((2, 1, n)), np.ones((1, 1, n))


def _fr(xs):
    return np.array([float(Fraction(x)) for x in xs])


# ------------------------------------------------------------ hand arithmetic

@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "hand_1d.json")))["cases"],
                         ids=lambda c: c["name"])
def test_hand_1d(orc, case):
    """4-cell periodic line, u = 1/2: stage values and results against exact
    rationals worked out by hand (tests/golden/hand_1d.json)."""
    args = _line(_fr(case["psi0"]))
    out, st = orc.step(*args, nonos=True, stages=True)
    np.testing.assert_allclose(st["psi1"].ravel(), _fr(case["psi1"]), rtol=0, atol=1e-15)
    if "v1_faces_0_to_4" in case:
        np.testing.assert_allclose(st["v1"].ravel(), _fr(case["v1_faces_0_to_4"]), rtol=0,
                                   atol=1e-14)
    np.testing.assert_allclose(out.ravel(), _fr(case["psi_nonos"]), rtol=0, atol=1e-14)
    out0 = orc.step(*args, nonos=False)
    np.testing.assert_allclose(out0.ravel(), _fr(case["psi_no_limiter"]), rtol=0, atol=1e-14)
    # a second corrective pass (iord 3): its velocity field is the first
    # pass's antidiffusive velocity
    out3, st3 = orc.step(*args, iord=3, nonos=False, stages=True)
    np.testing.assert_allclose(st3["v1"].ravel(), _fr(case["v_pass2_no_limiter_faces_0_to_4"]),
                               rtol=0, atol=1e-14)
    np.testing.assert_allclose(out3.ravel(), _fr(case["psi_iord3_no_limiter"]), rtol=0, atol=1e-14)
    out3n = orc.step(*args, iord=3, nonos=True)
    np.testing.assert_allclose(out3n.ravel(), _fr(case["psi_iord3_nonos"]), rtol=0, atol=1e-14)


def test_hand_1d_along_every_axis(orc):
    """The same line laid along y and along z (other Courant numbers zero)
    gives the same numbers: the 3-D scheme reduces to the 1-D one."""
    ref = orc.step(*_line([1.0, 2.0, 3.0, 4.0]))
    psi = np.array([1.0, 2.0, 3.0, 4.0])
    # along y
    out_y = orc.step(psi.reshape(1, 4, 1), np.zeros((1, 4, 2)), np.full((1, 5, 1), 0.5),
                     np.zeros((2, 4, 1)), np.ones((1, 4, 1)))
    # along z
    out_z = orc.step(psi.reshape(4, 1, 1), np.zeros((4, 1, 2)), np.zeros((4, 2, 1)),
                     np.full((5, 1, 1), 0.5), np.ones((4, 1, 1)))
    np.testing.assert_array_equal(out_y.ravel(), ref.ravel())
    np.testing.assert_array_equal(out_z.ravel(), ref.ravel())


# ------------------------------------------------------ closed form (donor cell)

@pytest.mark.parametrize("c", [(0.3, 0.2, 0.1), (-0.25, 0.4, -0.3), (0.0, -0.5, 0.45)])
def test_donor_cell_fourier_closed_form(orc, c):
    """iord = 1 with constant Courant numbers on a periodic grid is a linear
    constant-coefficient scheme: each Fourier mode is multiplied per step by
    g = 1 - sum_d [pos(C_d)(1 - e^{-i th_d}) + neg(C_d)(e^{i th_d} - 1)]."""
    rng = np.random.default_rng(7)
    shape = (6, 10, 12)
    psi = rng.uniform(0.5, 1.5, shape)
    u1, u2, u3 = inputs.constant_courant(shape, c)
    nsteps = 5
    out = orc.run(psi, u1, u2, u3, np.ones(shape), nsteps, iord=1)
    th = [2 * np.pi * np.fft.fftfreq(n) for n in shape]
    tz, ty, tx = np.meshgrid(*th, indexing="ij")
    g = np.ones(shape, dtype=complex)
    for cd, t in zip(c, (tx, ty, tz)):
        g -= max(cd, 0.0) * (1 - np.exp(-1j * t)) + min(cd, 0.0) * (np.exp(1j * t) - 1)
    want = np.fft.ifftn(np.fft.fftn(psi) * g ** nsteps).real
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-13)


# ----------------------------------------------------------- exact shifts

@pytest.mark.parametrize("axis,sign", [(2, 1), (2, -1), (1, 1), (1, -1), (0, 1), (0, -1)])
@pytest.mark.parametrize("nonos", [True, False])
def test_courant_one_is_an_exact_shift(orc, axis, sign, nonos):
    """|C| = 1 along one axis, h = 1: the upwind pass moves psi by exactly one
    cell, the pseudo-velocity vanishes (|U| - U^2/G = 0, no cross flow) and the
    step is a bitwise roll for psi in [1, 2) (differences are exact there)."""
    rng = np.random.default_rng(11)
    shape = (5, 6, 7)
    psi = rng.uniform(1.0, 2.0, shape)
    c = [0.0, 0.0, 0.0]
    c[2 - axis] = float(sign)
    u1, u2, u3 = inputs.constant_courant(shape, c)
    out = orc.step(psi, u1, u2, u3, np.ones(shape), nonos=nonos)
    np.testing.assert_array_equal(out, np.roll(psi, sign, axis=axis))


# ---------------------------------------------------------- constant field

def _fields_for_constant(kind, shape, bc):
    if kind == "constant":
        u1, u2, u3 = inputs.constant_courant(shape, (0.21, -0.17, 0.33))
        h = inputs.random_smooth(3, shape).h
    elif kind == "rotation":
        f = inputs.rotation(seed=5, shape=shape)
        u1, u2, u3, h = f.u1, f.u2, f.u3, f.h
    else:
        f = inputs.random_smooth(9, shape, bc=bc, divergence_free=True, cmax=0.45)
        u1, u2, u3, h = f.u1, f.u2, f.u3, f.h
    return u1, u2, u3, h


@pytest.mark.parametrize("kind,bc", [("constant", 0), ("rotation", 0),
                                     ("streamfunction", 0), ("streamfunction", 1)])
def test_constant_field_is_preserved_bitwise(orc, kind, bc):
    """psi = 1 under discretely divergence-free Courant numbers (constant,
    solid-body rotation, or a streamfunction quantised to 2**-16 so every
    flux difference is exact) stays exactly 1, with variable h."""
    shape = (8, 12, 16)
    u1, u2, u3, h = _fields_for_constant(kind, shape, bc)
    psi = np.ones(shape)
    out = orc.run(psi, u1, u2, u3, h, 3, bc=bc)
    np.testing.assert_array_equal(out, psi)


# --------------------------------------------------------------- mass

def test_mass_is_conserved_periodic(orc):
    """Flux form + periodic faces: sum h*psi is unchanged up to the rounding
    of the per-cell division by h (bound: ~10 n u (1 + sum|C|) sum|h psi|)."""
    shape = (8, 12, 16)
    f = inputs.random_smooth(21, shape, cmax=0.15)
    m0 = orc.mass(f.psi, f.h)
    nsteps = 10
    out = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, nsteps)
    m1 = orc.mass(out, f.h)
    bound = 10 * nsteps * U * (1 + 6 * 0.15) * np.abs(f.h * f.psi).sum()
    assert abs(m1 - m0) <= bound
    # and it is genuinely small, not just under a loose bound
    assert abs(m1 - m0) / m0 < 1e-13


def test_mass_budget_open_boundaries(orc):
    """Open (zero-gradient) boundaries: the mass change of one step equals
    the net inflow of the first-order fluxes through the domain faces (the
    corrective fluxes vanish there)."""
    shape = (6, 10, 14)
    f = inputs.random_smooth(33, shape, bc=inputs.BC_OPEN, cmax=0.15)
    m0 = orc.mass(f.psi, f.h)
    out = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, bc=inputs.BC_OPEN)
    m1 = orc.mass(out, f.h)
    inflow = orc.open_inflow(f.psi, f.u1, f.u2, f.u3)
    assert abs(inflow) > 1e-3
    assert abs((m1 - m0) - inflow) <= 1e-12 * np.abs(f.h * f.psi).sum()


def test_mass_sum_is_exact_to_rounding(orc):
    """Dot2 against the exact rational sum of h*psi on small arrays, including
    cancelling signs: the error is within one rounding of the exact value
    plus a term of order u^2 * sum|h psi|."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(1, 300))
        h = rng.uniform(0.5, 1.5, n)
        psi = rng.normal(size=n) * 10.0 ** rng.integers(-3, 4, n)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(h, psi))
        got = orc.mass(psi, h)
        err = abs(Fraction(got) - exact)
        cond = sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(h, psi))
        assert err <= Fraction(U) * abs(exact) + Fraction(4 * n * n) * Fraction(U) ** 2 * cond


# ------------------------------------------------ positivity and monotonicity

@pytest.mark.parametrize("bc", [0, 1])
def test_positivity_and_no_new_extrema(orc, bc):
    """Divergence-free flow with outflow <= h and the limiter on: psi stays
    non-negative, the global max never grows and the global min never drops
    (to rounding).  Uses a zero background with a sharp block, where the
    unlimited scheme does overshoot."""
    shape = (10, 16, 16)
    f = inputs.random_smooth(41, shape, bc=bc, divergence_free=True, cmax=0.4, hvar=0.0)
    psi = np.zeros(shape)
    psi[3:7, 5:11, 4:12] = 1.0
    lo, hi = psi.min(), psi.max()
    cur = psi
    for _ in range(12):
        cur = orc.step(cur, f.u1, f.u2, f.u3, f.h, bc=bc, nonos=True)
        assert cur.min() >= lo - 4 * U
        assert cur.max() <= hi * (1 + 8 * U)
    un = psi
    for _ in range(12):
        un = orc.step(un, f.u1, f.u2, f.u3, f.h, bc=bc, nonos=False)
    assert un.max() > hi + 1e-3 or un.min() < lo - 1e-3


# ------------------------------------------------------- order of accuracy

def _order_1d(orc, iord, hvar, sizes=(64, 128, 256), C=0.4):
    """Max error against the exact solution of d(h psi)/dt + d(C psi)/dx = 0:
    psi is constant along dx/dt = C/h(x), i.e. int_{X0}^{x} h = C t."""
    errs = []
    for N in sizes:
        x = np.arange(N) + 0.5
        psi0 = 2 + np.sin(2 * np.pi * x / N)
        steps = int(round(N / 4 / C))
        h = 1 + hvar * np.sin(2 * np.pi * x / N)
        H = lambda s: s - hvar * N / (2 * np.pi) * np.cos(2 * np.pi * s / N)
        X0 = x - C * steps
        for _ in range(60):
            X0 = X0 + (H(x) - H(X0) - C * steps) / (1 + hvar * np.sin(2 * np.pi * X0 / N))
        exact = 2 + np.sin(2 * np.pi * X0 / N)
        out = orc.run(psi0.reshape(1, 1, N), np.full((1, 1, N + 1), C), np.zeros((1, 2, N)),
                      np.zeros((2, 1, N)), h.reshape(1, 1, N), steps, iord=iord, nonos=False)
        errs.append(np.abs(out.ravel() - exact).max())
    return [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]


@pytest.mark.parametrize("hvar", [0.0, 0.3])
def test_donor_cell_is_first_order(orc, hvar):
    for r in _order_1d(orc, 1, hvar):
        assert 1.85 < r < 2.15


@pytest.mark.parametrize("hvar", [0.0, 0.3])
def test_mpdata_is_second_order_1d(orc, hvar):
    """One corrective pass makes the scheme second order; with variable h
    this holds only with the face density G in the pseudo-velocity."""
    for r in _order_1d(orc, 2, hvar):
        assert 3.7 < r < 4.4


@pytest.mark.parametrize("c", [(0.3, 0.2, 0.0), (0.2, -0.15, 0.1)])
def test_mpdata_is_second_order_oblique(orc, c):
    """Oblique constant flow: second order requires the cross-derivative
    terms (B2, B3 with the averaged transverse Courant numbers)."""
    errs = []
    for N in (16, 32, 64):
        nz = N if c[2] != 0.0 else 1
        zc, yc, xc = [np.arange(n) + 0.5 for n in (nz, N, N)]
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        prof = lambda X, Y, Z: (2 + np.sin(2 * np.pi * X / N) * np.cos(2 * np.pi * Y / N)
                                * (np.cos(2 * np.pi * Z / nz) if nz > 1 else 1.0))
        steps = int(round(N / 4 / 0.4))
        u1, u2, u3 = inputs.constant_courant((nz, N, N), c)
        out = orc.run(prof(X, Y, Z), u1, u2, u3, np.ones((nz, N, N)), steps, nonos=False)
        exact = prof(X - c[0] * steps, Y - c[1] * steps, Z - c[2] * steps)
        errs.append(np.abs(out - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.6, ratios


# ------------------------------------------------------------- symmetries

def test_translation_equivariance_bitwise(orc):
    """Constant Courant numbers, periodic grid: rolling the input rolls the
    output, bit for bit (every cell runs the same operations)."""
    shape = (6, 9, 11)
    rng = np.random.default_rng(5)
    psi = rng.uniform(0.2, 1.0, shape)
    u1, u2, u3 = inputs.constant_courant(shape, (0.3, -0.2, 0.15))
    h = np.ones(shape)
    a = orc.step(psi, u1, u2, u3, h)
    sh = (2, -3, 4)
    b = orc.step(np.roll(psi, sh, axis=(0, 1, 2)), u1, u2, u3, h)
    np.testing.assert_array_equal(np.roll(a, sh, axis=(0, 1, 2)), b)


@pytest.mark.parametrize("bc", [0, 1])
def test_mirror_symmetry(orc, bc):
    """Reflecting x (reverse the cells, reverse and negate the x-faces) maps
    the solution onto its reflection, to rounding."""
    f = inputs.random_smooth(51, (6, 8, 10), bc=bc, cmax=0.15)
    a = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 3, bc=bc)
    b = orc.run(f.psi[:, :, ::-1], -f.u1[:, :, ::-1], f.u2[:, :, ::-1], f.u3[:, :, ::-1],
                f.h[:, :, ::-1], 3, bc=bc)
    np.testing.assert_allclose(b[:, :, ::-1], a, rtol=0, atol=1e-13)


@pytest.mark.parametrize("bc", [0, 1])
def test_axis_permutation_symmetry(orc, bc):
    """Swapping x and y (transpose the arrays, exchange u1 and u2) maps the
    solution onto its transpose, to rounding."""
    f = inputs.random_smooth(61, (5, 9, 7), bc=bc, cmax=0.15)
    a = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 3, bc=bc)
    t = lambda x: np.ascontiguousarray(np.swapaxes(x, 1, 2))
    b = orc.run(t(f.psi), t(f.u2), t(f.u1), t(f.u3), t(f.h), 3, bc=bc)
    np.testing.assert_allclose(t(b), a, rtol=0, atol=1e-13)


def test_cyclic_axis_permutation_symmetry(orc):
    """x -> y -> z -> x: the pseudo-velocity is written once and applied by
    cyclic permutation, so rotating the axes of the problem rotates the
    answer (to rounding)."""
    f = inputs.random_smooth(71, (6, 7, 8), cmax=0.15)
    a = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 2)
    # new axes (z', y', x') = (y, x, z): array axes (0,1,2) -> (1,2,0)
    r = lambda x: np.ascontiguousarray(np.transpose(x, (1, 2, 0)))
    b = orc.run(r(f.psi), r(f.u3), r(f.u1), r(f.u2), r(f.h), 2)
    np.testing.assert_allclose(b, r(a), rtol=0, atol=1e-13)


# ----------------------------------------------------------- small details

def test_iord_one_is_the_first_pass(orc):
    f = inputs.random_smooth(81, (4, 5, 6), cmax=0.15)
    out, st = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, iord=2, stages=True)
    out1 = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, iord=1)
    np.testing.assert_array_equal(out1, st["psi1"])


def test_bounds_are_the_7_point_extrema(orc):
    """The limiter bounds against a brute-force loop over the 7-point
    neighbourhood of both fields (the paper's stage 8, Listing 1)."""
    f = inputs.random_smooth(91, (4, 5, 6), cmax=0.15)
    _, st = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, stages=True)
    p1 = st["psi1"]
    nz, ny, nx = f.psi.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                vals = []
                for dk, dj, di in [(0, 0, 0), (0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0),
                                   (-1, 0, 0), (1, 0, 0)]:
                    kk, jj, ii = (k + dk) % nz, (j + dj) % ny, (i + di) % nx
                    vals += [f.psi[kk, jj, ii], p1[kk, jj, ii]]
                assert st["mx"][k, j, i] == max(vals)
                assert st["mn"][k, j, i] == min(vals)


def test_parameter_validation(orc):
    f = inputs.random_smooth(1, (2, 3, 4))
    for iord in (0, 17):
        with pytest.raises(ValueError):
            orc.step(f.psi, f.u1, f.u2, f.u3, f.h, iord=iord)
    with pytest.raises(ValueError):
        orc.step(f.psi, f.u1, f.u2, f.u3, f.h, bc=2)
    with pytest.raises(ValueError):
        orc.step(f.psi, f.u1[:, :, :-1], f.u2, f.u3, f.h)


# ------------------------------------------- variable-sign option (|psi1|)

def test_vsign_is_the_default_scheme_on_positive_fields(orc):
    """|psi1| = psi1 where the field is positive: the option changes nothing."""
    f = inputs.random_smooth(21, (6, 10, 12))
    assert f.psi.min() > 0.3
    a = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 4)
    b = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 4, vsign=True)
    np.testing.assert_array_equal(a, b)


def test_vsign_odd_symmetry_bitwise(orc):
    """Without the limiter the scheme with |psi1| in the ratios is odd in psi
    bit for bit: the donor passes are linear and V depends on |psi1| only.
    (Without the option the ratio denominators psi_a + psi_b + eps change
    under negation, so the identity fails.)"""
    f = inputs.random_smooth(22, (6, 10, 12))
    psi = f.psi - 1.0
    assert psi.min() < 0.0 < psi.max()
    a = orc.run(psi, f.u1, f.u2, f.u3, f.h, 3, nonos=False, vsign=True)
    b = orc.run(-psi, f.u1, f.u2, f.u3, f.h, 3, nonos=False, vsign=True)
    np.testing.assert_array_equal(b, -a)
    c = orc.run(psi, f.u1, f.u2, f.u3, f.h, 1, nonos=False)
    d = orc.run(-psi, f.u1, f.u2, f.u3, f.h, 1, nonos=False)
    assert not np.array_equal(d, -c)


def _sine_wave(n, c=0.5):
    x = (np.arange(n) + 0.5) / n
    psi = np.sin(2 * np.pi * x)[None, None, :]
    return (psi, np.full((1, 1, n + 1), c), np.zeros((1, 2, n)), np.zeros((2, 1, n)),
            np.ones((1, 1, n)), int(round(n / c)))


def test_vsign_advects_a_sign_changing_wave(orc):
    """One period of a sine wave: with |psi1| the scheme stays finite, beats
    the donor-cell pass and, with the limiter, creates no new extrema; the
    plain ratios divide by psi_a + psi_b + eps near the zero crossings and
    blow up."""
    psi, u1, u2, u3, h, steps = _sine_wave(64)
    v = orc.run(psi, u1, u2, u3, h, steps, nonos=False, vsign=True)
    d = orc.run(psi, u1, u2, u3, h, steps, iord=1)
    assert np.isfinite(v).all()
    assert np.sqrt(np.mean((v - psi) ** 2)) < 0.7 * np.sqrt(np.mean((d - psi) ** 2))
    lim = orc.run(psi, u1, u2, u3, h, steps, nonos=True, vsign=True)
    assert lim.max() <= psi.max() + 1e-14 and lim.min() >= psi.min() - 1e-14
    with np.errstate(all="ignore"):
        plain = orc.run(psi, u1, u2, u3, h, steps, nonos=False)
    assert not np.isfinite(plain).all() or np.abs(plain).max() > 10


# ------------------------------------------ more corrective passes (iord > 2)

@pytest.mark.parametrize("axis,sign", [(2, 1), (1, -1), (0, 1)])
@pytest.mark.parametrize("nonos", [True, False])
@pytest.mark.parametrize("iord", [3, 4])
def test_more_passes_keep_the_courant_one_shift(orc, axis, sign, nonos, iord):
    """|C| = 1: the first antidiffusive velocity vanishes, so every further
    pass has a zero velocity field and the step stays an exact roll."""
    rng = np.random.default_rng(12)
    shape = (5, 6, 7)
    psi = rng.uniform(1.0, 2.0, shape)
    c = [0.0, 0.0, 0.0]
    c[2 - axis] = float(sign)
    u1, u2, u3 = inputs.constant_courant(shape, c)
    out = orc.step(psi, u1, u2, u3, np.ones(shape), nonos=nonos, iord=iord)
    np.testing.assert_array_equal(out, np.roll(psi, sign, axis=axis))


@pytest.mark.parametrize("kind,bc", [("rotation", 0), ("streamfunction", 1)])
def test_more_passes_preserve_a_constant_field(orc, kind, bc):
    shape = (8, 12, 16)
    u1, u2, u3, h = _fields_for_constant(kind, shape, bc)
    psi = np.ones(shape)
    out = orc.run(psi, u1, u2, u3, h, 2, bc=bc, iord=4)
    np.testing.assert_array_equal(out, psi)


@pytest.mark.parametrize("iord", [3, 5])
def test_more_passes_conserve_mass(orc, iord):
    shape = (8, 12, 16)
    f = inputs.random_smooth(22, shape, cmax=0.15)
    m0 = orc.mass(f.psi, f.h)
    out = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 5, iord=iord)
    assert abs(orc.mass(out, f.h) - m0) / m0 < 1e-13


@pytest.mark.parametrize("bc", [0, 1])
def test_more_passes_stay_positive_without_new_extrema(orc, bc):
    shape = (10, 16, 16)
    f = inputs.random_smooth(42, shape, bc=bc, divergence_free=True, cmax=0.4, hvar=0.0)
    psi = np.zeros(shape)
    psi[3:7, 5:11, 4:12] = 1.0
    cur = psi
    for _ in range(8):
        cur = orc.step(cur, f.u1, f.u2, f.u3, f.h, bc=bc, nonos=True, iord=3)
        assert cur.min() >= -4 * U
        assert cur.max() <= 1 + 8 * U
    un = psi
    for _ in range(8):
        un = orc.step(un, f.u1, f.u2, f.u3, f.h, bc=bc, nonos=False, iord=3)
    assert un.max() > 1 + 1e-3 or un.min() < -1e-3


def _errors_1d(orc, iord, hvar, C, sizes=(64, 128, 256)):
    """Max errors of the 1-D solutions of _order_1d (same exact solution)."""
    errs = []
    for N in sizes:
        x = np.arange(N) + 0.5
        psi0 = 2 + np.sin(2 * np.pi * x / N)
        steps = int(round(N / 4 / C))
        h = 1 + hvar * np.sin(2 * np.pi * x / N)
        H = lambda s: s - hvar * N / (2 * np.pi) * np.cos(2 * np.pi * s / N)
        X0 = x - C * steps
        for _ in range(60):
            X0 = X0 + (H(x) - H(X0) - C * steps) / (1 + hvar * np.sin(2 * np.pi * X0 / N))
        exact = 2 + np.sin(2 * np.pi * X0 / N)
        out = orc.run(psi0.reshape(1, 1, N), np.full((1, 1, N + 1), C), np.zeros((1, 2, N)),
                      np.zeros((2, 1, N)), h.reshape(1, 1, N), steps, iord=iord, nonos=False)
        errs.append(np.abs(out.ravel() - exact).max())
    return np.array(errs)


@pytest.mark.parametrize("hvar", [0.0, 0.3])
def test_a_second_pass_reduces_the_error_1d(orc, hvar):
    """A second corrective pass removes part of the first pass's remaining
    truncation error (Smolarkiewicz 1984): the scheme stays (at least) second
    order and its error at every resolution is about half that of iord 2."""
    e2 = _errors_1d(orc, 2, hvar, 0.25)
    e3 = _errors_1d(orc, 3, hvar, 0.25)
    assert np.all(e3 < 0.55 * e2), e3 / e2
    assert np.all(e3[:-1] / e3[1:] > 3.6), e3[:-1] / e3[1:]


@pytest.mark.parametrize("c", [(0.3, 0.2, 0.0), (0.25, -0.15, 0.1)])
def test_a_second_pass_reduces_the_error_oblique(orc, c):
    """Oblique flow: the second pass's cross terms take the transverse
    components of the first antidiffusive velocity; with them the error at
    64 cells drops to well under a third of iord 2's."""
    def err(iord, N):
        nz = N if c[2] != 0.0 else 1
        zc, yc, xc = [np.arange(n) + 0.5 for n in (nz, N, N)]
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        prof = lambda X, Y, Z: (2 + np.sin(2 * np.pi * X / N) * np.cos(2 * np.pi * Y / N)
                                * (np.cos(2 * np.pi * Z / nz) if nz > 1 else 1.0))
        steps = int(round(N / 4 / 0.4))
        u1, u2, u3 = inputs.constant_courant((nz, N, N), c)
        out = orc.run(prof(X, Y, Z), u1, u2, u3, np.ones((nz, N, N)), steps, nonos=False,
                      iord=iord)
        return np.abs(out - prof(X - c[0] * steps, Y - c[1] * steps, Z - c[2] * steps)).max()
    e3 = [err(3, N) for N in (32, 64)]
    assert e3[1] < 0.3 * err(2, 64)
    assert e3[0] / e3[1] > 3.6


def test_more_passes_bound_over_every_iterate(orc):
    """The limiter bounds of the second corrective pass against a brute-force
    7-point max/min over psi^n, psi^(1) and psi^(2) (psi^(2) = the iord 2
    step); over psi^n and psi^(2) alone they would differ."""
    f = inputs.random_smooth(92, (4, 5, 6), cmax=0.3)
    _, st = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, iord=3, stages=True)
    p2 = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, iord=2)
    fields = [f.psi, st["psi1"], p2]
    offs = [(0, 0, 0), (0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]

    def brute(fs, red):
        return red([np.roll(a, (-dk, -dj, -di), axis=(0, 1, 2)) for a in fs
                    for dk, dj, di in offs], axis=0)
    np.testing.assert_array_equal(st["mx"], brute(fields, np.max))
    np.testing.assert_array_equal(st["mn"], brute(fields, np.min))
    assert ((brute([f.psi, p2], np.max) != st["mx"]).any() or
            (brute([f.psi, p2], np.min) != st["mn"]).any())


# ------------------------------------------------- divergent-flow term (div)

def test_divergence_term_by_hand(orc):
    """4-cell line with uneven face Courant numbers: V and the step with and
    without the term against exact rationals (tests/golden/hand_div_1d.json)."""
    g = json.load(open(os.path.join(GOLDEN, "hand_div_1d.json")))
    psi = _fr(g["psi0"]).reshape(1, 1, 4)
    u1 = _fr(g["u1_faces_0_to_4"]).reshape(1, 1, 5)
    args = (psi, u1, np.zeros((1, 2, 4)), np.zeros((2, 1, 4)), np.ones((1, 1, 4)))
    for key, div in (("without_term", False), ("with_term", True)):
        out, st = orc.step(*args, nonos=False, stages=True, div=div)
        np.testing.assert_allclose(st["psi1"].ravel(), _fr(g["psi1"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(st["v1"].ravel(), _fr(g[key]["v1_faces_0_to_4"]), rtol=0,
                                   atol=1e-14)
        np.testing.assert_allclose(out.ravel(), _fr(g[key]["psi"]), rtol=0, atol=1e-14)


def _rk4_back(x, vel, T, nsub=2000):
    """Foot of the characteristic dx/dt = vel(x) through x after time T."""
    dt = T / nsub
    for _ in range(nsub):
        k1 = -vel(x)
        k2 = -vel(x + 0.5 * dt * k1)
        k3 = -vel(x + 0.5 * dt * k2)
        k4 = -vel(x + dt * k3)
        x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return x


def _divergent_1d_errors(orc, div, sizes, iord=2, C0=0.3, amp=0.5):
    """d psi/dt + d(u psi)/dx = 0 with steady u(x) = C0 (1 + amp sin(2 pi x/N)):
    u psi is constant along dx/dt = u, so psi(x, T) = psi0(X) u(X) / u(x) with
    X the foot of the characteristic (integrated by RK4 to 1e-12)."""
    errs = []
    for N in sizes:
        vel = lambda x: C0 * (1 + amp * np.sin(2 * np.pi * x / N))
        f = np.arange(N + 1, dtype=float)
        U = vel(f)
        U[-1] = U[0]
        x = np.arange(N) + 0.5
        psi0 = lambda X: 2 + np.sin(2 * np.pi * X / N)
        steps = int(round(N / 4 / C0))
        out = orc.run(psi0(x).reshape(1, 1, N), U.reshape(1, 1, N + 1), np.zeros((1, 2, N)),
                      np.zeros((2, 1, N)), np.ones((1, 1, N)), steps, iord=iord, nonos=False,
                      div=div)
        X = _rk4_back(x, vel, steps)
        errs.append(np.abs(out.ravel() - psi0(X) * vel(X) / vel(x)).max())
    return np.array(errs)


@pytest.mark.parametrize("iord", [2, 3])
def test_divergence_term_restores_second_order_1d(orc, iord):
    """In a divergent flow the donor-cell error has a part proportional to
    psi times the divergence; without the term MPDATA is only first order
    there, with it second order."""
    e_on = _divergent_1d_errors(orc, True, (64, 128, 256), iord)
    e_off = _divergent_1d_errors(orc, False, (64, 128, 256), iord)
    assert np.all(e_on[:-1] / e_on[1:] > 3.5), e_on[:-1] / e_on[1:]
    assert np.all(e_off[:-1] / e_off[1:] < 2.4), e_off[:-1] / e_off[1:]
    assert e_on[-1] < 0.15 * e_off[-1]


def test_divergence_term_transverse_parts_2d(orc):
    """Separable divergent flow u(x), v(y): psi u(x) v(y) is constant along the
    characteristics.  Second order needs the transverse parts of the
    divergence across each face."""
    def err(N, div):
        c1, c2, amp = 0.25, 0.2, 0.4
        ux = lambda x: c1 * (1 + amp * np.sin(2 * np.pi * x / N))
        vy = lambda y: c2 * (1 + amp * np.cos(2 * np.pi * y / N))
        f = np.arange(N + 1, dtype=float)
        cc = np.arange(N) + 0.5
        U1 = np.broadcast_to(ux(f)[None, None, :], (1, N, N + 1)).copy()
        U1[..., -1] = U1[..., 0]
        U2 = np.broadcast_to(vy(f)[None, :, None], (1, N + 1, N)).copy()
        U2[:, -1, :] = U2[:, 0, :]
        prof = lambda X, Y: 2 + np.sin(2 * np.pi * X / N) * np.cos(2 * np.pi * Y / N)
        Y, X = np.meshgrid(cc, cc, indexing="ij")
        steps = int(round(N / 4 / 0.3))
        out = orc.run(prof(X, Y)[None], U1, U2, np.zeros((2, N, N)), np.ones((1, N, N)), steps,
                      nonos=False, div=div)
        Y0, X0 = np.meshgrid(_rk4_back(cc, vy, steps), _rk4_back(cc, ux, steps), indexing="ij")
        exact = prof(X0, Y0) * ux(X0) * vy(Y0) / (ux(X) * vy(Y))
        return np.abs(out[0] - exact).max()
    e = [err(N, True) for N in (128, 256)]
    assert e[0] / e[1] > 3.7, e
    assert e[1] < 0.1 * err(256, False)


@pytest.mark.parametrize("kind,bc", [("constant", 0), ("rotation", 0), ("streamfunction", 1)])
def test_divergence_term_vanishes_on_solenoidal_flows(orc, kind, bc):
    """Constant, solid-body and quantised-streamfunction Courant numbers have
    an exactly zero discrete divergence, so the term adds exact zeros."""
    shape = (8, 12, 16)
    u1, u2, u3, h = _fields_for_constant(kind, shape, bc)
    psi = inputs.random_smooth(23, shape).psi
    a = orc.run(psi, u1, u2, u3, h, 3, bc=bc)
    b = orc.run(psi, u1, u2, u3, h, 3, bc=bc, div=True)
    np.testing.assert_array_equal(a, b)


def test_divergence_term_conserves_mass(orc):
    shape = (8, 12, 16)
    f = inputs.random_smooth(24, shape, cmax=0.15)  # random faces: divergent
    m0 = orc.mass(f.psi, f.h)
    out = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 5, div=True, iord=3)
    assert abs(orc.mass(out, f.h) - m0) / m0 < 1e-13
    assert not np.array_equal(out, orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 5, iord=3))


def test_results_do_not_depend_on_the_thread_count(orc):
    """Every output element is computed by one thread from inputs no thread
    writes, so one thread and several give the same bits (the CPU baseline
    may be timed on any number of cores)."""
    f = inputs.random_smooth(61, (6, 20, 24), bc=1, cmax=0.3)
    before = orc.threads()
    try:
        assert orc.set_threads(1) == 1
        one = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 3, bc=f.bc, iord=3, div=True)
        orc.set_threads(max(2, before))
        many = orc.run(f.psi, f.u1, f.u2, f.u3, f.h, 3, bc=f.bc, iord=3, div=True)
    finally:
        orc.set_threads(before)
    np.testing.assert_array_equal(one, many)
    with pytest.raises(ValueError):
        orc.set_threads(0)


# ------------------------------------ time-dependent velocity (step_tv)

def test_time_term_by_hand(orc):
    """4-cell line, Courant numbers 1/2 at the start of the step and uneven
    ones at its end: the pseudo-velocity with the time-variation term and the
    step with and without the limiter and with a second corrective pass,
    against exact rationals (tests/golden/hand_tv_1d.json)."""
    g = json.load(open(os.path.join(GOLDEN, "hand_tv_1d.json")))
    u1 = _fr(g["u1_faces_0_to_4"]).reshape(1, 1, 5)
    w1 = _fr(g["w1_faces_0_to_4"]).reshape(1, 1, 5)
    z2, z3 = np.zeros((1, 2, 4)), np.zeros((2, 1, 4))
    for c in g["cases"]:
        psi = _fr(c["psi0"]).reshape(1, 1, 4)
        args = (psi, u1, z2, z3, w1, z2, z3, np.ones((1, 1, 4)))
        out = orc.step_tv(*args, nonos=False)
        np.testing.assert_allclose(out.ravel(), _fr(c["psi_no_limiter"]), rtol=0, atol=1e-14)
        out = orc.step_tv(*args, nonos=True)
        np.testing.assert_allclose(out.ravel(), _fr(c["psi_nonos"]), rtol=0, atol=1e-14)
        out = orc.step_tv(*args, nonos=False, iord=3)
        np.testing.assert_allclose(out.ravel(), _fr(c["psi_iord3_no_limiter"]), rtol=0, atol=1e-14)


def _ramp(s, S, C0, a):
    """Courant number at time level s of a run of S steps: a quarter sine
    from C0 to C0 (1 + a), so the end differs from the start."""
    return C0 * (1 + a * np.sin(np.pi * s / (2 * S)))


def _time_varying_1d_errors(orc, term, sizes, hvar=0.0, iord=2, C0=0.3, a=1.0):
    """d(h psi)/dt + d(C(t) psi)/dx = 0 with a Courant number uniform in space
    and rising in time: psi is constant along the characteristics, on which
    the integral of h over x grows by the integral of C over t, D =
    C0 S (1 + 2a/pi) after S steps."""
    errs = []
    for N in sizes:
        S = int(round(N / 4 / C0))
        x = np.arange(N) + 0.5
        h = 1 + hvar * np.sin(2 * np.pi * x / N)
        levels = [(np.full((1, 1, N + 1), _ramp(s, S, C0, a)), np.zeros((1, 2, N)),
                   np.zeros((2, 1, N))) for s in range(S + 1)]
        out = orc.run_tv((2 + np.sin(2 * np.pi * x / N)).reshape(1, 1, N), levels,
                         h.reshape(1, 1, N), nonos=False, term=term, iord=iord)
        D = C0 * S * (1 + 2 * a / np.pi)
        H = lambda s: s - hvar * N / (2 * np.pi) * np.cos(2 * np.pi * s / N)
        X0 = x - D
        for _ in range(80):
            X0 = X0 + (H(x) - H(X0) - D) / (1 + hvar * np.sin(2 * np.pi * X0 / N))
        errs.append(np.abs(out.ravel() - (2 + np.sin(2 * np.pi * X0 / N))).max())
    return np.array(errs)


@pytest.mark.parametrize("hvar", [0.0, 0.3])
def test_time_term_restores_second_order_1d(orc, hvar):
    """Holding the Courant number of the start of the step over the step
    shifts the solution by half the change of the Courant number over the
    run: first order.  The time-variation term makes it second order (also
    with variable h, where the term carries no face density)."""
    e_on = _time_varying_1d_errors(orc, True, (64, 128, 256), hvar)
    e_off = _time_varying_1d_errors(orc, False, (64, 128, 256), hvar)
    assert np.all(e_on[:-1] / e_on[1:] > 3.5), e_on[:-1] / e_on[1:]
    assert np.all(e_off[:-1] / e_off[1:] < 2.3), e_off[:-1] / e_off[1:]
    assert e_on[-1] < 0.1 * e_off[-1]


def test_time_term_second_order_3d(orc):
    """Uniform oblique flow whose three components change in time by
    different amounts: second order needs the term on every axis."""
    C0 = np.array([0.2, -0.15, 0.1])
    amp = np.array([1.0, 0.6, -0.8])

    def err(N, term):
        S = int(round(N / 4 / 0.25))
        c = [np.arange(N) + 0.5] * 3
        Z, Y, X = np.meshgrid(*c, indexing="ij")
        prof = lambda X, Y, Z: (2 + np.sin(2 * np.pi * X / N) * np.cos(2 * np.pi * Y / N)
                                * np.cos(2 * np.pi * Z / N))
        levels = []
        for s in range(S + 1):
            cs = _ramp(s, S, C0, amp)
            levels.append((np.full((N, N, N + 1), cs[0]), np.full((N, N + 1, N), cs[1]),
                           np.full((N + 1, N, N), cs[2])))
        out = orc.run_tv(prof(X, Y, Z), levels, np.ones((N, N, N)), nonos=False, term=term)
        D = C0 * S * (1 + 2 * amp / np.pi)
        return np.abs(out - prof(X - D[0], Y - D[1], Z - D[2])).max()
    e = [err(N, True) for N in (32, 64)]
    f = [err(N, False) for N in (32, 64)]
    assert e[0] / e[1] > 3.6, e
    assert f[0] / f[1] < 2.5, f
    assert e[1] < 0.4 * f[1]


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("opts", [{}, {"div": True}, {"vsign": True}, {"iord": 3}],
                         ids=["plain", "div", "vsign", "iord3"])
def test_time_term_vanishes_for_steady_flow(orc, bc, opts):
    """With the same Courant numbers at both ends of the step the term adds
    exact zeros: bitwise the plain step."""
    f = inputs.random_smooth(71, (6, 10, 14), bc=bc, cmax=0.25)
    a = orc.step(f.psi, f.u1, f.u2, f.u3, f.h, bc=bc, **opts)
    b = orc.step_tv(f.psi, f.u1, f.u2, f.u3, f.u1, f.u2, f.u3, f.h, bc=bc, **opts)
    np.testing.assert_array_equal(a, b)


def _two_levels(seed, shape, bc, cmax=0.2, divergence_free=False):
    f = inputs.random_smooth(seed, shape, bc=bc, cmax=cmax, divergence_free=divergence_free)
    g = inputs.random_smooth(seed + 1, shape, bc=bc, cmax=cmax, divergence_free=divergence_free)
    return f, (g.u1, g.u2, g.u3)


def test_time_term_conserves_mass_and_positivity(orc):
    """Periodic: the term is a flux, so mass stays conserved to rounding.
    With divergence-free Courant numbers at both ends psi is constant along
    the characteristics, and with the limiter the step stays positive and
    makes no new extrema."""
    f, w = _two_levels(72, (8, 12, 16), 0, divergence_free=True)
    psi = np.where(f.psi > f.psi.mean(), f.psi, 0.0)
    out = orc.step_tv(psi, f.u1, f.u2, f.u3, *w, f.h)
    m0, m1 = orc.mass(psi, f.h), orc.mass(out, f.h)
    assert abs(m1 - m0) / m0 < 1e-14
    assert out.min() >= -4 * U * psi.max()
    assert out.max() <= psi.max() * (1 + 4 * U)
    assert not np.array_equal(out, orc.step(psi, f.u1, f.u2, f.u3, f.h))


def test_time_term_is_zero_on_open_boundary_faces(orc):
    """Open boundaries: the pseudo-velocity normal to the boundary stays zero
    with the term, so the mass budget is the first-order boundary flux of
    the start-of-step Courant numbers."""
    f, w = _two_levels(73, (6, 10, 12), 1)
    out = orc.step_tv(f.psi, f.u1, f.u2, f.u3, *w, f.h, bc=1)
    d = orc.mass(out, f.h) - orc.mass(f.psi, f.h)
    inflow = orc.open_inflow(f.psi, f.u1, f.u2, f.u3)
    assert abs(d - inflow) < 1e-12 * orc.mass(f.psi, f.h)
