"""The paper's model-based partitioning (Theorem 1, Algorithm 1) on the host:
the oracle pinned to the paper's printed numbers, to Theorem 1 and to
exhaustive search, and the library's implementation checked against it."""
import random

import pytest

from oracle import fpm
from paper_1507_01265_amd import _lib

# Section 4: the 240x240x128 domain, frames of 120x128 cells, speeds in
# cells/s; theoretical times of Table 1 (odd teams 120 + dm frames).
FRAME = 120 * 128
TABLE1_THEORETICAL = {0: 1.486, 4: 1.470, 6: 1.401, 7: 1.422, 8: 1.386, 9: 1.398, 10: 1.397,
                      11: 1.429, 12: 1.402}


def test_worked_example_arithmetic():
    # the uneven split's predicted time printed in section 4
    t = max(120 * 128 * 128 / 1418579, 120 * 112 * 128 / 1436742)
    assert round(t, 3) == 1.386
    assert fpm.time_of({128: 1418579 / FRAME}, 128) == pytest.approx(t)


def _table1_speed():
    """A speed function (cells/s per frame count) consistent with Table 1's
    theoretical column, reading each time as the larger share's time; the
    smaller shares run at the printed s(112) and never dominate; sizes the
    table does not list take the even split's time (1.486 s)."""
    s = {}
    for x in range(1, 240):
        if x < 120:
            s[x] = 1436742.0
        else:
            t = TABLE1_THEORETICAL.get(x - 120, TABLE1_THEORETICAL[0])
            s[x] = FRAME * x / t
    return s


def test_algorithm1_reproduces_table1_choice():
    s = _table1_speed()
    x_l, x_r, t = fpm.algorithm1(s, 480, 4, 1)
    assert (x_l, x_r) == (112, 128)  # the paper's choice: dm = 8
    assert round(t * FRAME, 3) == 1.386
    # Theorem 1's condition is violated by this profile (section 3)
    holds, bad = fpm.satisfies_theorem1(s, list(range(110, 131)))
    assert not holds and bad


@pytest.mark.parametrize("p", [2, 4])
def test_theorem1_balanced_is_optimal(p):
    # s(x) = a x / (x + c): s(x)/x = a / (x + c) decreases, so Theorem 1 holds
    s = {x: 3.0 * x / (x + 5.0) for x in range(1, 64)}
    holds, _ = fpm.satisfies_theorem1(s, list(range(1, 64)))
    assert holds
    n = 12 * p // 2 if p == 4 else 16
    x_l, x_r, t = fpm.algorithm1(s, n, p, 1)
    assert x_l == x_r == n // p
    assert t == pytest.approx(fpm.best_split_brute_force(s, n, p, 1))


def test_algorithm1_is_the_best_of_its_family():
    rng = random.Random(7)
    for trial in range(200):
        p = rng.choice([2, 4, 6, 8])
        dx = rng.choice([1, 2])
        share = dx * rng.randint(2, 12)
        n = p * share
        s = {x: rng.uniform(0.5, 2.0) * x ** rng.uniform(0.5, 1.5) for x in range(dx, 2 * share, dx)}
        assert fpm.algorithm1(s, n, p, dx) == fpm.best_pair_brute_force(s, n, p, dx)


def test_algorithm1_scale_invariance():
    s = _table1_speed()
    a = fpm.algorithm1(s, 480, 4, 1)
    b = fpm.algorithm1({x: 7.25 * v for x, v in s.items()}, 480, 4, 1)
    assert a[:2] == b[:2] and b[2] == pytest.approx(a[2] / 7.25)


def test_algorithm1_rejects_bad_shapes():
    s = {x: 1.0 for x in range(1, 100)}
    for args in ((30, 3, 1), (30, 4, 1), (32, 4, 3)):
        with pytest.raises(ValueError):
            fpm.algorithm1(s, *args)


def _table(s, dx, top):
    """speed[k] = s(k*dx) for k = 0..top/dx (speed[0] unused)."""
    return [1.0] + [s[k * dx] for k in range(1, top // dx + 1)]


def test_library_partition_matches_oracle():
    rng = random.Random(11)
    s1 = _table1_speed()
    assert _lib.mpdata_fpm_partition(_table(s1, 1, 239), 480, 4, 1) == fpm.algorithm1(s1, 480, 4, 1)
    for trial in range(300):
        p = rng.choice([2, 4, 8])
        dx = rng.choice([1, 2, 4])
        share = dx * rng.randint(1, 16)
        n = p * share
        s = {x: rng.uniform(0.5, 2.0) * x ** rng.uniform(0.3, 1.7)
             for x in range(dx, 2 * share + dx, dx)}
        got = _lib.mpdata_fpm_partition(_table(s, dx, 2 * share), n, p, dx)
        assert got == fpm.algorithm1(s, n, p, dx)  # bit for bit, time included


def test_library_check_matches_oracle():
    rng = random.Random(13)
    for trial in range(100):
        dx = rng.choice([1, 2])
        top = dx * rng.randint(2, 30)
        s = {x: rng.uniform(0.5, 2.0) * x ** rng.uniform(0.5, 1.2) for x in range(dx, top + 1, dx)}
        holds, bad = fpm.satisfies_theorem1(s, list(range(dx, top + 1, dx)))
        count, first = _lib.mpdata_fpm_check(_table(s, dx, top), dx)
        assert count == len(bad)
        assert first == (bad[0] if bad else None)


def test_library_rejects_bad_arguments():
    with pytest.raises(_lib.MpdataError):
        _lib.mpdata_fpm_partition([1.0] * 10, 30, 3, 1)    # p odd
    with pytest.raises(_lib.MpdataError):
        _lib.mpdata_fpm_partition([1.0] * 4, 32, 4, 1)     # table too short
    with pytest.raises(_lib.MpdataError):
        _lib.mpdata_fpm_partition([1.0, 1.0, -1.0] + [1.0] * 20, 16, 2, 1)  # negative speed
    with pytest.raises(_lib.MpdataError):
        _lib.mpdata_fpm_check([1.0], 1)
