"""The golden values of the 4-cell line are re-derived in exact rationals by
the committed script tests/golden/derive_1d.py (Python fractions only; it
imports neither the oracle nor the library) and must equal the stored
files."""
import json
import os
import sys

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import derive_1d  # noqa: E402


@pytest.mark.parametrize("name", sorted(derive_1d.FILES))
def test_stored_golden_values_equal_their_derivation(name):
    with open(os.path.join(GOLDEN, name)) as f:
        stored = json.load(f)
    assert stored == derive_1d.FILES[name]()


def test_derivation_is_independent_of_the_code_under_test():
    src = open(derive_1d.__file__).read()
    for mod in ("oracle", "paper_1507_01265_amd", "numpy"):
        assert f"import {mod}" not in src and f"from {mod}" not in src


def test_limit_of_eps_in_the_limiter():
    from fractions import Fraction as Fr
    # an inactive face: nothing flows in and the cell sits at its maximum
    assert derive_1d._capped(Fr(0), Fr(0)) == 0
    assert derive_1d._capped(Fr(1, 3), Fr(0)) == 1
    assert derive_1d._capped(Fr(1, 3), Fr(1, 2)) == Fr(2, 3)
    assert derive_1d._ratio(Fr(0), Fr(0)) == 0
