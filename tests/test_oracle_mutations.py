"""The oracle's pins catch plausible slips.

Each case below plants one mistake in a private copy of the oracle's C
source (compiled into a temporary directory, never into ``oracle/``), swaps
it in, and runs the pin checks of ``test_oracle_pins.py``; at least one of
them must fail.  This is the evidence that the pins constrain every stage
and not only the ones a given test happens to touch.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "mpdata_oracle.c")

PV = "double V = (fabs(U) - U * U / G) * A - (U / G) * (Us * Bs + Ut * Bt);"
MUTANTS = {
    "drop_cross_terms": (PV, "double V = (fabs(U) - U * U / G) * A;"),
    "no_face_density": (PV, "double V = (fabs(U) - U * U) * A - U * (Us * Bs + Ut * Bt);"),
    "cross_term_sign": (PV, "double V = (fabs(U) - U * U / G) * A + (U / G) * (Us * Bs + Ut * Bt);"),
    "cross_term_factor": ("double Bs = 0.5 * (s_hi - s_lo)", "double Bs = (s_hi - s_lo)"),
    "transposed_A": ("double A = (pb - pa) / (pb + pa + eps);",
                     "double A = (pa - pb) / (pb + pa + eps);"),
    "donor_operands_swapped": ("return pos(c) * l + neg(c) * r;", "return pos(c) * r + neg(c) * l;"),
    "update_sign": ("out[cell(g, i, j, k)] = vc - div / h[cell(g, i, j, k)];",
                    "out[cell(g, i, j, k)] = vc + div / h[cell(g, i, j, k)];"),
    "upwind_wrong_face": ("c1[xface(g, i + 1, j, k)]);\n                double f2lo",
                          "c1[xface(g, i, j, k)]);\n                double f2lo"),
    "bounds_wrong_neighbour": ("{0, 0, 0},  {-1, 0, 0}, {1, 0, 0}", "{0, 0, 0},  {-1, 0, 0}, {-1, 0, 0}"),
    "bounds_one_field": ("bounds(&g, it, k + 1, mx, mn);", "bounds(&g, it, 1, mx, mn);"),
    "limiter_factors_swapped": ("return fmin(1.0, fmin(bdn_a, bup_b)) * pos(v)",
                                "return fmin(1.0, fmin(bup_a, bdn_b)) * pos(v)"),
    "inflow_sign": ("double in = ((pos(x_lo) - neg(x_hi))", "double in = ((pos(x_lo) + neg(x_hi))"),
    "beta_without_h": ("bup[c] = (mx[c] - pc) * h[c] / (in + eps);", "bup[c] = (mx[c] - pc) / (in + eps);"),
    "mass_drops_errors": ("c = c + (perr + serr);", "c = c + serr;"),
    "vsign_ignored": ("for (long c = 0; c < n; ++c) a1[c] = fabs(cur[c]);",
                      "for (long c = 0; c < n; ++c) a1[c] = cur[c];"),
    "later_pass_keeps_courant": ("        c1 = v[0];\n        c2 = v[1];\n        c3 = v[2];\n", ""),
    "bounds_not_cumulative": ("bounds(&g, it, k + 1, mx, mn);",
                              "const double *two[2] = {psi, cur};\n            bounds(&g, two, 2, mx, mn);"),
    "div_term_sign": ("if (div) V = V - 0.25 * (U / G) * dv;", "if (div) V = V + 0.25 * (U / G) * dv;"),
    "div_term_factor": ("if (div) V = V - 0.25 * (U / G) * dv;", "if (div) V = V - 0.5 * (U / G) * dv;"),
    "div_x_face_own_axis_only": (
        """                    dv = ((u1[xface(g, fres(f + 1, g->nx, bc), j, k)] -
                           u1[xface(g, fres(f - 1, g->nx, bc), j, k)]) +""",
        """                    dv = ((u1[xface(g, fres(f + 1, g->nx, bc), j, k)] -
                           u1[xface(g, fres(f - 1, g->nx, bc), j, k)]) + 0.0 * """),
    "tv_term_sign": ("v1[o] = v1[o] + 0.5 * (w1[o] - u1[o]);", "v1[o] = v1[o] - 0.5 * (w1[o] - u1[o]);"),
    "tv_term_factor": ("v1[o] = v1[o] + 0.5 * (w1[o] - u1[o]);", "v1[o] = v1[o] + (w1[o] - u1[o]);"),
    "tv_term_every_pass": ("if (k == 1 && w1)", "if (w1)"),
    "tv_term_no_z": ("v3[o] = v3[o] + 0.5 * (w3[o] - u3[o]);", "v3[o] = v3[o];"),
    "tv_donor_pass_at_end_level": ("donor_cell_pass(&g, psi, u1, u2, u3, h, own[1]);",
                                   "donor_cell_pass(&g, psi, w1 ? w1 : u1, w1 ? w2 : u2, w1 ? w3 : u3, h, own[1]);"),
    "vsign_in_corrective_pass": ("donor_cell_pass(&g, cur, v[0], v[1], v[2], h, own[k + 1]);",
                                 "donor_cell_pass(&g, p->vsign ? a1 : cur, v[0], v[1], v[2], h, own[k + 1]);"),
}


def _checks():
    """Cheap pin checks (names -> callables raising AssertionError)."""
    import json
    golden = json.load(open(os.path.join(pins.GOLDEN, "hand_1d.json")))["cases"]
    out = {}
    for c in golden:
        out["hand_" + c["name"]] = (lambda c=c: pins.test_hand_1d(oracle, c))
    out["fourier"] = lambda: pins.test_donor_cell_fourier_closed_form(oracle, (-0.25, 0.4, -0.3))
    out["order_1d_var_h"] = lambda: pins.test_mpdata_is_second_order_1d(oracle, 0.3)
    out["order_oblique"] = lambda: pins.test_mpdata_is_second_order_oblique(oracle, (0.3, 0.2, 0.0))
    out["positivity_periodic"] = lambda: pins.test_positivity_and_no_new_extrema(oracle, 0)
    out["bounds_brute_force"] = lambda: pins.test_bounds_are_the_7_point_extrema(oracle)
    out["mass_exact"] = lambda: pins.test_mass_sum_is_exact_to_rounding(oracle)
    out["mass_periodic"] = lambda: pins.test_mass_is_conserved_periodic(oracle)
    out["hand_limiter_variable_h"] = _limiter_variable_h
    out["vsign_positive"] = lambda: pins.test_vsign_is_the_default_scheme_on_positive_fields(oracle)
    out["vsign_odd"] = lambda: pins.test_vsign_odd_symmetry_bitwise(oracle)
    out["vsign_wave"] = lambda: pins.test_vsign_advects_a_sign_changing_wave(oracle)
    out["iord3_bounds"] = lambda: pins.test_more_passes_bound_over_every_iterate(oracle)
    out["iord3_error_1d"] = lambda: pins.test_a_second_pass_reduces_the_error_1d(oracle, 0.0)
    out["div_hand"] = lambda: pins.test_divergence_term_by_hand(oracle)
    out["div_order_1d"] = lambda: pins.test_divergence_term_restores_second_order_1d(oracle, 2)
    out["div_2d"] = lambda: pins.test_divergence_term_transverse_parts_2d(oracle)
    out["tv_hand"] = lambda: pins.test_time_term_by_hand(oracle)
    out["tv_order_1d"] = lambda: pins.test_time_term_restores_second_order_1d(oracle, 0.0)
    out["tv_order_3d"] = lambda: pins.test_time_term_second_order_3d(oracle)
    return out


def _limiter_variable_h():
    """With h != 1 the limiter must still keep every step inside the local
    bounds of psi^n and psi1 (beta carries the factor h)."""
    rng = np.random.default_rng(2)
    n = 24
    psi = np.zeros((1, 1, n))
    psi[..., 6:12] = 1.0
    h = rng.uniform(0.25, 0.5, (1, 1, n))
    u1 = np.full((1, 1, n + 1), 0.2)
    for _ in range(6):
        out, st = oracle.step(psi, u1, np.zeros((1, 2, n)), np.zeros((2, 1, n)), h,
                              stages=True)
        assert np.all(out <= st["mx"] + 1e-14) and np.all(out >= st["mn"] - 1e-14)
        psi = out


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = tmp_path / "m.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libm.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-I", os.path.dirname(SRC), "-o", str(lib), str(mutated), "-lm"],
                   check=True)
    saved_lib, saved_path = oracle._lib, oracle._LIB
    failed = []
    try:
        oracle._lib, oracle._LIB = None, str(lib)
        # checks run cheapest first; one failing check is enough
        for cname, fn in _checks().items():
            try:
                fn()
            except (AssertionError, ValueError):
                failed.append(cname)
                break
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path
    assert failed, f"mutant {name} passed every pin"
