"""Exact-rational derivation of the golden values of a 4-cell MPDATA line.

Writes ``hand_1d.json``, ``hand_div_1d.json`` and ``hand_tv_1d.json`` beside this file (or, with
``--check``, compares what it derives with them).  Python's ``fractions``
only; nothing here imports the oracle or the library, so the stored values
are independent of both.

The scheme on a periodic line of cells with unit density (h = 1, so the
face density G is 1) and face Courant numbers U_f (face f between cells
f - 1 and f, face N the same face as face 0), from the MPDATA literature the
paper defers to in section 5.2:

* donor-cell pass (Smolarkiewicz 1984): the flux through a face is
  U times the value of the upwind cell; a cell loses the difference of its
  upper and lower face fluxes;
* antidiffusive pseudo-velocity on a line (the cross terms vanish with no
  transverse flow): V = (|U| - U^2/G) (p_b - p_a)/(p_b + p_a), with the
  divergent-flow term -(1/4)(U/G)(U_{f+1} - U_{f-1}) when asked for, and
  with Courant numbers that change over the step (U at its start, W at its
  end) the time-variation term (W - U)/2 in the first corrective pass;
* non-oscillatory limiter (Smolarkiewicz & Grabowski 1990): bounds over the
  3-point neighbourhood of psi^n and every iterate of the step, factors
  beta_up = (mx - p) h / IN and beta_dn = (p - mn) h / OUT from the
  antidiffusive donor fluxes, and the limited velocity
  min(1, beta_dn_a, beta_up_b) pos(V) + min(1, beta_up_a, beta_dn_b) neg(V);
* a further corrective pass (iord 3) repeats the pseudo-velocity, limiter
  and donor-cell pass on the previous pass's result, with the previous
  pass's (limited) velocity in the place of U.

The regularising eps of the ratios is taken in its limit eps -> 0+: a ratio
0/(0 + eps) is 0, and a limiter factor x/(0 + eps) with x > 0 exceeds 1 and
is capped at 1.  The tests compare the oracle (eps = 1e-15) with these values
to 1e-14.
"""
from __future__ import annotations

import json
import os
import sys
from fractions import Fraction as Fr

HERE = os.path.dirname(os.path.abspath(__file__))


def _pos(x):
    return x if x > 0 else Fr(0)


def _neg(x):
    return x if x < 0 else Fr(0)


def _ratio(num, den):
    """num/(den + eps) in the limit eps -> 0+, for den >= 0."""
    if den == 0:
        if num != 0:
            raise ZeroDivisionError("ratio with a zero denominator and a nonzero numerator")
        return Fr(0)
    return num / den


def _capped(num, den):
    """min(1, num/(den + eps)) in the limit eps -> 0+, for num, den >= 0."""
    if den == 0:
        return Fr(1) if num > 0 else Fr(0)
    return min(Fr(1), num / den)


def donor_pass(p, u):
    """One donor-cell pass of the periodic line p with face velocities u
    (len(p) + 1 faces)."""
    n = len(p)
    flux = [u[f] * (p[(f - 1) % n] if u[f] > 0 else p[f % n]) for f in range(n + 1)]
    return [p[i] - (flux[i + 1] - flux[i]) for i in range(n)]


def pseudo_velocity(p, u, div=False):
    """Antidiffusive velocity on faces 0..N of the line p (G = 1)."""
    n = len(p)
    v = []
    for f in range(n + 1):
        a, b = p[(f - 1) % n], p[f % n]
        U = u[f]
        val = (abs(U) - U * U) * _ratio(b - a, b + a)
        if div:
            # centred divergence across face f: the face beyond b minus the
            # face below a (periodic face indices)
            val -= Fr(1, 4) * U * (u[(f + 1) % n] - u[(f - 1) % n])
        v.append(val)
    return v


def limit(p, v, iterates):
    """Limited velocity of the pass that corrects p with v; the bounds run
    over the 3-point neighbourhood of every array in iterates."""
    n = len(p)
    mx = [max(q[(i + d) % n] for q in iterates for d in (-1, 0, 1)) for i in range(n)]
    mn = [min(q[(i + d) % n] for q in iterates for d in (-1, 0, 1)) for i in range(n)]
    fa = [v[f] * (p[(f - 1) % n] if v[f] > 0 else p[f % n]) for f in range(n + 1)]
    bup, bdn = [], []
    for i in range(n):
        lo, hi = fa[i], fa[i + 1]
        inflow = _pos(lo) - _neg(hi)
        outflow = _pos(hi) - _neg(lo)
        bup.append(_capped(mx[i] - p[i], inflow))
        bdn.append(_capped(p[i] - mn[i], outflow))
    out = []
    for f in range(n + 1):
        a, b = (f - 1) % n, f % n
        out.append(min(bdn[a], bup[b]) * _pos(v[f]) + min(bup[a], bdn[b]) * _neg(v[f]))
    return out


def step(p0, u, iord=2, nonos=True, div=False, w=None):
    """One MPDATA step; returns (psi1, [V of each corrective pass before
    limiting], result).  w: the face Courant numbers at the end of the step
    (time-dependent velocity; u holds those at its start): the first
    corrective pass adds (w - u)/2 to every face's pseudo-velocity."""
    its = [list(p0), donor_pass(p0, u)]
    vel, vs = u, []
    for j in range(iord - 1):
        cur = its[-1]
        v = pseudo_velocity(cur, vel, div)
        if w is not None and j == 0:
            v = [v[f] + (w[f] - u[f]) / 2 for f in range(len(v))]
        vs.append(v)
        if nonos:
            v = limit(cur, v, its)
        its.append(donor_pass(cur, v))
        vel = v
    return its[1], vs, its[-1]


def _s(xs):
    return [str(x) for x in xs]


def derive_hand_1d():
    u = [Fr(1, 2)] * 5
    cases = []
    for name, p0 in (("donor_then_corrective", [1, 2, 3, 4]), ("limiter_step", [0, 0, 1, 1])):
        p0 = [Fr(x) for x in p0]
        psi1, vs, psi_nonos = step(p0, u)
        _, _, psi_free = step(p0, u, nonos=False)
        _, vs3, psi3_free = step(p0, u, iord=3, nonos=False)
        _, _, psi3_nonos = step(p0, u, iord=3)
        c = {"name": name, "psi0": _s(p0), "psi1": _s(psi1)}
        if name == "donor_then_corrective":
            c["v1_faces_0_to_4"] = _s(vs[0])
        c.update({"psi_nonos": _s(psi_nonos), "psi_no_limiter": _s(psi_free),
                  "v_pass2_no_limiter_faces_0_to_4": _s(vs3[1]),
                  "psi_iord3_no_limiter": _s(psi3_free), "psi_iord3_nonos": _s(psi3_nonos)})
        cases.append(c)
    return {
        "source": "Exact rational values derived by the committed script tests/golden/derive_1d.py "
                  "(Python fractions, eps taken in its limit 0+) from the donor-cell flux and update "
                  "(Smolarkiewicz 1984), the antidiffusive pseudo-velocity with G = 1 "
                  "(Smolarkiewicz 1984) and the non-oscillatory limiter (Smolarkiewicz & Grabowski "
                  "1990) -- the equations the paper defers to in section 5.2. Grid 4x1x1, periodic, "
                  "u1 = 1/2 on every face, h = 1; the oracle's eps = 1e-15 moves no value by more "
                  "than 1e-14. The iord 3 values add a second corrective pass: its pseudo-velocities "
                  "come from psi_no_limiter (psi^(2)) with the first pass's antidiffusive velocities "
                  "in the place of u1 (G = 1, no cross terms on a line), and its donor-cell fluxes "
                  "update psi^(2). With the limiter the second pass of the first case is inactive "
                  "(every beta > 1 against bounds over psi^0, psi^(1) and psi^(2)); in the second "
                  "case the first pass's limited velocities are all zero, so the second pass has "
                  "nothing to correct.",
        "cases": cases,
    }


def derive_hand_div_1d():
    p0 = [Fr(x) for x in (1, 2, 3, 4)]
    u = [Fr(1, 2), Fr(1, 4), Fr(1, 8), Fr(3, 8), Fr(1, 2)]
    psi1, vs, out = step(p0, u, nonos=False)
    _, vs_d, out_d = step(p0, u, nonos=False, div=True)
    return {
        "source": "Exact rational values derived by the committed script tests/golden/derive_1d.py "
                  "(Python fractions) for the divergent-flow term of the antidiffusive "
                  "pseudo-velocity (Smolarkiewicz 1984; the term -(1/4)(U/G) times the centred "
                  "divergence across the face, G = 1 here): a 4-cell periodic line, h = 1, uneven "
                  "positive face Courant numbers (the flow is divergent), iord 2, no limiter. On a "
                  "line the divergence across face f is U(f+1) - U(f-1). The first-order pass: every "
                  "face flux is U_f times the value of the cell below it. The oracle's eps = 1e-15 "
                  "moves no value by more than 1e-14.",
        "psi0": _s(p0),
        "u1_faces_0_to_4": _s(u),
        "psi1": _s(psi1),
        "without_term": {"v1_faces_0_to_4": _s(vs[0]), "psi": _s(out)},
        "with_term": {"v1_faces_0_to_4": _s(vs_d[0]), "psi": _s(out_d)},
    }


def derive_hand_tv_1d():
    u = [Fr(1, 2)] * 5
    w = [Fr(3, 4), Fr(1, 2), Fr(5, 8), Fr(1, 4), Fr(3, 4)]
    cases = []
    for name, p0 in (("donor_then_corrective", [1, 2, 3, 4]), ("limiter_step", [0, 0, 1, 1])):
        p0 = [Fr(x) for x in p0]
        psi1, vs, psi_free = step(p0, u, nonos=False, w=w)
        _, _, psi_nonos = step(p0, u, nonos=True, w=w)
        _, vs3, psi3_free = step(p0, u, iord=3, nonos=False, w=w)
        cases.append({"name": name, "psi0": _s(p0), "psi1": _s(psi1),
                      "v1_faces_0_to_4": _s(vs[0]), "psi_no_limiter": _s(psi_free),
                      "psi_nonos": _s(psi_nonos),
                      "v_pass2_no_limiter_faces_0_to_4": _s(vs3[1]),
                      "psi_iord3_no_limiter": _s(psi3_free)})
    return {
        "source": "Exact rational values derived by the committed script tests/golden/derive_1d.py "
                  "(Python fractions, eps taken in its limit 0+) for the time-variation term of "
                  "the antidiffusive pseudo-velocity: a 4-cell periodic line, h = 1, face Courant "
                  "numbers u1 = 1/2 at the start of the step and w1 (uneven, face 4 = face 0) at "
                  "its end. The donor-cell pass and the standard pseudo-velocity take u1; the first "
                  "corrective pass adds (w1 - u1)/2 on every face (holding u1 over the step leaves "
                  "the first-order flux (1/2) dt (du/dt) psi, which the term takes back); a second "
                  "corrective pass (iord 3) corrects its own pass and adds nothing. The limiter is "
                  "the one of hand_1d.json.",
        "u1_faces_0_to_4": _s(u),
        "w1_faces_0_to_4": _s(w),
        "cases": cases,
    }


FILES = {"hand_1d.json": derive_hand_1d, "hand_div_1d.json": derive_hand_div_1d,
         "hand_tv_1d.json": derive_hand_tv_1d}


def main(argv):
    check = "--check" in argv
    bad = 0
    for name, fn in FILES.items():
        path = os.path.join(HERE, name)
        data = fn()
        if check:
            with open(path) as f:
                stored = json.load(f)
            ok = stored == data
            print(f"{name}: {'matches' if ok else 'DIFFERS'}")
            bad += not ok
        else:
            with open(path, "w") as f:
                json.dump(data, f, indent=2)
                f.write("\n")
            print(f"wrote {path}")
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
