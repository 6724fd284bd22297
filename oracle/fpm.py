"""Oracle of the paper's model-based partitioning -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the product (the library's
``mpdata_fpm_*`` entry points and ``paper_1507_01265_amd.teams``) never
does, and this module imports nothing from the product.

Plain Python, written from the paper's text (section 3, Theorem 1 and the
condition it states; section 4, Algorithm 1), step by step in the paper's
notation:

* a speed function s(x) gives the speed of a processor on a workload of
  size x; the time of that workload is x / s(x);
* Theorem 1's condition: s(x)/x never increases as x grows; when it holds
  the balanced distribution is optimal;
* Algorithm 1 (p identical processors, workload n, granularity dx, n/p a
  multiple of dx, p even): start from the even share x_l = x_r = n/p; move dx
  at a time from the x_l half of the processors to the x_r half, evaluate
  t = max(x_r/s(x_r), x_l/s(x_l)) and keep the best (x_l, x_r); the printed
  stopping test is garbled (it would stop after one move), so the moves
  continue while x_l keeps at least dx (reading: until x_l - dx < dx).

Speed functions are passed as callables or as dicts {x: s(x)}.
"""
from __future__ import annotations


def _speed(s, x):
    return s(x) if callable(s) else s[x]


def time_of(s, x):
    """Execution time x / s(x) of a workload of size x."""
    return x / _speed(s, x)


def satisfies_theorem1(s, xs):
    """Theorem 1's condition on the sizes xs (ascending): s(x)/x >= s(y)/y
    for every x < y.  Returns (holds, list of violating (x, y) pairs)."""
    bad = []
    for i, x in enumerate(xs):
        for y in xs[i + 1:]:
            if _speed(s, x) / x < _speed(s, y) / y:
                bad.append((x, y))
    return (not bad), bad


def algorithm1(s, n, p, dx):
    """Algorithm 1: returns (x_lopt, x_ropt, t_min)."""
    if p % 2 or n % p or (n // p) % dx:
        raise ValueError("Algorithm 1 needs p even and n/p a multiple of dx")
    x_l = x_r = n // p
    x_lopt = x_ropt = x_l
    t_min = time_of(s, x_l)
    while x_l - dx >= dx:
        x_r += dx
        x_l -= dx
        t = max(time_of(s, x_r), time_of(s, x_l))
        if t < t_min:
            t_min = t
            x_ropt = x_r
            x_lopt = x_l
    return x_lopt, x_ropt, t_min


def best_pair_brute_force(s, n, p, dx):
    """Every split of the odd/even family (half the processors x_l, half
    x_r, x_l + x_r = 2n/p, multiples of dx) timed; the first minimum in
    increasing x_r.  Used to check Algorithm 1 by exhaustion."""
    share = n // p
    best = None
    for x_r in range(share, 2 * share, dx):
        x_l = 2 * share - x_r
        if x_l < dx:
            break
        t = max(time_of(s, x_r), time_of(s, x_l))
        if best is None or t < best[2]:
            best = (x_l, x_r, t)
    return best


def best_split_brute_force(s, n, p, dx):
    """Min over every distribution (x_1..x_p), each a positive multiple of
    dx summing to n, of max_i x_i/s(x_i) (small n and p only)."""
    units = n // dx
    best = [None]

    def rec(i, left, worst):
        if best[0] is not None and worst >= best[0]:
            return
        if i == p - 1:
            if left >= 1:
                w = max(worst, time_of(s, left * dx))
                if best[0] is None or w < best[0]:
                    best[0] = w
            return
        for u in range(1, left - (p - 1 - i) + 1):
            rec(i + 1, left - u, max(worst, time_of(s, u * dx)))

    rec(0, units, 0.0)
    return best[0]
