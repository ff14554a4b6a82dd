"""Host model of the exact probe filter for dot lists, against the oracle (no GPU).

The filter lists the dots (window pairs with WLCS >= T) of a plot without
combing every strip.  It rests on one property of the plot: moving the
x-window by one letter drops one letter and adds one, so the LLCS changes by
at most one, and |WLCS(i + d, j) - WLCS(i, j)| <= |d| (pinned by the oracle's
invariant tests).  So:

* probe rows: every h-th x-window, starting at half the remainder of
  (rows - 1) / h (so the rows before the first probe and after the last are
  no farther from it than any other row), each listed completely at the
  lowered threshold T - floor(h / 2);
* every other row i has a designated nearest probe p (the lower one on ties),
  at most floor(h / 2) rows away; a dot (i, j) implies
  WLCS(p, j) >= T - |i - p| >= T - floor(h / 2), so p lists (p, j);
* candidates: for each listed probe entry (p, j, v), the rows i whose
  designated probe is p with v + |i - p| >= T; each is evaluated exactly.

The model below follows those steps with the oracle's rows and entries and
must give exactly the oracle's dot list; the kernels follow the same steps.
A probe threshold one higher (a plausible off-by-one) must miss dots.
"""
import numpy as np
import pytest

import workloads


def probes(rows: int, h: int) -> list:
    first = ((rows - 1) % h) // 2
    return list(range(first, rows, h))


def nearest_probe(i: int, rows: int, h: int) -> int:
    P = probes(rows, h)
    return min(P, key=lambda p: (abs(i - p), p))  # the nearest, the lower one on ties


def filtered_dots(oracle_mod, x, y, w, T, h, probe_slack=None):
    rows, cols = len(x) - w, len(y) - w
    if rows <= 0 or cols <= 0:
        return set()
    P = probes(rows, h)
    Pset = set(P)
    H = h // 2
    Tp = max(0, T - (H if probe_slack is None else probe_slack))
    prow = oracle_mod.wlcs_rows(x, y, w, P)
    dots = set()
    for p, vals in zip(P, prow):
        for j in np.nonzero(vals >= Tp)[0]:
            v = int(vals[j])
            if v >= T:
                dots.add((p, int(j), v))
            for d in range(-H, H + 1):
                i = p + d
                if d == 0 or not 0 <= i < rows or i in Pset:
                    continue
                if nearest_probe(i, rows, h) != p or v + abs(d) < T:
                    continue
                got = int(oracle_mod.wlcs_at(x, y, w, [i], [int(j)])[0])
                if got >= T:
                    dots.add((i, int(j), got))
    return dots


def oracle_dots(oracle_mod, x, y, w, T):
    plot = oracle_mod.wlcs(x, y, w)
    r, c = np.nonzero(plot >= T)
    return {(int(a), int(b), int(plot[a, b])) for a, b in zip(r, c)}


def _case(seed, w, m, n, planted=True):
    g = workloads.rng(seed)
    x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
    if planted and m > 3 * w and n > 3 * w:
        seg = x[w:3 * w].copy()
        hit = g.random(seg.size) < 0.1
        seg[hit] = workloads.iid(g, int(hit.sum()), workloads.DNA)
        y[n // 3:n // 3 + 2 * w] = seg
    return x, y


def designated_as_the_kernel_computes(i: int, rows: int, h: int) -> int:
    """The candidate kernel's closed form of a row's designated probe."""
    first = ((rows - 1) % h) // 2
    last = first + (rows - 1 - first) // h * h
    if i <= first:
        return first
    if i >= last:
        return last
    lo = first + (i - first) // h * h
    return lo if i - lo <= lo + h - i else lo + h


def test_nearest_probe_is_within_half_a_step():
    for rows in list(range(1, 41)) + [49936, 29872]:
        for h in (1, 2, 3, 4, 5, 6, 7, 8, 12, 50):
            P = probes(rows, h)
            assert all(b - a == h for a, b in zip(P, P[1:]))
            assert P[0] <= h // 2 and rows - 1 - P[-1] <= h // 2
            for i in (range(rows) if rows < 100 else list(range(200)) + list(range(rows - 200, rows))):
                p = nearest_probe(i, rows, h)
                assert abs(i - p) <= h // 2
                assert designated_as_the_kernel_computes(i, rows, h) == p, (rows, h, i)


@pytest.mark.parametrize("h", [1, 2, 3, 4, 5, 8, 13, 200])
@pytest.mark.parametrize("w,T", [(8, 6), (16, 11), (24, 17)])
def test_filter_gives_the_oracles_dot_list(oracle_mod, h, w, T):
    x, y = _case(7000 + 31 * h + w, w, 90 + w, 260 + w)
    want = oracle_dots(oracle_mod, x, y, w, T)
    assert want
    assert filtered_dots(oracle_mod, x, y, w, T, h) == want


def test_probe_threshold_one_too_high_misses_dots(oracle_mod):
    """Negative control: listing probe rows at T - floor(h/2) + 1 loses dots
    whose designated probe sits exactly floor(h/2) rows away."""
    missed = False
    for seed in range(12):
        w, T, h = 12, 9, 4
        x, y = _case(7500 + seed, w, 70 + w, 200 + w)
        want = oracle_dots(oracle_mod, x, y, w, T)
        got = filtered_dots(oracle_mod, x, y, w, T, h, probe_slack=h // 2 - 1)
        assert got <= want
        if got != want:
            missed = True
            break
    assert missed
