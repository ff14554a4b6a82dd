"""Pins for the alignment-score oracle (no GPU).

The score is Section 2's alignment score: match 1, mismatch 0, gap -1/2.  The
oracle computes it by its own dynamic program; it is pinned by the paper's
reduction (score = LLCS of the '$'-blown-up strings minus (m + n)/2, checked
through the LCS oracle, a different code path), by brute force over all
alignments of tiny strings, by the paper's blow-up example, and by closed
forms."""
import functools
import itertools
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def blow(s: bytes) -> bytes:
    return b"".join(b"$" + bytes([c]) for c in s)


def brute_score(a: bytes, b: bytes) -> float:
    @functools.lru_cache(maxsize=None)
    def best(p, q):
        if p == len(a):
            return -0.5 * (len(b) - q)
        if q == len(b):
            return -0.5 * (len(a) - p)
        return max(best(p + 1, q + 1) + (1.0 if a[p] == b[q] else 0.0),
                   best(p + 1, q) - 0.5, best(p, q + 1) - 0.5)
    return best(0, 0)


def test_blowup_example_of_the_paper():
    for line in open(os.path.join(HERE, "golden", "dollar_blowup.txt")):
        line = line.split("#")[0].split()
        if line:
            assert blow(line[0].encode()) == line[1].encode()


def test_score_equals_blown_up_lcs_exhaustive(oracle_mod):
    for la in range(0, 5):
        for lb in range(0, 5):
            for a in itertools.product(b"AB", repeat=la):
                for b in itertools.product(b"AB", repeat=lb):
                    a, b = bytes(a), bytes(b)
                    want = oracle_mod.llcs(blow(a), blow(b)) - 0.5 * (la + lb)
                    assert oracle_mod.score(a, b) == want


@pytest.mark.parametrize("alpha", [workloads.DNA, workloads.PROTEIN])
def test_score_random(oracle_mod, alpha):
    g = workloads.rng(301)
    for _ in range(200):
        a = workloads.iid(g, int(g.integers(0, 9)), alpha).tobytes()
        b = workloads.iid(g, int(g.integers(0, 9)), alpha).tobytes()
        s = oracle_mod.score(a, b)
        assert s == brute_score(a, b)
        assert s == oracle_mod.llcs(blow(a), blow(b)) - 0.5 * (len(a) + len(b))


def test_score_closed_forms(oracle_mod):
    g = workloads.rng(302)
    for w in (1, 5, 17):
        a = workloads.iid(g, w, workloads.DNA).tobytes()
        assert oracle_mod.score(a, a) == w
        b = workloads.iid(g, w, workloads.DNA).tobytes()
        assert oracle_mod.score(a, b) >= sum(x == y for x, y in zip(a, b))  # the gapless alignment
        assert oracle_mod.score(a, b"") == -0.5 * w
    assert oracle_mod.score(b"ACAC", b"GTGT") == 0.0


@pytest.mark.parametrize("step", [1, 3, 5])
def test_score_plot_rows_and_step(oracle_mod, step):
    g = workloads.rng(303 + step)
    w = 7
    x, y = workloads.iid(g, 40, workloads.DNA), workloads.iid(g, 33, workloads.DNA)
    plot = oracle_mod.score_plot(x, y, w, step=step)
    assert plot.dtype == np.int8
    rows = (40 - w + step - 1) // step
    assert plot.shape == (rows, 33 - w)
    for r in range(rows):
        i = r * step
        for j in range(0, 33 - w, 5):
            assert plot[r, j] == oracle_mod.score(x[i:i + w].tobytes(), y[j:j + w].tobytes())
    full = oracle_mod.score_plot(x, y, w, step=1)
    np.testing.assert_array_equal(plot, full[::step])
    assert oracle_mod.score_plot(x, y, w, step=step, full_range=True).shape == \
        ((40 - w + 1 + step - 1) // step, 33 - w + 1)
