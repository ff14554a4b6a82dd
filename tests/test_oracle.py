"""Pins for the CPU oracle (runs without a GPU).

The oracle is the plain definition of the alignment plot (Section 2: WLCS(i, j)
for the w-windows starting at i in x and j in y, i < m-w, j < n-w).  These tests
tie it to things other than itself: brute-force subsequence enumeration,
textbook LCS values, closed-form special cases (w = 1 is the classic equality
dot plot of Section 1, x = y puts w on the diagonal, disjoint letters give 0),
invariants any LCS plot satisfies, and an independent indel-distance dynamic
program for the derived indel output.  The last test plants plausible mistakes
in a Python copy of the definition and checks that the pins reject each one.
"""
import itertools
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- brute force
def brute_llcs(a, b) -> int:
    """Largest r such that some r letters of a, kept in order, are a
    subsequence of b (enumeration of subsets; tiny inputs only)."""
    a, b = bytes(a), bytes(b)
    for r in range(len(a), -1, -1):
        for idx in itertools.combinations(range(len(a)), r):
            it = iter(b)
            if all(a[i] in it for i in idx):
                return r
    return 0


def brute_plot(x, y, w, full_range=False):
    x, y = bytes(x), bytes(y)
    rows = max(len(x) - w + (1 if full_range else 0), 0)
    cols = max(len(y) - w + (1 if full_range else 0), 0)
    out = np.zeros((rows, cols), dtype=np.uint8)
    for i in range(rows):
        for j in range(cols):
            out[i, j] = brute_llcs(x[i:i + w], y[j:j + w])
    return out


def indel_dp(a, b) -> int:
    """Insertion/deletion distance by its own dynamic program (no substitutions)."""
    la, lb = len(a), len(b)
    d = [[0] * (lb + 1) for _ in range(la + 1)]
    for p in range(la + 1):
        for q in range(lb + 1):
            if p == 0 or q == 0:
                d[p][q] = p + q
            else:
                best = min(d[p - 1][q] + 1, d[p][q - 1] + 1)
                if a[p - 1] == b[q - 1]:
                    best = min(best, d[p - 1][q - 1])
                d[p][q] = best
    return d[la][lb]


# ---------------------------------------------------------------- LLCS pins
def _hand_values():
    rows = []
    with open(os.path.join(HERE, "golden", "llcs_hand.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                rows.append((line[0], line[1], int(line[2])))
    return rows


@pytest.mark.parametrize("a,b,v", _hand_values())
def test_llcs_hand_values(oracle_mod, a, b, v):
    assert oracle_mod.llcs(a, b) == v
    assert oracle_mod.llcs(b, a) == v


def test_llcs_exhaustive_binary(oracle_mod):
    for la in range(0, 6):
        for lb in range(0, 6):
            for a in itertools.product(b"AB", repeat=la):
                for b in itertools.product(b"AB", repeat=lb):
                    assert oracle_mod.llcs(bytes(a), bytes(b)) == brute_llcs(a, b)


@pytest.mark.parametrize("alphabet", [workloads.DNA, workloads.PROTEIN])
def test_llcs_random_vs_brute(oracle_mod, alphabet):
    g = workloads.rng(11)
    for _ in range(300):
        a = workloads.iid(g, int(g.integers(0, 11)), alphabet)
        b = workloads.iid(g, int(g.integers(0, 11)), alphabet)
        assert oracle_mod.llcs(a, b) == brute_llcs(a, b)


# ---------------------------------------------------------------- plot pins
@pytest.mark.parametrize("seed", range(6))
def test_plot_vs_brute(oracle_mod, seed):
    g = workloads.rng(100 + seed)
    for _ in range(4):
        w = int(g.integers(1, 7))
        m, n = int(g.integers(w, w + 9)), int(g.integers(w, w + 9))
        alpha = [b"AB", workloads.DNA, workloads.PROTEIN][seed % 3]
        x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
        for full in (False, True):
            got = oracle_mod.wlcs(x, y, w, full_range=full)
            want = brute_plot(x, y, w, full_range=full)
            assert got.shape == want.shape == (max(m - w + full, 0), max(n - w + full, 0))
            np.testing.assert_array_equal(got, want)


def test_plot_shape_is_paper_range(oracle_mod):
    # i in 1..m-w and j in 1..n-w: (m-w) x (n-w) entries; the last letter of
    # each string therefore never enters the default plot.
    x, y = b"ACGTACGTAC", b"CGTAGT"
    assert oracle_mod.wlcs(x, y, 3).shape == (7, 3)
    assert oracle_mod.wlcs(x, y, 3, full_range=True).shape == (8, 4)
    assert oracle_mod.wlcs(x, y, 6).shape == (4, 0)
    assert oracle_mod.wlcs(x, y, 7).shape == (3, 0)


def test_w1_is_equality_dot_plot(oracle_mod):
    g = workloads.rng(7)
    x, y = workloads.iid(g, 60, workloads.DNA), workloads.iid(g, 45, workloads.DNA)
    plot = oracle_mod.wlcs(x, y, 1)
    np.testing.assert_array_equal(plot, (x[:-1, None] == y[None, :-1]).astype(np.uint8))


def test_self_diagonal_and_disjoint(oracle_mod):
    g = workloads.rng(8)
    x = workloads.iid(g, 80, workloads.DNA)
    for w in (1, 5, 16):
        plot = oracle_mod.wlcs(x, x, w)
        assert np.all(np.diag(plot) == w)
        assert np.all(plot <= w)
    y = workloads.iid(g, 70, b"EFHIK")
    assert not oracle_mod.wlcs(x, y, 8).any()


def test_single_window_is_textbook_llcs(oracle_mod):
    # m = n = w + 1 leaves one window pair: the LLCS of the two w-prefixes.
    for a, b, v in _hand_values():
        if len(a) == len(b) and len(a) > 0:
            w = len(a)
            plot = oracle_mod.wlcs(a + "A", b + "A", w)
            assert plot.shape == (1, 1) and plot[0, 0] == v


def _invariants(plot, x, y, w):
    assert plot.min() >= 0 and plot.max() <= w
    d = plot.astype(np.int16)
    assert np.abs(np.diff(d, axis=0)).max(initial=0) <= 1
    assert np.abs(np.diff(d, axis=1)).max(initial=0) <= 1
    assert np.abs(d[1:, 1:] - d[:-1, :-1]).max(initial=0) <= 1
    # at least the letters matched position by position (w - Hamming distance)
    rows, cols = plot.shape
    eq = (x[:, None] == y[None, :]).astype(np.int32)
    for i in range(0, rows, max(rows // 7, 1)):
        for j in range(0, cols, max(cols // 7, 1)):
            assert plot[i, j] >= sum(eq[i + t, j + t] for t in range(w))


@pytest.mark.parametrize("w,alpha", [(4, workloads.DNA), (9, workloads.DNA),
                                     (16, workloads.DNA), (12, workloads.PROTEIN)])
def test_plot_invariants_and_symmetry(oracle_mod, w, alpha):
    g = workloads.rng(w)
    x, y = workloads.iid(g, 150, alpha), workloads.iid(g, 131, alpha)
    plot = oracle_mod.wlcs(x, y, w)
    _invariants(plot, x, y, w)
    np.testing.assert_array_equal(oracle_mod.wlcs(y, x, w), plot.T)


def test_rows_and_at_agree_with_plot(oracle_mod):
    g = workloads.rng(9)
    x, y = workloads.iid(g, 120, workloads.DNA), workloads.iid(g, 97, workloads.DNA)
    w = 11
    plot = oracle_mod.wlcs(x, y, w)
    rows = np.array([0, 5, 108, 77])
    np.testing.assert_array_equal(oracle_mod.wlcs_rows(x, y, w, rows), plot[rows])
    ii = g.integers(0, plot.shape[0], 50)
    jj = g.integers(0, plot.shape[1], 50)
    np.testing.assert_array_equal(oracle_mod.wlcs_at(x, y, w, ii, jj), plot[ii, jj])
    # threads do not change the answer
    np.testing.assert_array_equal(oracle_mod.wlcs(x, y, w, nthreads=1), plot)


def test_epilogues(oracle_mod):
    g = workloads.rng(10)
    x, y = workloads.iid(g, 40, workloads.DNA), workloads.iid(g, 150, workloads.DNA)
    w = 6
    plot = oracle_mod.wlcs(x, y, w)
    ind = oracle_mod.indel(plot, w)
    for i in range(0, plot.shape[0], 5):
        for j in range(0, plot.shape[1], 7):
            assert ind[i, j] == indel_dp(bytes(x[i:i + w]), bytes(y[j:j + w]))
    thr = 4
    bm = oracle_mod.dot_bitmap(plot, thr)
    assert bm.shape == (plot.shape[0], (plot.shape[1] + 63) // 64) and bm.dtype == np.uint64
    for i in range(plot.shape[0]):
        for j in range(bm.shape[1] * 64):
            bit = (int(bm[i, j // 64]) >> (j % 64)) & 1
            assert bit == (1 if j < plot.shape[1] and plot[i, j] >= thr else 0)


def test_workload_shapes():
    p = workloads.config(1)
    assert (p.m, p.n, p.w) == (1000, 1000, 16)
    p2 = workloads.config(2, scale=0.1)
    assert p2.w == 64 and p2.threshold == 48 and len(p2.planted) >= 1
    assert set(np.unique(p2.y).tobytes()) <= set(workloads.DNA)
    p3 = workloads.config(3, scale=0.1)
    assert set(np.unique(p3.x).tobytes()) <= set(workloads.PROTEIN)
    # identical seeds give identical strings
    np.testing.assert_array_equal(workloads.config(1).x, p.x)


def test_planted_windows_score_high(oracle_mod):
    # the planted homologies are what the threshold is meant to find
    p = workloads.config(2, scale=0.1)
    xs, ys = p.planted[0]
    vals = oracle_mod.wlcs_at(p.x, p.y, p.w, [xs + 10], [ys + 10])
    rand = oracle_mod.wlcs_at(p.x, p.y, p.w, [xs + 10], [(ys + p.n // 2) % (p.n - p.w - 1)])
    assert vals[0] > rand[0]


# ---------------------------------------------------------------- mutants
def _plot_py(x, y, w, match_bonus=1, mismatch_takes_diag=False, offset=0, full=False,
             swap_xy=False):
    x, y = bytes(x), bytes(y)
    if swap_xy:
        x, y = y, x
    rows = max(len(x) - w + (1 if full else 0), 0)
    cols = max(len(y) - w + (1 if full else 0), 0)
    out = np.zeros((rows, cols), dtype=np.int32)
    for i in range(rows):
        for j in range(cols):
            a, b = x[i + offset:i + offset + w], y[j:j + w]
            L = [[0] * (len(b) + 1) for _ in range(len(a) + 1)]
            for p in range(1, len(a) + 1):
                for q in range(1, len(b) + 1):
                    if a[p - 1] == b[q - 1]:
                        L[p][q] = L[p - 1][q - 1] + match_bonus
                    else:
                        L[p][q] = max(L[p - 1][q], L[p][q - 1],
                                      L[p - 1][q - 1] + (1 if mismatch_takes_diag else 0))
            out[i, j] = L[len(a)][len(b)]
    return out


@pytest.mark.parametrize("mutant", [
    dict(match_bonus=2),            # wrong match score
    dict(mismatch_takes_diag=True),  # mismatch scored like a match
    dict(offset=1),                 # x-window shifted by one
    dict(full=True),                # wrong output range
    dict(swap_xy=True),             # operands transposed
])
def test_pins_reject_mutants(mutant):
    """Each planted mistake must fail at least one pin used above."""
    g = workloads.rng(12)
    x, y = workloads.iid(g, 13, workloads.DNA), workloads.iid(g, 10, workloads.DNA)
    w = 4
    good = _plot_py(x, y, w)
    np.testing.assert_array_equal(good, brute_plot(x, y, w))
    bad = _plot_py(x, y, w, **mutant)
    assert bad.shape != good.shape or np.any(bad != brute_plot(x, y, w))


# ---- O-batch: the same recurrence, 64 y-windows side by side ---------------

def test_batch_equals_scalar_on_the_1k_dna_pair(oracle_mod):
    """The loop-interchanged oracle equals the plain one on the whole
    1,000 x 1,000 DNA plot at w = 16, for any thread count."""
    p = workloads.config(1)
    want = oracle_mod.wlcs(p.x, p.y, p.w)
    np.testing.assert_array_equal(oracle_mod.wlcs_batch(p.x, p.y, p.w), want)
    np.testing.assert_array_equal(oracle_mod.wlcs_batch(p.x, p.y, p.w, nthreads=1), want)
    np.testing.assert_array_equal(oracle_mod.wlcs_batch(p.x, p.y, p.w, nthreads=5), want)


@pytest.mark.parametrize("w", [1, 2, 3, 7, 15, 16, 17, 31, 33, 63, 64, 65, 100, 127, 128, 129, 200, 255])
def test_batch_equals_scalar_on_random_shapes(oracle_mod, w):
    """Every window class, column counts that are and are not multiples of
    the 64 lanes, the full range, selected rows, three alphabets."""
    g = workloads.rng(5000 + w)
    for alpha in (workloads.DNA, workloads.PROTEIN, b"AB"):
        m = w + int(g.integers(1, 40))
        n = w + int(g.choice([1, 63, 64, 65, 127, 130, int(g.integers(1, 300))]))
        x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
        for full in (False, True):
            want = oracle_mod.wlcs(x, y, w, full_range=full)
            np.testing.assert_array_equal(oracle_mod.wlcs_batch(x, y, w, full_range=full), want)
            if want.shape[0] > 2:
                rows = g.choice(want.shape[0], size=min(5, want.shape[0]), replace=False)
                np.testing.assert_array_equal(oracle_mod.wlcs_batch(x, y, w, rows=rows, full_range=full),
                                              want[rows])


def test_batch_degenerate_and_errors(oracle_mod):
    x = workloads.iid(workloads.rng(5300), 40, workloads.DNA)
    assert oracle_mod.wlcs_batch(x, x[:10], 12).shape == (28, 0)
    assert oracle_mod.wlcs_batch(x[:12], x, 12).shape == (0, 28)
    with pytest.raises(ValueError):
        oracle_mod.wlcs_batch(x, x, 8, rows=[40])
    with pytest.raises(ValueError):
        oracle_mod.wlcs_batch(x, x, 0)


def test_full_plot_digests_match_the_scalar_oracle(oracle_mod):
    """The stored per-row digests of the full 50,000 x 50,000 and 30,000 x
    30,000 plots (written by O-batch) agree with the plain dynamic program on
    rows spread over both plots."""
    import hashlib
    import json
    import os
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(gold, "plot_digests.json")) as f:
        recs = {r["config"]: r for r in json.load(f)["plots"]}
    for cfg, rows in ((2, [0, 7777, 24968, 49935]), (3, [0, 15000, 29871])):
        rec = recs[cfg]
        p = workloads.config(cfg)
        with open(os.path.join(gold, rec["row_digests_file"]), "rb") as f:
            raw = f.read()
        assert hashlib.sha256(raw).hexdigest() == rec["row_digests_sha256"]
        want = np.frombuffer(raw, dtype="<u8")
        assert want.size == rec["rows"] == p.m - p.w
        got = oracle_mod.wlcs_rows(p.x, p.y, p.w, rows)
        for r, row in zip(rows, got):
            assert int.from_bytes(hashlib.blake2b(row.tobytes(), digest_size=8).digest(), "little") == want[r]
