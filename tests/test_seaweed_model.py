"""Host-side models of the seaweed method, checked against the oracle (no GPU).

These pin the readings of the paper that the HIP kernels are built on, with
tiny pure-Python models that share nothing with either the oracle or the
kernels:

* the combing rule of the seaweed algorithm (Section 2, Algorithm 1, whose
  figures are lost: the rule is read from the prose): seaweeds start at the
  top of every column and the left of every row; in a match cell the two
  seaweeds turn, in a mismatch cell they cross unless they have crossed
  before.  Labelled by start column (left starts lowest), a mismatch cell sends
  the larger label down and the smaller one right;
* Theorem 2.1 in its string-substring form: LLCS(x, y[a:b]) equals b - a minus
  the number of seaweeds that start and end inside columns [a, b);
* Theorem 3.1's window count: WLCS(j) = w - d(j), with d(j) the seaweeds that
  start and leave the bottom within window j; the count is kept with a ring of
  pending start marks, O(1) per column;
* the relabelling freedom the kernels use: restarting the combing at any
  column, and clamping labels that are older than every open window (the bit
  bound of Propositions 3.3 and 3.4), leave every count unchanged;
* the branch-free cell form of the kernels: with Z = 0 on a match and Z at
  least every label on a mismatch, bottom = max(s, min(t, Z)) and
  right = s xor t xor bottom;
* the padding rows of the kernels: rows of a letter that y never holds, put on
  top of the strip, let every seaweed from the top pass straight down, so the
  padded strip has exactly the exits of the strip itself;
* the score-plot schedule: in strings blown up with a separator before every
  letter (Section 2's reduction of the alignment score), a separator column
  reduces to one max and one min per (separator row, letter row) pair taken
  bottom-up, and a letter column to a mismatch min/max on the separator row
  followed by the general cell; the kernels' form of it, with up to 15 unused
  pairs skipped at the top of the strip, gives the same exits.
"""
import itertools
import re

import numpy as np
import pytest

import workloads

LEFT = -1  # every seaweed entering from the left boundary; below all top labels


def comb(xw, y, start=0):
    """Comb one strip (rows xw, columns y[start:]) and return, per column l,
    the start label of the seaweed leaving its bottom, plus the labels in flight
    to the right after every column."""
    w = len(xw)
    h = [LEFT] * w
    exits, flight = [], []
    for l in range(start, len(y)):
        t = l
        for k in range(w):
            s = h[k]
            if xw[k] == y[l]:
                h[k], t = t, s          # match: the seaweeds turn
            else:
                h[k], t = min(s, t), max(s, t)  # cross unless crossed already
        exits.append(t)
        flight.append(list(h))
    return exits, flight


def plot_by_count(x, y, w, full=False):
    """Whole plot from per-strip combing and the sliding count."""
    rows = max(len(x) - w + (1 if full else 0), 0)
    cols = max(len(y) - w + (1 if full else 0), 0)
    out = np.zeros((rows, cols), dtype=np.uint8)
    for i in range(rows):
        exits, _ = comb(x[i:i + w], y)
        for j in range(cols):
            d = sum(1 for l in range(j, j + w) if exits[l] >= j)
            out[i, j] = w - d
    return out


def ring_count(exits, w, ncols):
    """The kernels' O(1)-per-column count: a running total plus a ring of w
    pending marks keyed by start column."""
    ring = [0] * w     # bit p <-> start column (l - w + 1 + p) after the shift
    cur, out = 0, []
    for l in range(len(exits)):
        f = ring[0]                                # mark for start l - w
        ring = ring[1:] + [0]
        p = exits[l] - (l - w + 1)                 # w-1-span of the exit
        valid = exits[l] != LEFT and 0 <= p < w   # left starts never count
        if valid:
            ring[p] = 1
        cur += int(valid) - f
        if l >= w - 1 and l - w + 1 < ncols:
            out.append(w - cur)
    return out


@pytest.mark.parametrize("seed", range(4))
def test_theorem_2_1_all_substrings(oracle_mod, seed):
    g = workloads.rng(200 + seed)
    for _ in range(6):
        w = int(g.integers(1, 7))
        xw = workloads.iid(g, w, workloads.DNA).tobytes()
        y = workloads.iid(g, int(g.integers(1, 14)), workloads.DNA).tobytes()
        exits, _ = comb(xw, y)
        for a in range(len(y) + 1):
            for b in range(a, len(y) + 1):
                inside = sum(1 for l in range(a, b) if exits[l] >= a)
                assert oracle_mod.llcs(xw, y[a:b]) == (b - a) - inside


def test_exits_form_permutation():
    g = workloads.rng(210)
    for _ in range(20):
        w = int(g.integers(1, 9))
        xw = workloads.iid(g, w, b"AB").tobytes()
        y = workloads.iid(g, 30, b"AB").tobytes()
        exits, flight = comb(xw, y)
        tops = [e for e in exits if e != LEFT]
        assert len(set(tops)) == len(tops)
        assert all(e <= l for l, e in enumerate(exits))
        # every seaweed (w from the left, one per column from the top) either
        # left through the bottom or is still in flight at the right edge
        assert sorted(exits + flight[-1]) == [LEFT] * w + list(range(len(y)))


def test_exhaustive_binary_windows(oracle_mod):
    for w in range(1, 4):
        for x in itertools.product(b"AB", repeat=w + 2):
            x = bytes(x)
            for y in itertools.product(b"AB", repeat=w + 3):
                y = bytes(y)
                np.testing.assert_array_equal(plot_by_count(x, y, w), oracle_mod.wlcs(x, y, w))


@pytest.mark.parametrize("w,alpha", [(1, workloads.DNA), (5, workloads.DNA),
                                     (16, workloads.DNA), (9, workloads.PROTEIN)])
def test_count_plot_equals_oracle(oracle_mod, w, alpha):
    g = workloads.rng(220 + w)
    x, y = workloads.iid(g, w + 25, alpha), workloads.iid(g, w + 40, alpha)
    x, y = x.tobytes(), y.tobytes()
    for full in (False, True):
        np.testing.assert_array_equal(plot_by_count(x, y, w, full), oracle_mod.wlcs(x, y, w, full))


@pytest.mark.parametrize("w", [1, 3, 8, 16])
def test_ring_count_equals_direct(oracle_mod, w):
    g = workloads.rng(230 + w)
    x, y = workloads.iid(g, w + 12, workloads.DNA).tobytes(), \
        workloads.iid(g, w + 60, workloads.DNA).tobytes()
    want = oracle_mod.wlcs(x, y, w)
    for i in range(want.shape[0]):
        exits, _ = comb(x[i:i + w], y)
        assert ring_count(exits, w, want.shape[1]) == list(want[i])


@pytest.mark.parametrize("w", [2, 7, 16])
def test_in_flight_formula(oracle_mod, w):
    # after column j+w-1, WLCS(i, j) = number of seaweeds in flight that
    # started at or after column j
    g = workloads.rng(240 + w)
    x, y = workloads.iid(g, w + 5, workloads.DNA).tobytes(), \
        workloads.iid(g, w + 30, workloads.DNA).tobytes()
    want = oracle_mod.wlcs(x, y, w)
    for i in range(want.shape[0]):
        _, flight = comb(x[i:i + w], y)
        got = [sum(1 for v in flight[j + w - 1] if v >= j) for j in range(want.shape[1])]
        assert got == list(want[i])


@pytest.mark.parametrize("w", [3, 8, 16])
def test_tile_restart(oracle_mod, w):
    # combing afresh from column c gives every window that starts at c or later
    g = workloads.rng(250 + w)
    x, y = workloads.iid(g, w + 3, workloads.DNA).tobytes(), \
        workloads.iid(g, 90, workloads.DNA).tobytes()
    want = oracle_mod.wlcs(x, y, w)
    for i in range(want.shape[0]):
        for c in (0, 1, 17, 40):
            exits, _ = comb(x[i:i + w], y, start=c)
            rel = [e - c if e != LEFT else LEFT for e in exits]
            got = ring_count(rel, w, want.shape[1] - c)
            assert got == list(want[i, c:])


def test_label_clamp_is_exact(oracle_mod):
    """Collapsing all labels older than the oldest open window into one value,
    at arbitrary columns, changes no count (monotone relabelling commutes with
    the max/min of the combing rule)."""
    g = workloads.rng(260)
    w = 6
    x, y = workloads.iid(g, 10, workloads.DNA).tobytes(), \
        workloads.iid(g, 120, workloads.DNA).tobytes()
    want = oracle_mod.wlcs(x, y, w)
    for i in range(want.shape[0]):
        xw = x[i:i + w]
        h = [LEFT] * w
        exits = []
        for l in range(len(y)):
            if l % 13 == 0:
                floor = l - w           # starts < floor can no longer count
                h = [v if v >= floor else LEFT for v in h]
            t = l
            for k in range(w):
                s = h[k]
                if xw[k] == y[l]:
                    h[k], t = t, s
                else:
                    h[k], t = min(s, t), max(s, t)
            exits.append(t)
        assert ring_count(exits, w, want.shape[1]) == list(want[i])


def test_clamp_too_tight_fails(oracle_mod):
    """Negative control: clamping labels that an open window still needs
    (floor one column too high) must break some count."""
    g = workloads.rng(261)
    w = 6
    bad_found = False
    for trial in range(20):
        x, y = workloads.iid(g, 10, workloads.DNA).tobytes(), \
            workloads.iid(g, 80, workloads.DNA).tobytes()
        want = oracle_mod.wlcs(x, y, w)
        for i in range(want.shape[0]):
            h = [LEFT] * w
            exits = []
            for l in range(len(y)):
                floor = l - w + 2
                h = [v if v >= floor else LEFT for v in h]
                t = l
                for k in range(w):
                    s = h[k]
                    if x[i + k] == y[l]:
                        h[k], t = t, s
                    else:
                        h[k], t = min(s, t), max(s, t)
                exits.append(t)
            if ring_count(exits, w, want.shape[1]) != list(want[i]):
                bad_found = True
                break
        if bad_found:
            break
    assert bad_found


def _shipped_encoding():
    """The letter encoding, pad code and rebase period as the kernels ship them
    (read from the kernels' header, so a change there fails the pins below
    until they are brought along)."""
    import pathlib
    src = (pathlib.Path(__file__).resolve().parents[1] / "paper_0909_2000_amd" / "csrc" /
           "kernels.hpp").read_text()
    shift = int(re.search(r"constexpr int kCodeShift = (\d+);", src).group(1))
    pad = int(re.search(r"constexpr uint32_t kPadCode = (\d+);", src).group(1))
    rebase = int(re.search(r"constexpr int kRebase = (\d+);", src).group(1))
    # the two code maps, exactly as written there
    assert "f_code(uint32_t c) { return (uint16_t)(c << kCodeShift); }" in src
    assert "g_code(uint32_t c) { return (uint16_t)(((64u - c) & 63u) << kCodeShift); }" in src
    return shift, pad, rebase


def _max_label(w, rebase):
    """Largest label the general schedule gives a seaweed from the top, for
    window w: walk the tile's columns as the kernel does (w - 1 warm-up
    columns, then groups of four columns per four windows, the origin moved to
    window jj - 1 whenever jj is a multiple of the rebase period; the seaweed
    entering the top of column l carries l - origin + 1) over three periods."""
    org, top = -w, 0
    for l in range(w - 1):
        top = max(top, l - org + 1)
    for jj in range(0, 3 * rebase, 4):
        if jj > 0 and jj % rebase == 0:
            org = jj - 1
        for l in range(jj + w - 1, jj + w + 3):
            top = max(top, l - org + 1)
    return top


def test_branch_free_cell_form():
    """The packed-16-bit cell as the kernels ship it: x letters as
    f(a) = a << 10 and y letters as g(b) = ((64 - b) mod 64) << 10 add (mod
    2^16) to Z = 0 iff a == b and to Z >= 1024 otherwise, for all 63 letter
    codes of y against all 64 x codes (the 64th, 63, is the pad code of the
    padding rows, which must match no letter).  Every label stays below 1024
    for every window up to 255 (the largest, 511 + 2w, comes just before the
    first rebase), so bottom = max(s, min(t, Z)) and right = s ^ t ^ bottom is
    the combing rule (match: bottom = s, right = t; mismatch: bottom =
    max(s, t), right = min(s, t)) for every pair of labels that can occur."""
    shift, pad, rebase = _shipped_encoding()
    assert (shift, pad, rebase) == (10, 63, 512)
    a = np.arange(64, dtype=np.int64)[:, None]          # x codes, pad included
    b = np.arange(63, dtype=np.int64)[None, :]          # y letters
    z = ((a << shift) + (((64 - b) & 63) << shift)) & 0xFFFF
    assert np.array_equal(z == 0, a == b)
    assert (z[a[:, 0] == pad] != 0).all()               # the pad code matches no letter
    zmin = int(z[z != 0].min())
    assert zmin == 1 << shift
    top = max(_max_label(w, rebase) for w in range(1, 256))
    assert top == 511 + 2 * 255 and top < zmin
    assert all(_max_label(w, rebase) == 511 + 2 * w for w in (1, 16, 64, 129, 200, 255))
    # the cell identity for every pair of labels up to the largest one, at Z = 0
    # (match) and at the smallest mismatch Z and the largest (worst cases)
    s = np.arange(top + 1, dtype=np.int64)[:, None]
    t = np.arange(top + 1, dtype=np.int64)[None, :]
    for zv in (0, zmin, int(z.max())):
        bottom = np.maximum(s, np.minimum(t, zv))
        right = s ^ t ^ bottom
        if zv == 0:
            assert np.array_equal(bottom, np.broadcast_to(s, bottom.shape))
            assert np.array_equal(right, np.broadcast_to(t, right.shape))
        else:
            assert np.array_equal(bottom, np.maximum(s, t))
            assert np.array_equal(right, np.minimum(s, t))


def test_cell_form_fails_past_the_label_bound():
    """Negative control: a label at the smallest mismatch Z (what a missed
    rebase would produce) breaks the mismatch rule."""
    shift, _, _ = _shipped_encoding()
    zmin = 1 << shift
    s, t = zmin, 5
    bottom = max(s, min(t, zmin))
    right = s ^ t ^ bottom
    assert (bottom, right) == (max(s, t), min(s, t))  # still right at s == Z ...
    s, t = 5, zmin + 1
    bottom = max(s, min(t, zmin))
    assert bottom != max(s, t)                         # ... but not above it


@pytest.mark.parametrize("pad", [1, 7, 15])
def test_padding_rows_are_transparent(oracle_mod, pad):
    """Strips padded on top with rows of a letter absent from y give the same
    exits in every column as the unpadded strip, hence the same plot; a pad
    letter that does occur in y changes them (the check is not vacuous)."""
    g = workloads.rng(600 + pad)
    for w in (5, 9, 16):
        x = workloads.iid(g, w + 20, workloads.DNA).tobytes()
        y = workloads.iid(g, 120, workloads.DNA).tobytes()
        want = oracle_mod.wlcs(x, y, w)
        changed = False
        for i in range(want.shape[0]):
            plain, _ = comb(x[i:i + w], y)
            padded, _ = comb(b"#" * pad + x[i:i + w], y)
            assert padded == plain
            assert ring_count(padded, w, want.shape[1]) == list(want[i])
            matching, _ = comb(b"A" * pad + x[i:i + w], y)
            changed |= matching != plain
        assert changed


def comb_blown_up(letters, yl, cap):
    """The kernels' schedule for blown-up strings ('$' a1 '$' a2 ... against
    '$' b1 '$' b2 ...): cap pair slots, the first cap - len(letters) (< 16)
    unused; returns the exit label of every column."""
    npairs = len(letters)
    pad = cap - npairs
    assert 0 <= pad < 16
    h = [LEFT] * (2 * cap)
    code = [None] * pad + list(letters)
    exits = []
    for l in range(2 * len(yl)):
        if l % 2 == 0:  # separator column: bottom-up pairs, then the new top seaweed
            out = None
            for r in range(cap - 1, -1, -1):
                if r >= pad:
                    a, b = h[2 * r], h[2 * r + 1]
                    if r == cap - 1:
                        out = max(a, b)
                    else:
                        h[2 * r + 2] = max(a, b)
                    h[2 * r + 1] = min(a, b)
                elif r == pad - 1:
                    h[2 * r + 2] = l
            if pad == 0:
                h[0] = l
        else:           # letter column: top-down
            c, out = yl[l // 2], l
            for r in range(pad, cap):
                a = h[2 * r]
                h[2 * r], out = min(a, out), max(a, out)  # separator row: a mismatch
                s_ = h[2 * r + 1]
                if code[r] == c:
                    h[2 * r + 1], out = out, s_
                else:
                    h[2 * r + 1], out = min(s_, out), max(s_, out)
        exits.append(out)
    return exits


def fused_pass(h, code, pad, cap, c, yl_c):
    """One top-down pass through the pair slots combing the separator column
    c - 1 and the letter column c together: at slot r the separator column
    sends max(h[2r], h[2r+1]) to row 2r + 2 (carried to slot r + 1) and keeps
    the min in row 2r + 1, and the letter column then crosses the carried label
    on the separator row and meets its letter on the letter row.

    The unused top slots (r < pad, whose letter matches nothing) run the same
    steps: the letter column's label is the largest of all and passes through
    them unchanged, and after each of them the separator column's carry is
    raised to its top label (larger than anything the slot holds), so both
    columns enter slot pad with their own top labels.  Returns the exits."""
    top = c - 1
    carry, out = top, c
    for r in range(cap):
        yield r
        a, b = h[2 * r], h[2 * r + 1]
        mx, b = max(a, b), min(a, b)
        h[2 * r], d = min(carry, out), max(carry, out)
        if code[r] == yl_c:
            h[2 * r + 1], out = d, b
        else:
            h[2 * r + 1], out = min(b, d), max(b, d)
        carry = max(mx, top) if r < pad else mx
    yield (carry, out)


def comb_blown_up_fused(letters, yl, cap, interleave):
    """The fused schedule: separator column c - 1 and letter column c in one
    pass; with interleave, two such passes (columns c - 1, c and c + 1, c + 2)
    advance together, the second one slot behind the first."""
    npairs = len(letters)
    pad = cap - npairs
    h = [LEFT] * (2 * cap)
    code = [None] * pad + list(letters)
    exits = []
    ncols = 2 * len(yl)
    c = 1
    while c < ncols:
        if interleave and c + 2 < ncols:
            A = fused_pass(h, code, pad, cap, c, yl[c // 2])
            B = fused_pass(h, code, pad, cap, c + 2, yl[(c + 2) // 2])
            ra = next(A)            # A enters its first slot
            rb = None
            while True:
                if not isinstance(ra, tuple):
                    ra = next(A)    # A: one slot down
                if rb is None:
                    rb = next(B)
                elif not isinstance(rb, tuple):
                    rb = next(B)    # B: one slot down, behind A
                if isinstance(ra, tuple) and isinstance(rb, tuple):
                    break
            exits += [ra[0], ra[1], rb[0], rb[1]]
            c += 4
        else:
            res = list(fused_pass(h, code, pad, cap, c, yl[c // 2]))[-1]
            exits += [res[0], res[1]]
            c += 2
    return exits


def fused_slots(h, code, pad, lo, hi, top, carry, out, yl_c):
    """Slots lo .. hi - 1 of one fused pass (see fused_pass), entered with the
    separator column's carry and the letter column's label; returns both as
    they leave slot hi - 1."""
    for r in range(lo, hi):
        a, b = h[2 * r], h[2 * r + 1]
        mx, b = max(a, b), min(a, b)
        h[2 * r], d = min(carry, out), max(carry, out)
        if code[r] == yl_c:
            h[2 * r + 1], out = d, b
        else:
            h[2 * r + 1], out = min(b, d), max(b, d)
        carry = max(mx, top) if r < pad else mx
    return carry, out


@pytest.mark.parametrize("cap,upper", [(16, 8), (32, 20), (32, 4)])
def test_split_blown_up_schedule_equals_combing(cap, upper):
    """The strip split over two waves: the upper slots 0 .. upper - 1 of every
    pass, then (here all at the end, the extreme case of the lower wave's lag)
    the lower slots entered with the labels the upper slots handed over.  The
    lower slots read nothing else from the upper ones, so the exits equal plain
    combing whatever the lag."""
    g = workloads.rng(950 + cap + upper)
    for trial in range(40):
        npairs = int(g.integers(cap - 3, cap + 1))
        letters = bytes(workloads.iid(g, npairs, workloads.DNA))
        yl = bytes(workloads.iid(g, int(g.integers(1, 14)), workloads.DNA))
        pad = cap - npairs
        code = [None] * pad + list(letters)
        h = [LEFT] * (2 * cap)
        handed = []
        for c in range(1, 2 * len(yl), 2):  # upper wave: every pass
            handed.append((c, fused_slots(h, code, pad, 0, upper, c - 1, c - 1, c, yl[c // 2])))
        exits = []
        for c, (carry, out) in handed:     # lower wave: every pass, afterwards
            exits += list(fused_slots(h, code, pad, upper, cap, c - 1, carry, out, yl[c // 2]))
        xb = b"".join(b"$" + bytes([ch]) for ch in letters)
        yb = b"".join(b"$" + bytes([ch]) for ch in yl)
        plain, _ = comb(xb, yb)
        assert exits == plain


@pytest.mark.parametrize("interleave", [False, True])
@pytest.mark.parametrize("cap", [16, 32])
def test_fused_blown_up_schedule_equals_combing(cap, interleave):
    """The fused (and the interleaved fused) score-plot schedule against plain
    combing of the blown-up strings: the same exit for every column."""
    g = workloads.rng(900 + cap + 7 * interleave)
    for trial in range(60):
        npairs = int(g.integers(cap - 15, cap + 1))
        letters = bytes(workloads.iid(g, npairs, workloads.DNA))
        yl = bytes(workloads.iid(g, int(g.integers(1, 14)), workloads.DNA))
        xb = b"".join(b"$" + bytes([c]) for c in letters)
        yb = b"".join(b"$" + bytes([c]) for c in yl)
        plain, _ = comb(xb, yb)
        assert comb_blown_up_fused(letters, yl, cap, interleave) == plain


@pytest.mark.parametrize("cap", [16, 32])
def test_blown_up_schedule_equals_combing(oracle_mod, cap):
    """The score-plot schedule against plain combing of the blown-up strings,
    and its window counts against the score oracle through the blow-up."""
    g = workloads.rng(700 + cap)
    for trial in range(60):
        npairs = int(g.integers(cap - 15, cap + 1))
        letters = bytes(workloads.iid(g, npairs, workloads.DNA))
        yl = bytes(workloads.iid(g, int(g.integers(1, 14)), workloads.DNA))
        xb = b"".join(b"$" + bytes([c]) for c in letters)
        yb = b"".join(b"$" + bytes([c]) for c in yl)
        plain, _ = comb(xb, yb)
        assert comb_blown_up(letters, yl, cap) == plain
    # one window of 2w columns: w - count is LLCS(x', y') and score = LLCS - w
    w = cap - 3
    letters = bytes(workloads.iid(g, w, workloads.DNA))
    yl = bytes(workloads.iid(g, w + 9, workloads.DNA))
    exits = comb_blown_up(letters, yl, cap)
    for j in range(0, 2 * (len(yl) - w) + 1, 2):
        d = sum(1 for l in range(j, j + 2 * w) if exits[l] >= j)
        score2 = 2 * (2 * w - d) - 2 * w
        want = oracle_mod.score(letters, yl[j // 2:j // 2 + w])
        assert score2 == 2 * want
