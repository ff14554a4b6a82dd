"""Pins for the oracle's step sizes and sparse dot list (runs without a GPU).

Section 3 introduces a step size h: only windows starting at multiples of h
are compared.  Entry (r, c) of the strided plot is WLCS of the x-window at r*hx
and the y-window at c*hy.  The sparse dot plot lists the window pairs whose
WLCS clears the threshold (Section 1) with their indel distance.  Pinned by
brute-force subsequence enumeration at the strided positions, by the plain
plot's entries, by an independent indel-distance program, and by mutants of
the index mapping that the pins must reject.
"""
import numpy as np
import pytest

import workloads
from test_oracle import brute_llcs, indel_dp


def brute_strided(x, y, w, hx, hy, full_range=False):
    x, y = bytes(x), bytes(y)
    rows = max(len(x) - w + (1 if full_range else 0), 0)
    cols = max(len(y) - w + (1 if full_range else 0), 0)
    out = np.zeros((-(-rows // hx), -(-cols // hy)), dtype=np.uint8)
    for r in range(out.shape[0]):
        for c in range(out.shape[1]):
            out[r, c] = brute_llcs(x[r * hx:r * hx + w], y[c * hy:c * hy + w])
    return out


@pytest.mark.parametrize("hx,hy", [(1, 1), (2, 1), (1, 3), (3, 2), (5, 7), (40, 40)])
def test_strided_vs_brute(oracle_mod, hx, hy):
    g = workloads.rng(100 + 7 * hx + hy)
    x, y = workloads.iid(g, 19, workloads.DNA), workloads.iid(g, 23, workloads.DNA)
    for w in (3, 5):
        for full in (False, True):
            got = oracle_mod.wlcs_strided(x, y, w, hx, hy, full_range=full)
            np.testing.assert_array_equal(got, brute_strided(x, y, w, hx, hy, full))


def test_strided_is_the_plots_entries(oracle_mod):
    g = workloads.rng(5)
    x, y = workloads.iid(g, 260, workloads.PROTEIN), workloads.iid(g, 301, workloads.PROTEIN)
    w = 24
    full = oracle_mod.wlcs(x, y, w)
    for hx, hy in [(1, 1), (2, 2), (5, 1), (1, 5), (7, 3), (236, 1), (1, 277), (1000, 1000)]:
        got = oracle_mod.wlcs_strided(x, y, w, hx, hy)
        assert got.shape == (-(-full.shape[0] // hx), -(-full.shape[1] // hy))
        np.testing.assert_array_equal(got, full[::hx, ::hy])


def test_strided_degenerate(oracle_mod):
    x = y = b"ACGTACGT"
    assert oracle_mod.wlcs_strided(x, y, 8, 3, 3).shape == (0, 0)       # m - w = 0 windows
    assert oracle_mod.wlcs_strided(x, y, 8, 3, 3, full_range=True).tolist() == [[8]]
    with pytest.raises(ValueError):
        oracle_mod.wlcs_strided(x, y, 4, 0, 1)


@pytest.mark.parametrize("hx,hy,thr", [(1, 1, 4), (2, 3, 3), (4, 1, 5), (1, 1, 0), (3, 3, 99)])
def test_dot_list_vs_brute(oracle_mod, hx, hy, thr):
    g = workloads.rng(31 + hx + thr)
    x = workloads.iid(g, 21, workloads.DNA)
    y = np.concatenate([x[3:15], workloads.iid(g, 9, workloads.DNA)])  # some high-scoring pairs
    w = 6
    plot = brute_strided(x, y, w, hx, hy)
    dots = oracle_mod.dot_list(oracle_mod.wlcs_strided(x, y, w, hx, hy), w, thr, hx, hy)
    want = [(r * hx, c * hy) for r in range(plot.shape[0]) for c in range(plot.shape[1]) if plot[r, c] >= thr]
    assert [(int(d["i"]), int(d["j"])) for d in dots] == want
    for d in dots:
        a, b = bytes(x[d["i"]:d["i"] + w]), bytes(y[d["j"]:d["j"] + w])
        assert d["wlcs"] == brute_llcs(a, b)
        assert d["indel"] == indel_dp(a, b)
        assert d["wlcs"] >= thr


def test_dot_record_layout(oracle_mod):
    # the record the library writes: uint32 i, uint32 j, uint16 wlcs, uint16 indel
    assert oracle_mod.DOT.itemsize == 12
    assert [oracle_mod.DOT.fields[k][1] for k in ("i", "j", "wlcs", "indel")] == [0, 4, 8, 10]


def _strided_py(x, y, w, hx, hy, swap_steps=False, row_step_on_y=False):
    x, y = bytes(x), bytes(y)
    rows, cols = len(x) - w, len(y) - w
    if swap_steps:
        hx, hy = hy, hx
    out = np.zeros((-(-rows // hx), -(-cols // hy)), dtype=np.int32)
    for r in range(out.shape[0]):
        for c in range(out.shape[1]):
            i = r * hx
            j = c * (hx if row_step_on_y else hy)
            out[r, c] = brute_llcs(x[i:i + w], y[j:j + w]) if j + w <= len(y) else -1
    return out


@pytest.mark.parametrize("mutant", [dict(swap_steps=True), dict(row_step_on_y=True)])
def test_pins_reject_index_mutants(mutant):
    g = workloads.rng(8)
    x, y = workloads.iid(g, 17, workloads.DNA), workloads.iid(g, 16, workloads.DNA)
    w, hx, hy = 4, 3, 2
    good = _strided_py(x, y, w, hx, hy)
    np.testing.assert_array_equal(good, brute_strided(x, y, w, hx, hy))
    bad = _strided_py(x, y, w, hx, hy, **mutant)
    assert bad.shape != good.shape or np.any(bad != good)
