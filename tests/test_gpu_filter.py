"""GPU: the exact threshold filter for dot lists (wlcs_pair_dots_filtered).

The filter combs only every h-th strip (and the last one) at a lowered
threshold and evaluates the rows those probes leave within reach (the plot
moves by at most one per row).  Its dot list must be exactly the oracle's:
the same set of (i, j, WLCS, indel distance) records and the same count, for
windows of every class, probe steps from 1 to beyond the number of rows,
thresholds from low (most window pairs are dots) to high, the full window
range, and a probe list too short for the probe entries (the gated fallback
then lists every strip).  At full size, the 50,000 x 50,000 DNA pair's list at
WLCS >= 48 equals the plain dot list of every strip."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_0909_2000_amd as wl
    return wl.Context(0)


def _planted(seed, w, m, n, alpha=workloads.DNA):
    g = workloads.rng(seed)
    x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
    for k in range(3):
        a, b = 40 + k * (m // 3), 60 + k * (n // 3)
        if a + 2 * w <= m and b + 2 * w <= n:
            seg = x[a:a + 2 * w].copy()
            hit = g.random(seg.size) < 0.08
            seg[hit] = workloads.iid(g, int(hit.sum()), alpha)
            y[b:b + 2 * w] = seg
    return x, y


def _check(ctx, oracle_mod, x, y, w, T, h, alpha=workloads.DNA, full=False, probe_cap=0):
    import paper_0909_2000_amd as wl
    plot = oracle_mod.wlcs(x, y, w, full_range=full)
    want = oracle_mod.dot_list(plot, w, T)
    pair = ctx.pair(x, y, alphabet=alpha)
    res = pair.dots_filtered(w, T, probe_step=h, probe_cap=probe_cap, dot_cap=max(1, want.size),
                             full_range=full)
    got, count = wl.dot_records(res)
    assert count == want.size, (w, T, h, count, want.size)
    np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))
    pair.close()
    return want.size


@pytest.mark.parametrize("w,T", [(16, 12), (40, 29), (64, 48), (100, 72), (128, 92), (200, 140)])
@pytest.mark.parametrize("h", [1, 2, 3, 4, 8, 13])
def test_filtered_dots_equal_the_oracle(ctx, oracle_mod, w, T, h):
    print(f"filter w={w} T={T} h={h}", flush=True)
    x, y = _planted(8000 + w + h, w, w + 300, w + 1700)
    assert _check(ctx, oracle_mod, x, y, w, T, h) > 0


@pytest.mark.parametrize("T", [0, 5, 9, 16])
def test_low_and_extreme_thresholds(ctx, oracle_mod, T):
    """T = 0 makes every window pair a dot; 16 = w only exact copies."""
    x, y = _planted(8100 + T, 16, 180, 700)
    for h in (1, 4, 7):
        _check(ctx, oracle_mod, x, y, 16, T, h)


def test_protein_full_range_and_steps_beyond_the_rows(ctx, oracle_mod):
    x, y = _planted(8200, 32, 32 + 90, 32 + 900, workloads.PROTEIN)
    for h, full in ((5, True), (89, False), (90, True), (400, False)):
        _check(ctx, oracle_mod, x, y, 32, 20, h, alpha=workloads.PROTEIN, full=full)


def test_short_probe_list_falls_back_to_every_strip(ctx, oracle_mod):
    """A probe list of one record overflows: nothing is listed from the probes
    and the gated launch lists every strip; the result is the same."""
    x, y = _planted(8300, 24, 24 + 400, 24 + 1500)
    for h in (4, 6):
        _check(ctx, oracle_mod, x, y, 24, 18, h, probe_cap=1)


def test_full_size_dna_pair_equals_the_plain_dot_list(ctx):
    """The 50,000 x 50,000 DNA pair at w = 64, WLCS >= 48: the filtered list
    at several probe steps equals the plain dot list of every strip (the
    plain path's plot is checked whole against the oracle elsewhere)."""
    import torch
    import paper_0909_2000_amd as wl
    p = workloads.config(2)
    pair = ctx.pair(p.x, p.y)
    cap = 4 << 20
    plain = pair.plot_strided(p.w, 1, 1, threshold=p.threshold, want_plot=False, dot_cap=cap)
    want, n_want = wl.dot_records(plain)
    assert 0 < n_want <= cap
    for h in (2, 4, 6, 8):
        print(f"full-size filter h={h}", flush=True)
        res = pair.dots_filtered(p.w, p.threshold, probe_step=h, dot_cap=cap)
        got, n_got = wl.dot_records(res)
        assert n_got == n_want, (h, n_got, n_want)
        np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))
    pair.close()
    torch.cuda.synchronize()
