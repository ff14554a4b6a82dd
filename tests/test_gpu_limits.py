"""GPU: strings of the maximum supported length (WLCS_MAX_LEN = 10^8 letters)
against the oracle on sampled ranges.

At this size the output offsets pass 2^32 bytes, the y tiles run to 10^8
windows (tens of thousands of label rebases per strip), and the plot has 10^8
rows or columns.  The oracle computes sampled blocks of 64 consecutive windows
from the matching slices of the strings (a window pair only reads its own
letters), so every comparison is element by element, bit-exact."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MAX_LEN = 100_000_000


def _say(*a):
    print(*a, flush=True)


def _starts(g, total, k=24, block=64):
    """First, last and k random block starts in [0, total - block]."""
    last = total - block
    return sorted({0, last, *[int(v) for v in g.integers(0, last + 1, size=k)]})


def test_longest_y(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(9100)
    w = 16
    x = workloads.iid(g, 80 + w, workloads.DNA)
    y = workloads.iid(g, MAX_LEN, workloads.DNA)
    y[5_000_000:5_000_000 + 40] = x[10:50]  # one homology, so the threshold has dots
    _say(f"longest y: m={x.size} n={y.size} w={w}")
    ctx = wl.Context(0)
    pair = ctx.pair(x, y)
    thr = 14  # rare between random 16-mers (about one window pair in 10^4)
    res = pair.plot(w, threshold=thr)
    torch.cuda.synchronize()
    S, B = res["wlcs"], res["bitmap"]
    rows, cols = S.shape
    assert (rows, cols) == (x.size - w, y.size - w)
    for j0 in _starts(g, cols):
        want = oracle_mod.wlcs(x, y[j0:j0 + 64 + w], w)
        np.testing.assert_array_equal(S[:, j0:j0 + 64].cpu().numpy(), want)
    for j0 in _starts(g, cols // 64 * 64)[::4]:
        j0 -= j0 % 64  # whole bitmap words
        want = oracle_mod.wlcs(x, y[j0:j0 + 64 + w], w)
        np.testing.assert_array_equal(B[:, j0 // 64].cpu().numpy().view("<u8"),
                                      oracle_mod.dot_bitmap(want, thr)[:, 0])
    # the homology's windows, and every dot agrees with the dense plot
    assert int(S[:, 5_000_000:5_000_000 + 25].max()) == w
    dense_dots = int((S >= thr).sum())
    sp = pair.plot_strided(w, 1, 1, threshold=thr, want_plot=False, dot_cap=dense_dots + 16)
    dots, count = wl.dot_records(sp)
    assert count == dense_dots > 0
    vals = S[torch.as_tensor(dots["i"].astype(np.int64), device="cuda"),
             torch.as_tensor(dots["j"].astype(np.int64), device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(vals, dots["wlcs"])


def test_longest_x(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(9200)
    w = 24
    x = workloads.iid(g, MAX_LEN, workloads.PROTEIN)
    y = workloads.iid(g, 100 + w, workloads.PROTEIN)
    _say(f"longest x: m={x.size} n={y.size} w={w}")
    ctx = wl.Context(0)
    pair = ctx.pair(x, y, alphabet=workloads.PROTEIN)
    S = pair.plot(w, indel=True)
    torch.cuda.synchronize()
    rows, cols = S["wlcs"].shape
    assert (rows, cols) == (x.size - w, y.size - w)
    for i0 in _starts(g, rows):
        want = oracle_mod.wlcs(x[i0:i0 + 64 + w], y, w)
        np.testing.assert_array_equal(S["wlcs"][i0:i0 + 64].cpu().numpy(), want)
        np.testing.assert_array_equal(S["indel"][i0:i0 + 64].cpu().numpy().view(np.uint16),
                                      oracle_mod.indel(want, w))


def test_longest_x_score_plot(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(9300)
    w, step = 100, 997
    x = workloads.iid(g, MAX_LEN, workloads.DNA)
    y = workloads.iid(g, 300 + w, workloads.DNA)
    _say(f"longest x, score plot: m={x.size} n={y.size} w={w} step={step}")
    ctx = wl.Context(0)
    S = ctx.score_plot(x, y, w, step=step)["score"]
    torch.cuda.synchronize()
    rows, cols = S.shape
    assert (rows, cols) == ((x.size - w + step - 1) // step, y.size - w)
    for r in sorted({0, rows - 1, *[int(v) for v in g.integers(0, rows, size=12)]}):
        i = r * step
        want = oracle_mod.score_plot(x[i:i + w], y, w, full_range=True)[0, :cols]
        np.testing.assert_array_equal(S[r].cpu().numpy(), want)
