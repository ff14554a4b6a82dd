"""GPU: alignment-score plots (match 1, mismatch 0, gap -1/2, vertical step)
against the score oracle, bit-exact, including the shape of the paper's
experiments (w = 100, step 5) on a synthetic 80,000 x 80,000 DNA pair."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    import paper_0909_2000_amd as wl
    wl._load()
    return wl.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# windows across the classes of the blown-up strip (2w rows, classes of 8
# rows = 4 pair slots, up to 256 rows), every count of unused top pairs from 0
# to 3 in small and large classes, and the register-budget boundaries (64 and
# 128 rows)
CASES = ([(w, step) for w in (1, 2, 5, 8, 16, 31, 32, 50, 64, 100, 127) for step in (1, 5)] + [(7, 3), (64, 2)]
         + [(w, 1) for w in (3, 4, 6, 9, 10, 11, 17, 33, 40, 48, 49, 65, 70, 80, 81, 90, 96, 97, 99, 101, 102,
                             112, 113, 125, 126)])


@pytest.mark.parametrize("w,step", CASES)
def test_small_score_plots(ctx, oracle_mod, w, step):
    _say(f"score case w={w} step={step}")
    g = workloads.rng(400 + 3 * w + step)
    alpha = workloads.PROTEIN if w % 2 else workloads.DNA
    x, y = workloads.iid(g, w + 90, alpha), workloads.iid(g, w + 150, alpha)
    want = oracle_mod.score_plot(x, y, w, step=step)
    thr = (w + 1) // 3
    res = ctx.score_plot(x, y, w, step=step, alphabet=alpha, threshold=thr)
    np.testing.assert_array_equal(res["score"].cpu().numpy(), want)
    np.testing.assert_array_equal(res["bitmap"].cpu().numpy().view(np.uint64), oracle_mod.dot_bitmap(want, thr))


def test_score_full_range_strides_and_thresholds(ctx, oracle_mod):
    import torch
    g = workloads.rng(450)
    w = 20
    x, y = workloads.iid(g, 123, workloads.DNA), workloads.iid(g, 301, workloads.DNA)
    want = oracle_mod.score_plot(x, y, w, step=4, full_range=True)
    rows, cols = want.shape
    for pad in (0, 1, 16):
        buf = torch.full((rows, cols + pad), 99, dtype=torch.int8, device="cuda")
        ctx.score_plot(x, y, w, step=4, full_range=True, out=buf[:, :cols])
        got = buf.cpu().numpy()
        np.testing.assert_array_equal(got[:, :cols], want)
        assert np.all(got[:, cols:] == 99)
    for thr in (-128, -w, 0, w, 127):
        bm = ctx.score_plot(x, y, w, step=4, full_range=True, threshold=thr, want_plot=False)["bitmap"]
        np.testing.assert_array_equal(bm.cpu().numpy().view(np.uint64), oracle_mod.dot_bitmap(want, thr))


def test_score_errors(ctx):
    import paper_0909_2000_amd as wl
    with pytest.raises(wl.WlcsError):
        ctx.score_plot(b"ACGT" * 50, b"ACGT" * 50, 128)
    with pytest.raises(wl.WlcsError):
        ctx.score_plot(b"ACGT" * 50, b"ACGT" * 50, 10, step=0)
    with pytest.raises(wl.WlcsError):
        ctx.score_plot(bytes(range(64)) * 3, bytes(range(64)) * 3, 10, alphabet=bytes(range(64)))


def test_paper_shaped_score_plot_sampled(ctx, oracle_mod):
    """w = 100 and a vertical step of 5 as in the paper's experiments, on a
    synthetic 80,000 x 80,000 DNA pair: sampled rows against the oracle."""
    import torch
    g = workloads.rng(460)
    m = n = 80_000
    x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
    w, step = 100, 5
    _say("paper-shaped score plot 80k x 80k, w=100, step 5")
    res = ctx.score_plot(x, y, w, step=step)
    torch.cuda.synchronize()
    S = res["score"]
    rows, cols = S.shape
    assert (rows, cols) == ((m - w + step - 1) // step, n - w)
    for r in (0, rows // 2, rows - 1):
        i = r * step
        want = oracle_mod.score_plot(x[i:i + w], y, w, step=1, full_range=True)[0, :cols]
        np.testing.assert_array_equal(S[r].cpu().numpy(), want)
    d = S.to(torch.int16)
    assert int(d.max()) <= w and int(d.min()) >= -w


@pytest.mark.parametrize("w,tile", [(12, 64), (40, 128), (100, 576), (99, 320), (126, 1024)])
def test_score_across_tiles_and_relabelling(ctx, oracle_mod, w, tile):
    """Long rows (many tiles, the ragged last pair, label rebases every 512
    windows of the blown-up strings) against the oracle on sampled rows."""
    import paper_0909_2000_amd as wl
    g = workloads.rng(480 + w)
    x, y = workloads.iid(g, w + 70, workloads.DNA), workloads.iid(g, 2 * w + 1700, workloads.DNA)
    c = wl.Context(0)
    c.set_tile(1, 255, tile)
    res = c.score_plot(x, y, w, step=3)["score"].cpu().numpy()
    rows = res.shape[0]
    for r in sorted({0, rows // 2, rows - 1}):
        want = oracle_mod.score_plot(x[3 * r:3 * r + w], y, w, full_range=True)[0, :res.shape[1]]
        np.testing.assert_array_equal(res[r], want)
