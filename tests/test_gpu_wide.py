"""GPU parity of the 256-row class (windows of 129..255 letters), which runs
every strip as a chain of four waves, each holding a run of 8-row blocks of
the padded strip: every window length from 129 to 255 (each one a split of
the rows over the chain of its own) against the oracle, with the bitmap and
the indel distance, on two strip blocks (the second ragged) and several tile
pairs (the last one ragged); and the strided and sparse variant of the chain
(steps on x and y, the dot list) on every fourth length."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _pair(w, m, n):
    """x, y with two copies of x windows in y (one exact, one mutated), so
    values up to w occur (n >= 2 w + 25)."""
    g = workloads.rng(9100 + w)
    alpha = workloads.PROTEIN if w % 2 else workloads.DNA
    x = workloads.iid(g, m, alpha)
    y = workloads.iid(g, n, alpha)
    y[5:5 + w] = x[3:3 + w]
    seg = x[m - w - 1:m - 1].copy()
    hit = g.random(w) < 0.05
    seg[hit] = workloads.iid(g, int(hit.sum()), alpha)
    y[w + 20:2 * w + 20] = seg
    return x, y, alpha


@pytest.fixture(scope="module")
def ctx():
    import paper_0909_2000_amd as wl
    c = wl.Context(0)
    c.set_tile(129, 255, 64)  # several tile pairs per row, the last one ragged
    yield c
    c.set_tile(129, 255, 0)


@pytest.mark.parametrize("w", list(range(129, 256)))
def test_every_wide_window_vs_oracle(ctx, oracle_mod, w):
    m, n = w + 70, 2 * w + 100
    x, y, alpha = _pair(w, m, n)
    thr = (3 * w + 3) // 4
    print(f"wide w={w} m={m} n={n} thr={thr}", flush=True)
    want = oracle_mod.wlcs(x, y, w)
    assert want.max() == w
    res = ctx.plot(x, y, w, alphabet=alpha, threshold=thr, indel=True)
    np.testing.assert_array_equal(res["wlcs"].cpu().numpy(), want)
    np.testing.assert_array_equal(res["bitmap"].cpu().numpy().view("<u8"), oracle_mod.dot_bitmap(want, thr))
    np.testing.assert_array_equal(res["indel"].cpu().numpy().view(np.uint16), oracle_mod.indel(want, w))


@pytest.mark.parametrize("w", list(range(129, 256, 4)))
def test_wide_strided_and_dots_vs_oracle(ctx, oracle_mod, w):
    import paper_0909_2000_amd as wl
    hx, hy = 2 + w % 3, 1 + w % 2
    m, n = w + 160, 2 * w + 200
    x, y, alpha = _pair(w, m, n)
    want = oracle_mod.wlcs_strided(x, y, w, hx, hy)
    thr = int(np.quantile(want, 0.99))
    print(f"wide strided w={w} hx={hx} hy={hy} thr={thr}", flush=True)
    pair = ctx.pair(x, y, alphabet=alpha)
    res = pair.plot_strided(w, hx, hy, threshold=thr, indel=True, dot_cap=want.size + 1)
    np.testing.assert_array_equal(res["wlcs"].cpu().numpy(), want)
    np.testing.assert_array_equal(res["indel"].cpu().numpy().view(np.uint16), oracle_mod.indel(want, w))
    dots, count = wl.dot_records(res)
    ref = oracle_mod.dot_list(want, w, thr, hx, hy)
    assert count == ref.size > 0
    np.testing.assert_array_equal(dots.view(np.uint8), ref.view(np.uint8))
    pair.close()
