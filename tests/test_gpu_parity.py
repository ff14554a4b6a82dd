"""GPU parity: the HIP seaweed path (and the GPU DP baseline) against the CPU
oracle, element by element, bit-exact (integer output, no tolerance).

Every call goes through the C ABI of libwlcs.so via the thin binding; the
oracle is the plain per-window dynamic program.  Sizes span several tiles,
ragged tails, every window class (16/32/64/128/256 capacity, exact and
partial), the label relabelling every 512 windows, all three output-store
paths (16-byte rows, 4-byte rows, bytes), the epilogues and the degenerate
cases.  Full-size configurations are checked on sampled rows the oracle
computes in seconds plus invariants over the whole matrix.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0909_2000_amd as wl
    wl._load()  # raises if libwlcs.so is missing: no fallback
    return wl


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cpu(t):
    return t.cpu().numpy()


def _bitmap_u64(t):
    return _cpu(t).view(np.uint64)


CASES = []
for w in (1, 2, 3, 5, 8, 15, 16, 17, 31, 32, 33, 48, 63, 64, 65, 100, 127, 128):
    CASES.append((w, w + 1, w + 1))      # a single window pair
    CASES.append((w, w + 70, w + 200))   # ragged, several 64-window blocks
    CASES.append((w, w + 131, w + 97))
for w in (129, 200, 255):
    CASES.append((w, w + 5, w + 90))


@pytest.mark.parametrize("w,m,n", CASES)
def test_small_plots_vs_oracle(ctx, oracle_mod, w, m, n):
    _say(f"case w={w} m={m} n={n}")
    g = workloads.rng(1000 + 7 * w + m + n)
    alpha = workloads.DNA if w % 2 else workloads.PROTEIN
    x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
    want = oracle_mod.wlcs(x, y, w)
    got = ctx.plot(x, y, w, alphabet=alpha)["wlcs"]
    np.testing.assert_array_equal(_cpu(got), want)
    got_dp = ctx.plot_dp(x, y, w, alphabet=alpha)["wlcs"]
    np.testing.assert_array_equal(_cpu(got_dp), want)


@pytest.mark.parametrize("tile", [64, 128, 576, 1024, 2048])
def test_tiles_and_relabelling(ctx, oracle_mod, tile):
    # long rows cross many tiles and (for tiles >= 512) the label rebase
    _say(f"tiles tile={tile}")
    g = workloads.rng(2000 + tile)
    for w in (16, 37, 64, 128):
        x, y = workloads.iid(g, 70 + w, workloads.DNA), workloads.iid(g, 3100 + w, workloads.DNA)
        want = oracle_mod.wlcs(x, y, w)
        ctx.set_tile(1, 255, tile)
        try:
            got = _cpu(ctx.plot(x, y, w)["wlcs"])
        finally:
            ctx.set_tile(1, 255, 0)
        np.testing.assert_array_equal(got, want)


_LONG_W_CACHE = {}


def _long_window_case(oracle_mod, w):
    """x of 70 windows (two strip blocks, the second ragged) and y of 4,300
    windows holding mutated copies of x, so the thresholded outputs have dots;
    the oracle's plot of it (computed once per window)."""
    if w not in _LONG_W_CACHE:
        g = workloads.rng(2200 + w)
        x = workloads.iid(g, w + 70, workloads.DNA)
        y = workloads.iid(g, w + 4300, workloads.DNA)
        for k, ys in enumerate((300, 1700, 3900)):
            seg = x[10 * k:10 * k + w].copy()
            hit = g.random(w) < 0.08
            seg[hit] = workloads.iid(g, int(hit.sum()), workloads.DNA)
            y[ys:ys + w] = seg
        _LONG_W_CACHE[w] = (x, y, oracle_mod.wlcs(x, y, w))
    return _LONG_W_CACHE[w]


@pytest.mark.parametrize("w", [129, 160, 200, 255])
@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_long_windows_across_rebases(ctx, oracle_mod, w, tile):
    """Windows of 129..255 (the 256-row class, a chain of four waves per
    strip, whose labels reach 511 + 2w < 1024 just before the first
    relabelling, in every wave of the chain) on rows long enough that
    one tile crosses the relabelling every 512 windows once (1,024-window
    tiles), three times (2,048) or four times (4,096, one evenly split pair of
    2,176): whole plot, bitmap and indel distance against the oracle."""
    _say(f"long windows w={w} tile={tile}")
    x, y, want = _long_window_case(oracle_mod, w)
    thr = (3 * w) // 4
    assert (want >= thr).sum() > 0
    ctx.set_tile(1, 255, tile)
    try:
        got = {k: _cpu(v) for k, v in ctx.plot(x, y, w, threshold=thr, indel=True).items()}
    finally:
        ctx.set_tile(1, 255, 0)
    np.testing.assert_array_equal(got["wlcs"], want)
    np.testing.assert_array_equal(got["indel"].view(np.uint16), oracle_mod.indel(want, w))
    np.testing.assert_array_equal(got["bitmap"].view("<u8"), oracle_mod.dot_bitmap(want, thr))


def test_long_windows_in_a_batch(ctx, oracle_mod):
    """Windows above 128 in a batch leave the persistent kernels for
    single-plot launches on the same stream: with 2,048-window tiles they
    cross three relabellings per tile, beside jobs of every batched class;
    every matrix whole against the oracle."""
    _say("long windows in a batch")
    pairs, specs, wants = [], [], []
    for w in (129, 200, 255):
        x, y, want = _long_window_case(oracle_mod, w)
        pairs.append(ctx.pair(x, y))
        specs.append({"pair": pairs[-1], "w": w})
        wants.append(want)
    g = workloads.rng(2290)
    for w in (16, 40, 64, 100, 128):
        x, y = workloads.iid(g, 90 + w, workloads.DNA), workloads.iid(g, 2500 + w, workloads.DNA)
        pairs.append(ctx.pair(x, y))
        specs.append({"pair": pairs[-1], "w": w})
        wants.append(oracle_mod.wlcs(x, y, w))
    ctx.set_tile(129, 255, 2048)
    try:
        res = ctx.batch(specs)
        got = [_cpu(r["wlcs"]) for r in res]
    finally:
        ctx.set_tile(129, 255, 0)
    for sp, gw, want in zip(specs, got, wants):
        assert gw.shape == want.shape, sp["w"]
        np.testing.assert_array_equal(gw, want, err_msg=f"w={sp['w']}")


@pytest.mark.parametrize("long_tile,short_tile,long_pairs", [
    (1024, 64, 1), (512, 128, 2), (576, 192, 3), (2048, 64, 1), (256, 1024, 4), (640, 64, 99)])
def test_two_tile_lengths(ctx, oracle_mod, long_tile, short_tile, long_pairs):
    """Long tiles for the first tile pairs of every strip block, short ones
    after them (the short region ending in the evenly split last pair; a
    count of long pairs beyond the row is cut to what fits): whole plots
    against the oracle, and equal to the plot with one tile length."""
    _say(f"two tile lengths {long_tile}/{short_tile} x {long_pairs}")
    g = workloads.rng(2100 + long_tile + short_tile + long_pairs)
    for w in (16, 37, 64, 128):
        x, y = workloads.iid(g, 100 + w, workloads.DNA), workloads.iid(g, 4700 + w, workloads.DNA)
        want = oracle_mod.wlcs(x, y, w)
        ctx.set_tiles(1, 255, long_tile, short_tile, long_pairs)
        try:
            got = {k: _cpu(v) for k, v in ctx.plot(x, y, w, threshold=(3 * w) // 4, indel=True).items()}
        finally:
            ctx.set_tile(1, 255, 0)
        np.testing.assert_array_equal(got["wlcs"], want)
        np.testing.assert_array_equal(got["indel"].view(np.uint16), oracle_mod.indel(want, w))
        np.testing.assert_array_equal(got["bitmap"].view("<u8"), oracle_mod.dot_bitmap(want, (3 * w) // 4))


def test_two_tile_lengths_strided_and_score(ctx, oracle_mod):
    """The same tilings through the strided/sparse and the score-plot paths."""
    g = workloads.rng(2150)
    x, y = workloads.iid(g, 400, workloads.DNA), workloads.iid(g, 5200, workloads.DNA)
    w, hx, hy = 48, 3, 2
    want = oracle_mod.wlcs_strided(x, y, w, hx, hy)
    thr = int(np.quantile(want, 0.99))
    ctx.set_tiles(1, 255, 1024, 128, 2)
    try:
        pair = ctx.pair(x, y)
        res = pair.plot_strided(w, hx, hy, threshold=thr, dot_cap=want.size + 1)
        got = _cpu(res["wlcs"])
        import paper_0909_2000_amd as wl
        dots, count = wl.dot_records(res)
        score = _cpu(ctx.score_plot(x, y, 30, step=4)["score"])
    finally:
        ctx.set_tile(1, 255, 0)
    np.testing.assert_array_equal(got, want)
    ref = oracle_mod.dot_list(want, w, thr, hx, hy)
    assert count == ref.size
    np.testing.assert_array_equal(dots.view(np.uint8), ref.view(np.uint8))
    np.testing.assert_array_equal(score, oracle_mod.score_plot(x, y, 30, step=4))


def test_tile_settings_rejected(ctx):
    import paper_0909_2000_amd as wl
    for args in [(1, 255, 100, 64, 1), (1, 255, 1024, 65, 1), (1, 255, 1024, 64, -1), (1, 255, 1 << 16, 64, 1),
                 (0, 255, 1024, 64, 1), (9, 8, 1024, 64, 1)]:
        with pytest.raises(wl.WlcsError) as e:
            ctx.set_tiles(*args)
        assert e.value.status == -1
    ctx.set_tiles(1, 255, 0, 0, 0)  # drops the rules


def test_valu_peak_probe(lib, ctx):
    """The measurement helper the roofline is reported against: packed 16-bit
    element operations per second within a plausible band around the
    published 78.6 T (256 CUs x 64 lanes x 2 x 2.4 GHz), and its argument
    checks."""
    import ctypes
    peak = ctx.measure_valu_peak(500)
    _say(f"measured packed-u16 VALU peak: {peak / 1e12:.1f} T ops/s")
    assert 40e12 < peak < 90e12
    v = ctypes.c_double(0.0)
    for iters in (0, -3, 2_000_000):
        assert lib._load().wlcs_measure_valu_peak(ctx.handle, iters, ctypes.byref(v)) == -1
    assert lib._load().wlcs_measure_valu_peak(ctx.handle, 10, None) == -1


def test_valu_issue_probe(lib, ctx):
    """The issue-rate helper: wave64 VALU instructions per second per SIMD,
    for each kind of stream and one to four waves per SIMD, between one per
    24 cycles and one per cycle of a 2.4 GHz clock; its argument checks."""
    import ctypes
    for kind in ("pk16", "b32", "bitop3", "cell", "cell_xor", "cell_two_xor"):
        rates = [ctx.measure_valu_issue(kind, k, 20000) for k in (1, 2, 3, 4)]
        _say(f"VALU issue {kind}: " + ", ".join(f"{r / 1e6:.0f} M/s" for r in rates))
        assert all(1e8 < r < 2.4e9 for r in rates), (kind, rates)
    v = ctypes.c_double(0.0)
    for kind, k, iters in ((6, 1, 100), (-1, 1, 100), (0, 0, 100), (0, 5, 100), (0, 1, 0), (0, 1, 2_000_000)):
        assert lib._load().wlcs_measure_valu_issue(ctx.handle, kind, k, iters, ctypes.byref(v)) == -1
    assert lib._load().wlcs_measure_valu_issue(ctx.handle, 0, 1, 10, None) == -1


def test_config1_full(ctx, oracle_mod):
    p = workloads.config(1)
    _say("config 1 full")
    want = oracle_mod.wlcs(p.x, p.y, p.w)
    got = _cpu(ctx.plot(p.x, p.y, p.w)["wlcs"])
    assert got.shape == (984, 984)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(_cpu(ctx.plot_dp(p.x, p.y, p.w)["wlcs"]), want)


@pytest.mark.parametrize("pad", [0, 16, 4, 1, 7])
def test_row_strides(lib, ctx, oracle_mod, pad):
    # ld = cols + pad exercises the 16-byte, 4-byte and byte store paths
    import torch
    g = workloads.rng(3000 + pad)
    w = 24
    x, y = workloads.iid(g, 150, workloads.DNA), workloads.iid(g, 400 + 4 * pad, workloads.DNA)
    want = oracle_mod.wlcs(x, y, w)
    rows, cols = want.shape
    ld = cols + pad
    buf = torch.full((rows, ld), 0xEE, dtype=torch.uint8, device="cuda")
    ctx.plot(x, y, w, out=buf[:, :cols])
    got = _cpu(buf)
    np.testing.assert_array_equal(got[:, :cols], want)
    assert np.all(got[:, cols:] == 0xEE)  # nothing written past the row


@pytest.mark.parametrize("pad", [0, 1, 3, 11])
def test_indel_row_strides(ctx, oracle_mod, pad):
    """Indel rows 397 + pad u16 apart: 400 and 408 start 16 bytes apart and
    take each lane's 8-byte stores, 397 and 398 the transposed 2-byte stores.
    Either way every value equals the oracle's 2w - 2 WLCS, the last partial
    block of each row included, and nothing is written past a row."""
    import torch
    g = workloads.rng(3100 + pad)
    for w in (16, 40, 64, 100):
        x, y = workloads.iid(g, 150 + w, workloads.DNA), workloads.iid(g, 397 + w, workloads.DNA)
        want = oracle_mod.wlcs(x, y, w)
        rows, cols = want.shape
        buf = torch.full((rows, cols + pad), -7, dtype=torch.int16, device="cuda")
        res = ctx.plot(x, y, w, threshold=w // 2, indel=True, indel_out=buf[:, :cols])
        got = _cpu(buf)
        np.testing.assert_array_equal(got[:, :cols].view(np.uint16), oracle_mod.indel(want, w))
        assert np.all(got[:, cols:] == -7)
        np.testing.assert_array_equal(_cpu(res["wlcs"]), want)
        np.testing.assert_array_equal(_bitmap_u64(res["bitmap"]), oracle_mod.dot_bitmap(want, w // 2))


@pytest.mark.parametrize("w,thr", [(16, 12), (64, 48), (33, 0), (20, 21)])
def test_epilogues(ctx, oracle_mod, w, thr):
    g = workloads.rng(4000 + w)
    x, y = workloads.iid(g, 200 + w, workloads.DNA), workloads.iid(g, 333 + w, workloads.DNA)
    want = oracle_mod.wlcs(x, y, w)
    for fn in (ctx.plot, ctx.plot_dp):
        res = fn(x, y, w, threshold=thr, indel=True)
        np.testing.assert_array_equal(_cpu(res["wlcs"]), want)
        np.testing.assert_array_equal(_bitmap_u64(res["bitmap"]), oracle_mod.dot_bitmap(want, thr))
        np.testing.assert_array_equal(_cpu(res["indel"]).view(np.uint16), oracle_mod.indel(want, w))
        # epilogues alone, without the plot
        res2 = fn(x, y, w, threshold=thr, indel=True, want_plot=False)
        np.testing.assert_array_equal(_bitmap_u64(res2["bitmap"]), oracle_mod.dot_bitmap(want, thr))
        np.testing.assert_array_equal(_cpu(res2["indel"]).view(np.uint16), oracle_mod.indel(want, w))


@pytest.mark.parametrize("w", [16, 32, 40, 64])
def test_bitmap_threshold_extremes(ctx, oracle_mod, w):
    """Bitmap words built from byte flags (windows of at most 64 letters):
    thresholds at both ends of 0..255 and on either side of the largest value
    w, for classes filled exactly (16, 32, 64) and padded (40 in the 64-row
    class), on two strip blocks (the second ragged) and rows whose last word is
    partial; y holds mutated copies of x windows so values near w occur."""
    g = workloads.rng(4700 + w)
    x = workloads.iid(g, w + 70, workloads.DNA)
    y = workloads.iid(g, w + 301, workloads.DNA)
    for k, ys in enumerate((40, 150, 260)):  # one exact copy, two mutated
        seg = x[20 * k:20 * k + w].copy()
        hit = g.random(w) < 0.05 * k
        seg[hit] = workloads.iid(g, int(hit.sum()), workloads.DNA)
        y[ys:ys + w] = seg
    want = oracle_mod.wlcs(x, y, w)
    assert want.max() == w and (want == w - 1).any() and want.shape[1] % 64 != 0
    for thr in (0, 1, w // 2, w - 1, w, w + 1, 127, 128, 129, 255):
        _say(f"bitmap thresholds w={w} thr={thr}")
        res = ctx.plot(x, y, w, threshold=thr)
        np.testing.assert_array_equal(_cpu(res["wlcs"]), want)
        np.testing.assert_array_equal(_bitmap_u64(res["bitmap"]), oracle_mod.dot_bitmap(want, thr))


def test_bitmap_padding_words(ctx, oracle_mod):
    # cols not a multiple of 64: padding bits of the last word must be 0
    import torch
    g = workloads.rng(4500)
    for cols in (1, 20, 33, 64, 65, 100):
        w = 8
        x, y = workloads.iid(g, 40, workloads.DNA), workloads.iid(g, cols + w, workloads.DNA)
        want = oracle_mod.wlcs(x, y, w)
        words = (cols + 63) // 64
        bm = torch.full((want.shape[0], words), -1, dtype=torch.int64, device="cuda")
        ctx.plot(x, y, w, threshold=3, bitmap_out=bm, want_plot=False)
        np.testing.assert_array_equal(_bitmap_u64(bm), oracle_mod.dot_bitmap(want, 3))


def test_full_range_flag(ctx, oracle_mod):
    g = workloads.rng(5000)
    for w in (1, 9, 64):
        x, y = workloads.iid(g, w + 50, workloads.DNA), workloads.iid(g, w + 77, workloads.DNA)
        want = oracle_mod.wlcs(x, y, w, full_range=True)
        np.testing.assert_array_equal(_cpu(ctx.plot(x, y, w, full_range=True)["wlcs"]), want)
        np.testing.assert_array_equal(_cpu(ctx.plot_dp(x, y, w, full_range=True)["wlcs"]), want)


def test_degenerate(lib, ctx, oracle_mod):
    # empty plots succeed and return empty tensors
    for (m, n, w) in ((5, 10, 5), (10, 5, 5), (0, 0, 1), (3, 3, 4)):
        res = ctx.plot(b"A" * m, b"C" * n, w)
        assert tuple(res["wlcs"].shape) == (max(m - w, 0), max(n - w, 0))
    # one-letter alphabet: every cell matches
    x, y = b"A" * 80, b"A" * 90
    np.testing.assert_array_equal(_cpu(ctx.plot(x, y, 12, alphabet=b"A")["wlcs"]),
                                  np.full((68, 78), 12, dtype=np.uint8))
    # disjoint letters of one alphabet: nothing matches
    np.testing.assert_array_equal(_cpu(ctx.plot(b"AC" * 40, b"GT" * 45, 10)["wlcs"]), 0)
    # x = y: w on the diagonal
    g = workloads.rng(5100)
    x = workloads.iid(g, 300, workloads.PROTEIN)
    d = np.diag(_cpu(ctx.plot(x, x, 77, alphabet=workloads.PROTEIN)["wlcs"]))
    assert np.all(d == 77)
    # the largest alphabet (63 letters; the 64th code pads short windows), at
    # a window length that is padded (20 -> 32 rows) and one that is not (32)
    alpha = bytes(range(40, 103))
    x, y = workloads.iid(g, 200, alpha), workloads.iid(g, 300, alpha)
    for w in (20, 32):
        np.testing.assert_array_equal(_cpu(ctx.plot(x, y, w, alphabet=alpha)["wlcs"]),
                                      oracle_mod.wlcs(x, y, w))
    with pytest.raises(lib.WlcsError) as e:
        ctx.plot(x, y, 20, alphabet=bytes(range(40, 104)))  # 64 letters
    assert e.value.status == -3


def test_errors(lib, ctx):
    with pytest.raises(lib.WlcsError) as e:
        ctx.plot(b"ACGT" * 10, b"ACGN" * 10, 4)
    assert e.value.status == -3
    with pytest.raises(lib.WlcsError) as e:
        ctx.plot(b"ACGT" * 10, b"ACGT" * 10, 0)
    assert e.value.status == -2
    with pytest.raises(lib.WlcsError) as e:
        ctx.plot(b"ACGT" * 10, b"ACGT" * 10, 4, alphabet=b"ACGA")
    assert e.value.status == -3


def _invariants_gpu(t, w, chunk=4096):
    import torch
    rows = t.shape[0]
    for r0 in range(0, rows, chunk):
        d = t[r0:min(r0 + chunk + 1, rows)].to(torch.int16)
        assert int(d.max()) <= w and int(d.min()) >= 0
        if d.shape[0] > 1:
            assert int((d[1:] - d[:-1]).abs().max()) <= 1
        assert int((d[:, 1:] - d[:, :-1]).abs().max()) <= 1
        if d.shape[0] > 1:
            assert int((d[1:, 1:] - d[:-1, :-1]).abs().max()) <= 1


@pytest.mark.parametrize("k", [2, 3])
def test_full_size_sampled(ctx, oracle_mod, k):
    """Configurations 2 and 3 at full size, in the launch the benchmark times:
    sampled whole rows and entries against the oracle, invariants everywhere."""
    import torch
    p = workloads.config(k)
    _say(f"config {k} full size m={p.m} n={p.n} w={p.w}")
    res = ctx.plot(p.x, p.y, p.w, alphabet=p.alphabet, threshold=p.threshold)
    torch.cuda.synchronize()
    W = res["wlcs"]
    rows, cols = W.shape
    assert (rows, cols) == (p.m - p.w, p.n - p.w)
    g = workloads.rng(6000 + k)
    sample_rows = np.unique(np.concatenate([[0, rows - 1, rows // 2],
                                            g.integers(0, rows, 3),
                                            [xs for xs, _ in p.planted[:2]]]))
    want = oracle_mod.wlcs_rows(p.x, p.y, p.w, sample_rows)
    got = _cpu(W[torch.as_tensor(sample_rows, device="cuda")])
    np.testing.assert_array_equal(got, want)
    ii, jj = g.integers(0, rows, 2000), g.integers(0, cols, 2000)
    got_at = _cpu(W[torch.as_tensor(ii, device="cuda"), torch.as_tensor(jj, device="cuda")])
    np.testing.assert_array_equal(got_at, oracle_mod.wlcs_at(p.x, p.y, p.w, ii, jj))
    _invariants_gpu(W, p.w)
    if p.threshold is not None:
        bm = _bitmap_u64(res["bitmap"][torch.as_tensor(sample_rows, device="cuda")])
        np.testing.assert_array_equal(bm, oracle_mod.dot_bitmap(want, p.threshold))
    # planted homologies light up, random background stays low
    xs, ys = p.planted[0]
    assert int(W[xs + 5, ys + 5]) > int(W[xs + 5, (ys + cols // 2) % cols])


def test_symmetry_and_repeat(ctx):
    import torch
    g = workloads.rng(7000)
    x, y = workloads.iid(g, 900, workloads.DNA), workloads.iid(g, 700, workloads.DNA)
    a = ctx.plot(x, y, 40)["wlcs"]
    b = ctx.plot(y, x, 40)["wlcs"]
    assert torch.equal(a, b.t())
    # repeated launches with different tilings are bit-identical
    for tile in (64, 256, 1024):
        ctx.set_tile(1, 255, tile)
        try:
            assert torch.equal(ctx.plot(x, y, 40)["wlcs"], a)
        finally:
            ctx.set_tile(1, 255, 0)
