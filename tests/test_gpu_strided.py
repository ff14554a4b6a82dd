"""GPU parity of strided and sparse plots (Section 3's step size, Section 1's
dot plot as a list) against the oracle, through the C ABI
(wlcs_pair_plot_strided, wlcs_pair_plot_dp_strided).

Dense outputs are compared element by element with oracle.wlcs_strided.  The
dot list's order is not defined: the test compares the sorted records, which
are unique (one per window pair at or above the threshold), with
oracle.dot_list."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _pair_with_homology(g, m, n, alpha, w):
    """Random strings where y holds two mutated copies of parts of x, so that
    a threshold near the top of the range still has dots."""
    x = workloads.iid(g, m, alpha)
    y = workloads.iid(g, n, alpha)
    for _ in range(2):
        ln = min(3 * w, m // 3, n // 3)
        src = int(g.integers(0, m - ln))
        dst = int(g.integers(0, n - ln))
        seg = x[src:src + ln].copy()
        flip = g.random(ln) < 0.1
        seg[flip] = workloads.iid(g, int(flip.sum()), alpha)
        y[dst:dst + ln] = seg
    return x, y


CASES = [  # (m, n, w, hx, hy, alphabet)
    (700, 900, 16, 1, 3, "dna"),
    (900, 700, 33, 2, 1, "dna"),
    (1300, 1100, 64, 5, 5, "dna"),
    (800, 1500, 64, 3, 7, "protein"),
    (1000, 1000, 100, 5, 2, "dna"),
    (700, 800, 128, 4, 4, "protein"),
    (600, 700, 200, 5, 3, "dna"),
]


@pytest.mark.parametrize("m,n,w,hx,hy,alpha", CASES)
@pytest.mark.parametrize("path", ["seaweed", "dp"])
def test_strided_plot_and_dots_vs_oracle(oracle_mod, m, n, w, hx, hy, alpha, path):
    import torch
    import paper_0909_2000_amd as wl
    A = workloads.DNA if alpha == "dna" else workloads.PROTEIN
    g = workloads.rng(m + 7 * w + hx + 31 * hy)
    x, y = _pair_with_homology(g, m, n, A, w)
    want = oracle_mod.wlcs_strided(x, y, w, hx, hy)
    thr = int(np.quantile(want, 0.995)) if want.size else 0
    print(f"case {path} m={m} n={n} w={w} hx={hx} hy={hy} thr={thr}", flush=True)
    ctx = wl.Context(0)
    pair = ctx.pair(x, y, alphabet=A)
    fn = pair.plot_strided if path == "seaweed" else pair.plot_dp_strided
    res = fn(w, hx, hy, threshold=thr, indel=True, dot_cap=want.size + 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(res["wlcs"].cpu().numpy(), want)
    np.testing.assert_array_equal(res["indel"].cpu().numpy().view(np.uint16), oracle_mod.indel(want, w))
    dots, count = wl.dot_records(res)
    ref = oracle_mod.dot_list(want, w, thr, hx, hy)
    assert count == ref.size > 0
    np.testing.assert_array_equal(dots.view(np.uint8), ref.view(np.uint8))
    if hy == 1:  # the bitmap over the strided grid
        bm = fn(w, hx, 1, threshold=thr, want_plot=False)["bitmap"]
        np.testing.assert_array_equal(bm.cpu().numpy().view("<u8"), oracle_mod.dot_bitmap(want, thr))


@pytest.mark.parametrize("w,hy", [(16, 1), (16, 3), (100, 1), (100, 2)])
def test_dot_lists_at_the_threshold_extremes(oracle_mod, w, hy):
    """Threshold 0 lists every window pair (every lane of every block has
    dots: the wave scan and the per-lane records at full density), threshold
    w only the exact matches, and a threshold above w none at all."""
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(6100 + w + hy)
    x, y = _pair_with_homology(g, 260 + w, 300 + w, workloads.DNA, w)
    want = oracle_mod.wlcs_strided(x, y, w, 2, hy)
    ctx = wl.Context(0)
    pair = ctx.pair(x, y)
    for thr in (0, w, w + 1):
        res = pair.plot_strided(w, 2, hy, threshold=thr, want_plot=False, dot_cap=want.size + 1)
        torch.cuda.synchronize()
        dots, count = wl.dot_records(res)
        ref = oracle_mod.dot_list(want, w, thr, 2, hy)
        assert count == ref.size, (thr, count, ref.size)
        if thr == 0:
            assert count == want.size
        np.testing.assert_array_equal(dots.view(np.uint8), ref.view(np.uint8))


def test_dot_list_capacity_and_count_only(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(9)
    w, hx, hy = 32, 2, 1
    x, y = _pair_with_homology(g, 1200, 1300, workloads.DNA, w)
    want = oracle_mod.wlcs_strided(x, y, w, hx, hy)
    thr = int(np.quantile(want, 0.99))
    ref = oracle_mod.dot_list(want, w, thr, hx, hy)
    assert ref.size > 20
    ctx = wl.Context(0)
    pair = ctx.pair(x, y)
    # a list too short: the count is the whole number, every written record is a true dot
    cap = ref.size // 3
    res = pair.plot_strided(w, hx, hy, threshold=thr, want_plot=False, dot_cap=cap)
    dots, count = wl.dot_records(res)
    assert count == ref.size and dots.size == cap
    refset = {(int(d["i"]), int(d["j"]), int(d["wlcs"]), int(d["indel"])) for d in ref}
    assert {(int(d["i"]), int(d["j"]), int(d["wlcs"]), int(d["indel"])) for d in dots} <= refset
    assert len({(int(d["i"]), int(d["j"])) for d in dots}) == cap  # no record written twice
    # count only
    res = pair.plot_strided(w, hx, hy, threshold=thr, want_plot=False, dot_cap=0)
    torch.cuda.synchronize()
    assert int(res["dot_count"].item()) == ref.size


def test_empty_plot_sets_count_to_zero():
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    pair = ctx.pair(b"ACGTACGT", b"ACGTACGTACGT")
    dots_out = torch.full((4, 3), -1, dtype=torch.int32, device="cuda")
    count = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
    res = pair.plot_strided(8, 2, 2, threshold=1, want_plot=False, dots_out=dots_out,
                            count_out=count)  # m - w = 0 windows
    torch.cuda.synchronize()
    assert res["dot_count"] is count and int(count.item()) == 0
    assert bool((dots_out == -1).all())


def test_strided_errors():
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    pair = ctx.pair(workloads.iid(workloads.rng(1), 300, workloads.DNA),
                    workloads.iid(workloads.rng(2), 300, workloads.DNA))
    with pytest.raises(wl.WlcsError) as e:
        pair.plot_strided(16, 1, 2, threshold=10, bitmap=True)  # bitmap needs hy == 1
    assert e.value.status == -1
    with pytest.raises(wl.WlcsError) as e:
        pair.plot_strided(16, 0, 1)
    assert e.value.status == -2
    with pytest.raises(wl.WlcsError) as e:
        pair.plot_strided(16, 1, 1, want_plot=False)  # nothing asked for
    assert e.value.status == -1
    lib = wl._load()
    dummy = ctypes.c_void_p(1 << 20)  # never dereferenced: rejected on the host first
    st = lib.wlcs_pair_plot_strided(ctx.handle, pair._h, 16, 1, 1, None, 0, None, 0, 10, None, 0,
                                    dummy, 4, None, 0, None)  # a list without a counter
    assert st == -1
    st = lib.wlcs_pair_plot_strided(ctx.handle, pair._h, 16, 1, 1, None, 0, None, 0, 300, None, 0,
                                    None, 0, dummy, 0, None)  # threshold out of range
    assert st == -1


def test_full_size_dna_step5_sampled_rows(oracle_mod):
    """The 50,000 x 50,000 DNA pair with 20 planted homologies, w = 64, at
    the paper's vertical step of 5 and every y-window: sampled strided rows of
    the plot, and the dots of those rows, against the oracle."""
    import torch
    import paper_0909_2000_amd as wl
    p = workloads.config(2)
    w, hx = p.w, 5
    ctx = wl.Context(0)
    pair = ctx.pair(p.x, p.y)
    print("full size: 50k x 50k w=64 hx=5", flush=True)
    res = pair.plot_strided(w, hx, 1, threshold=p.threshold, dot_cap=1 << 20)
    torch.cuda.synchronize()
    rows = res["wlcs"].shape[0]
    assert rows == -(-(p.m - w) // hx)
    dots, count = wl.dot_records(res)
    assert 0 < count <= (1 << 20)
    sample = np.array([0, 1, rows // 3, rows // 2, rows - 1])
    want = oracle_mod.wlcs_rows(p.x, p.y, w, sample * hx)
    np.testing.assert_array_equal(res["wlcs"][torch.as_tensor(sample, device="cuda")].cpu().numpy(), want)
    # dots of the sampled rows
    for r, row in zip(sample, want):
        ref = {(int(r) * hx, int(j)) for j in np.nonzero(row >= p.threshold)[0]}
        got = {(int(d["i"]), int(d["j"])) for d in dots[dots["i"] == r * hx]}
        assert got == ref
    # every dot agrees with the dense plot it came with
    d = dots[:: max(1, dots.size // 2000)]
    plot = res["wlcs"]
    vals = plot[torch.as_tensor((d["i"] // hx).astype(np.int64), device="cuda"),
                torch.as_tensor(d["j"].astype(np.int64), device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(vals, d["wlcs"])
