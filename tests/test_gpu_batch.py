"""GPU: the batched persistent launch (wlcs_batch) and its captured graph.

Each plot of a batch must equal the oracle (whole matrices at small sizes,
sampled rows at the batch configuration's full size) and the same plot run
alone (bit-exact), whatever the queue order, tile choice or grid size.  Graph
replays are checked one by one, with eager work in between.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wl():
    import torch
    assert torch.cuda.is_available()
    import paper_0909_2000_amd as wl
    wl._load()
    return wl


@pytest.fixture(scope="module")
def ctx(wl):
    return wl.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.cpu().numpy()


def _mixed_specs(ctx, seed, count, lo, hi, ws, extras=True):
    g = workloads.rng(seed)
    specs, inputs = [], []
    for k in range(count):
        w = int(ws[k % len(ws)])
        m, n = int(g.integers(lo, hi)) + w, int(g.integers(lo, hi)) + w
        alpha = workloads.PROTEIN if k % 3 == 0 else workloads.DNA
        x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
        spec = {"pair": ctx.pair(x, y, alphabet=alpha), "w": w}
        if extras and k % 2 == 0:
            spec["threshold"] = (3 * w + 3) // 4
        if extras and k % 4 == 1:
            spec["indel"] = True
        if extras and k % 5 == 2:
            spec["full_range"] = True
        specs.append(spec)
        inputs.append((x, y, w))
    return specs, inputs


def _check_vs_oracle(oracle_mod, res, spec, x, y, w):
    full = spec.get("full_range", False)
    want = oracle_mod.wlcs(x, y, w, full_range=full)
    np.testing.assert_array_equal(_np(res["wlcs"]), want)
    if "threshold" in spec:
        np.testing.assert_array_equal(_np(res["bitmap"]).view(np.uint64),
                                      oracle_mod.dot_bitmap(want, spec["threshold"]))
    if spec.get("indel"):
        np.testing.assert_array_equal(_np(res["indel"]).view(np.uint16), oracle_mod.indel(want, w))


def test_small_mixed_batch_vs_oracle(ctx, oracle_mod):
    ws = (1, 5, 16, 17, 32, 48, 64, 100, 128, 129, 200, 255)
    specs, inputs = _mixed_specs(ctx, 11, 36, 1, 400, ws)
    _say(f"batch of {len(specs)} small plots")
    results = ctx.batch(specs)
    for res, spec, (x, y, w) in zip(results, specs, inputs):
        _check_vs_oracle(oracle_mod, res, spec, x, y, w)


def test_batch_equals_single_plots(ctx):
    import torch
    specs, inputs = _mixed_specs(ctx, 12, 24, 500, 3000, (16, 32, 64, 128, 40))
    _say("batch vs singles, 24 plots")
    results = ctx.batch(specs)
    for res, spec in zip(results, specs):
        alone = spec["pair"].plot(spec["w"], threshold=spec.get("threshold"), indel=spec.get("indel", False),
                                  full_range=spec.get("full_range", False))
        for key in alone:
            assert torch.equal(res[key], alone[key]), key


@pytest.mark.parametrize("grid,tile", [(1, 0), (16, 0), (8, 64), (3, 1024)])
def test_grid_and_tile_do_not_change_results(ctx, grid, tile):
    import torch
    specs, _ = _mixed_specs(ctx, 13, 12, 200, 1500, (16, 64, 128, 33), extras=False)
    ref = ctx.batch(specs)
    ctx.set_batch_grid(grid)
    if tile:
        ctx.set_batch_tile(1, 128, tile)
    try:
        got = ctx.batch(specs)
    finally:
        ctx.set_batch_grid(0)
        ctx.set_batch_tile(1, 128, 0)
    for a, b in zip(ref, got):
        assert torch.equal(a["wlcs"], b["wlcs"])


@pytest.mark.parametrize("min_units", [1, 1024, 1 << 20])
def test_min_units_shortens_tiles_without_changing_results(ctx, oracle_mod, min_units):
    """wlcs_ctx_set_batch_min_units: jobs with fewer units than asked for run
    on shorter tiles (down to 64 windows for 1 << 20); every plot still equals
    the batch without the setting, and the oracle on a few of them."""
    import torch
    specs, inputs = _mixed_specs(ctx, 14, 16, 100, 2500, (16, 32, 64, 128, 50), extras=True)
    ctx.set_batch_tile(1, 128, 4096)  # long tiles: few units per job
    try:
        ref = ctx.batch(specs)
        ctx.set_batch_min_units(min_units)
        try:
            got = ctx.batch(specs)
        finally:
            ctx.set_batch_min_units(0)
    finally:
        ctx.set_batch_tile(1, 128, 0)
    _say(f"min units {min_units}: {len(specs)} plots")
    for a, b in zip(ref, got):
        for key in a:
            assert torch.equal(a[key], b[key]), key
    for k in (0, 5, 11):
        _check_vs_oracle(oracle_mod, got[k], specs[k], *inputs[k])


def test_batch_row_strides_and_empty_jobs(ctx, oracle_mod):
    import torch
    g = workloads.rng(14)
    x, y = workloads.iid(g, 300, workloads.DNA), workloads.iid(g, 500, workloads.DNA)
    p = ctx.pair(x, y)
    tiny = ctx.pair(b"ACG", b"ACGT")  # empty plot for w >= 3
    want = oracle_mod.wlcs(x, y, 20)
    rows, cols = want.shape
    buf = torch.full((rows, cols + 5), 0x5A, dtype=torch.uint8, device="cuda")
    specs = [{"pair": p, "w": 20, "out": buf[:, :cols]}, {"pair": tiny, "w": 3},
             {"pair": p, "w": 20, "threshold": 15, "want_plot": False}]
    res = ctx.batch(specs)
    np.testing.assert_array_equal(_np(buf[:, :cols]), want)
    assert np.all(_np(buf[:, cols:]) == 0x5A)
    assert res[1]["wlcs"].numel() == 0
    np.testing.assert_array_equal(_np(res[2]["bitmap"]).view(np.uint64), oracle_mod.dot_bitmap(want, 15))


def test_graph_replays(ctx, oracle_mod):
    import torch
    specs, inputs = _mixed_specs(ctx, 15, 10, 50, 600, (16, 32, 64, 128, 130), extras=True)
    graph = ctx.batch_graph(specs)
    eager = ctx.batch(specs)
    torch.cuda.synchronize()
    for replay in range(4):
        for r in graph.results:  # wipe the outputs, then replay into them
            for t in r.values():
                t.fill_(0x33)
        other = ctx.plot(inputs[0][0], inputs[0][1], 7, alphabet=workloads.PROTEIN)["wlcs"]  # unrelated eager work
        graph.launch()
        torch.cuda.synchronize()
        for a, b in zip(graph.results, eager):
            for key in a:
                assert torch.equal(a[key], b[key]), (replay, key)
        assert other.numel() > 0
    for res, spec, (x, y, w) in zip(graph.results, specs, inputs):
        _check_vs_oracle(oracle_mod, res, spec, x, y, w)
    graph.close()


def _batch_digests():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_plots.txt")
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, w, rows, cols, d = line.split()
            out[int(k)] = (int(w), int(rows), int(cols), d)
    return out


def test_batch_configuration_full_size(ctx, oracle_mod):
    """256 DNA pairs, m, n uniform in [1000, 20000], w from {16, 32, 64, 128},
    in one persistent launch: every plot whole against the oracle (the digests
    of tests/golden/batch_plots.txt, written by
    tests/golden/make_batch_digests.py from the oracle alone) and against its
    single-plot run on the device, plus a sampled row and entries against the
    oracle directly."""
    import hashlib
    import torch
    pairs = workloads.batch_config()
    gold = _batch_digests()
    assert len(gold) == len(pairs) == 256
    _say(f"batch configuration: {len(pairs)} pairs")
    specs = [{"pair": ctx.pair(p.x, p.y), "w": p.w} for p in pairs]
    res = ctx.batch(specs)
    torch.cuda.synchronize()
    g = workloads.rng(16)
    bad = []
    for k, (p, r) in enumerate(zip(pairs, res)):
        W = r["wlcs"]
        rows, cols = W.shape
        assert (rows, cols) == (p.m - p.w, p.n - p.w)
        assert gold[k][:3] == (p.w, rows, cols), k
        if hashlib.blake2b(_np(W).tobytes(), digest_size=8).hexdigest() != gold[k][3]:
            bad.append(("oracle", k))
        if not torch.equal(W, specs[k]["pair"].plot(p.w)["wlcs"]):
            bad.append(("single plot", k))
        row = int(g.integers(0, rows))
        np.testing.assert_array_equal(_np(W[row:row + 1]), oracle_mod.wlcs_rows(p.x, p.y, p.w, [row]))
        ii, jj = g.integers(0, rows, 16), g.integers(0, cols, 16)
        got = _np(W[torch.as_tensor(ii, device="cuda"), torch.as_tensor(jj, device="cuda")])
        np.testing.assert_array_equal(got, oracle_mod.wlcs_at(p.x, p.y, p.w, ii, jj))
        r["wlcs"] = None  # release the pair's plot as the check goes
        del W
    assert not bad, bad[:20]


def _sorted_dots(res):
    import paper_0909_2000_amd as wl
    return wl.dot_records(res)


def test_strided_and_sparse_jobs_equal_alone(oracle_mod):
    """Batched jobs with step sizes and dot lists (windows up to 128 in the
    persistent launch, 200 as a separate launch) give exactly what each job
    gives alone through wlcs_pair_plot_strided; a graph replay zeroes the dot
    counters again each time."""
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(44)
    ctx = wl.Context(0)
    specs, alone_args = [], []
    for k, (w, hx, hy, sparse) in enumerate([(16, 1, 1, True), (32, 2, 3, True), (64, 5, 1, False),
                                              (64, 3, 2, True), (100, 1, 4, True), (128, 4, 1, True),
                                              (200, 5, 2, True), (48, 1, 1, False)]):
        m, n = int(g.integers(400, 2500)) + w, int(g.integers(400, 2500)) + w
        x = workloads.iid(g, m, workloads.DNA)
        y = workloads.iid(g, n, workloads.DNA)
        y[100:100 + 2 * w] = x[50:50 + 2 * w]  # a homology, so the lists are not empty
        pair = ctx.pair(x, y)
        thr = (3 * w + 3) // 4
        sp = {"pair": pair, "w": w, "hx": hx, "hy": hy, "threshold": thr, "indel": k % 2 == 0,
              "x": x, "y": y}
        if sparse:
            sp["dot_cap"] = 100000
        specs.append(sp)
    print("jobs:", [(s["pair"].m, s["pair"].n, s["w"], s["hx"], s["hy"], "dot_cap" in s) for s in specs], flush=True)
    batch_specs = [{k: v for k, v in s.items() if k not in ("x", "y")} for s in specs]
    res = ctx.batch(batch_specs)
    torch.cuda.synchronize()
    for s, r in zip(specs, res):
        alone = s["pair"].plot_strided(s["w"], s["hx"], s["hy"], threshold=s["threshold"], indel=s["indel"],
                                       dot_cap=s.get("dot_cap"))
        torch.cuda.synchronize()
        assert torch.equal(r["wlcs"], alone["wlcs"])
        for key in ("bitmap", "indel"):
            assert (key in r) == (key in alone)
            if key in r:
                assert torch.equal(r[key], alone[key])
        if "dot_cap" in s:
            got, n_got = _sorted_dots(r)
            want, n_want = _sorted_dots(alone)
            assert n_got == n_want > 0
            np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))
    # the oracle on two of them
    for s, r in list(zip(specs, res))[1:3]:
        want = oracle_mod.wlcs_strided(s["x"], s["y"], s["w"], s["hx"], s["hy"])
        np.testing.assert_array_equal(r["wlcs"].cpu().numpy(), want)
    # a captured graph: every replay zeroes and refills the counters
    graph = ctx.batch_graph(batch_specs)
    counts = [r["dot_count"] for r in graph.results if "dot_count" in r]
    first = None
    for rep in range(3):
        graph.launch()
        torch.cuda.synchronize()
        now = [int(c.item()) for c in counts]
        first = first or now
        assert now == first, rep
        for c in counts:  # eager work between replays
            c.fill_(999)
        torch.cuda.synchronize()
    graph.close()


@pytest.mark.parametrize("ws", [(16, 9), (32, 20), (64, 40), (128, 100), (16, 128), (64, 200), (255,)])
def test_batch_group_subsets_vs_oracle(ctx, oracle_mod, ws):
    """Jobs in only some of the three kernel groups (windows up to 32, up to
    64, up to 128; 200 and 255 run alone): the groups without jobs launch
    nothing and the others still see only their own jobs."""
    specs, inputs = _mixed_specs(ctx, 60 + sum(ws), 2 * len(ws) + 1, 20, 300, ws)
    _say(f"batch of windows {ws}")
    results = ctx.batch(specs)
    for res, spec, (x, y, w) in zip(results, specs, inputs):
        _check_vs_oracle(oracle_mod, res, spec, x, y, w)


def test_sparse_job_in_one_group_only(oracle_mod):
    """A dot-listing strided job among plain jobs of the other groups: only its
    group runs the strided/sparse kernel variant; every job equals the oracle."""
    import torch
    import paper_0909_2000_amd as wl
    g = workloads.rng(61)
    ctx = wl.Context(0)
    for sparse_w in (16, 64, 100):
        specs, inputs = [], []
        for w in (16, 30, 64, 50, 128, 90):
            m, n = int(g.integers(300, 900)) + w, int(g.integers(300, 900)) + w
            x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
            specs.append({"pair": ctx.pair(x, y), "w": w})
            inputs.append((x, y, w))
        m, n = 1200 + sparse_w, 1100 + sparse_w
        x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
        y[200:200 + 2 * sparse_w] = x[100:100 + 2 * sparse_w]  # a homology, so the list is not empty
        thr = (3 * sparse_w + 3) // 4
        specs.append({"pair": ctx.pair(x, y), "w": sparse_w, "hx": 3, "hy": 2, "threshold": thr,
                      "dot_cap": 50000})
        _say(f"sparse job w={sparse_w} among plain jobs")
        res = ctx.batch(specs)
        torch.cuda.synchronize()
        for r, (xx, yy, w) in zip(res[:-1], inputs):
            np.testing.assert_array_equal(_np(r["wlcs"]), oracle_mod.wlcs(xx, yy, w))
        want = oracle_mod.wlcs_strided(x, y, sparse_w, 3, 2)
        np.testing.assert_array_equal(_np(res[-1]["wlcs"]), want)
        dots, count = wl.dot_records(res[-1])
        ref = oracle_mod.dot_list(want, sparse_w, thr, 3, 2)
        assert count == ref.size > 0
        np.testing.assert_array_equal(dots.view(np.uint8), ref.view(np.uint8))
