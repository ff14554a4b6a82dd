"""GPU: the native tuner (wlcs_tune).  It times candidates on the device,
applies the fastest and keeps them in a JSON cache keyed by device; a second
context loads the entry without timing again; other devices' entries survive;
a malformed cache is refused without applying anything; and tiling never
changes a result (batched plots after tuning equal the plots made alone)."""
import json
import os
import time

import numpy as np

import pytest

import workloads

pytestmark = pytest.mark.gpu

TILES = {0, 256, 512, 1024, 2048, 4096}  # 0: the built-in choice
GRIDS = {0, 4, 6, 8, 16}
CLASSES = ("1-16", "17-32", "33-64", "65-128")


def _key(torch):
    p = torch.cuda.get_device_properties(0)
    return f"{getattr(p, 'gcnArchName', p.name).split(':')[0]}-{p.multi_processor_count}cu"


def test_tune_writes_applies_and_reloads(tmp_path):
    import torch
    import paper_0909_2000_amd as wl
    path = str(tmp_path / "cache.json")
    other = {"gfx000-1cu": {"batch_grid": 4, "batch_tiles": {"1-16": 64}}}
    with open(path, "w") as f:
        json.dump(other, f)
    ctx = wl.Context(0)
    print("tuning into", path, flush=True)
    ctx.tune(path)
    with open(path) as f:
        data = json.load(f)
    assert data["gfx000-1cu"] == other["gfx000-1cu"]  # other devices kept
    entry = data[_key(torch)]
    assert set(entry["batch_tiles"]) == set(CLASSES)
    assert set(entry["batch_tiles"].values()) <= TILES
    assert entry["batch_grid"] in GRIDS
    assert entry["batch_ms"]["tuned"] > 0 and entry["batch_ms"]["default"] > 0
    for key, tile in entry["batch_tiles"].items():
        lo, hi = map(int, key.split("-"))
        assert ctx.batch_tile(lo) == tile and ctx.batch_tile(hi) == tile
    assert entry["batch_ms"]["tuned"] <= entry["batch_ms"]["default"]
    assert ctx.batch_grid() == entry["batch_grid"]

    # a fresh context loads the entry: nothing is timed, the file is untouched
    before = open(path, "rb").read()
    mtime = os.stat(path).st_mtime_ns
    ctx2 = wl.Context(0)
    assert ctx2.batch_grid() == 0 and ctx2.batch_tile(64) == 0
    t0 = time.perf_counter()
    ctx2.tune(path)
    assert time.perf_counter() - t0 < 1.0
    assert open(path, "rb").read() == before and os.stat(path).st_mtime_ns == mtime
    assert ctx2.batch_grid() == entry["batch_grid"]
    assert ctx2.batch_tile(100) == entry["batch_tiles"]["65-128"]
    # a forced run replaces this device's entry and keeps the others
    ctx2.tune(path, force=True)
    with open(path) as f:
        again = json.load(f)
    assert again["gfx000-1cu"] == other["gfx000-1cu"] and _key(torch) in again


def test_tuned_batch_equals_plots_alone(tmp_path):
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    ctx.tune(None)  # tune, apply, write nothing
    assert ctx.batch_grid() in GRIDS
    g = workloads.rng(77)
    specs = []
    for k, w in enumerate((16, 32, 64, 128, 20, 100)):
        m, n = int(g.integers(300, 3000)) + w, int(g.integers(300, 3000)) + w
        x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
        specs.append({"pair": ctx.pair(x, y), "w": w, "threshold": (3 * w + 3) // 4, "indel": k % 2 == 0})
    print("batch after tuning:", [(s["pair"].m, s["pair"].n, s["w"]) for s in specs], flush=True)
    res = ctx.batch(specs)
    torch.cuda.synchronize()
    for s, r in zip(specs, res):
        alone = s["pair"].plot(s["w"], threshold=s["threshold"], indel=s["indel"])
        assert torch.equal(r["wlcs"], alone["wlcs"])
        assert torch.equal(r["bitmap"], alone["bitmap"])
        if s["indel"]:
            assert torch.equal(r["indel"], alone["indel"])


@pytest.mark.parametrize("text", ["not json", "[1, 2]", "{\"a\": 1"])
def test_unreadable_cache_is_refused(tmp_path, text):
    import paper_0909_2000_amd as wl
    path = tmp_path / "bad.json"
    path.write_text(text)
    ctx = wl.Context(0)
    with pytest.raises(wl.WlcsError) as e:
        ctx.tune(str(path))
    assert e.value.status == -1
    assert path.read_text() == text
    assert ctx.batch_grid() == 0


@pytest.mark.parametrize("entry", [
    {"batch_grid": 8, "batch_tiles": {"1-16": 100}},          # not a multiple of 64
    {"batch_grid": 8, "batch_tiles": {"1-16": -64}},          # negative
    {"batch_grid": 99, "batch_tiles": {"1-16": 512}},         # grid out of range
    {"batch_grid": 8, "batch_tiles": {"16": 512}},            # not a range
    {"batch_grid": 8},                                        # no tiles
])
def test_malformed_entry_applies_nothing(tmp_path, entry):
    import torch
    import paper_0909_2000_amd as wl
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({_key(torch): entry}))
    ctx = wl.Context(0)
    with pytest.raises(wl.WlcsError) as e:
        ctx.tune(str(path))
    assert e.value.status == -1
    assert ctx.batch_grid() == 0 and ctx.batch_tile(8) == 0


def test_cache_entry_is_applied_as_written(tmp_path):
    import torch
    import paper_0909_2000_amd as wl
    path = tmp_path / "cache.json"
    entry = {"batch_grid": 6, "batch_tiles": {"1-16": 256, "17-32": 768, "33-64": 0, "65-128": 2048},
             "batch_ms": {"default": 1.0, "tuned": 1.0}}
    path.write_text(json.dumps({_key(torch): entry}, indent=1))
    ctx = wl.Context(0)
    ctx.tune(str(path))
    assert ctx.batch_grid() == 6
    assert [ctx.batch_tile(w) for w in (16, 17, 64, 65, 128)] == [256, 768, 0, 2048, 2048]


def _plot_pair(wl, ctx, seed=70, m=4000, n=5000):
    g = workloads.rng(seed)
    x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
    return x, y, ctx.pair(x, y)


def test_tune_plot_records_applies_and_keeps_other_entries(tmp_path, oracle_mod):
    """wlcs_tune_plot times tilings of one shape, records the fastest in the
    context and the cache (the device's batch knobs and other devices'
    entries stay), a second context loads the record without timing, and
    wlcs_tune keeps the plot records when it completes the device entry.
    The plots are the same whichever tiling applies."""
    import torch
    import paper_0909_2000_amd as wl
    path = tmp_path / "cache.json"
    other = {"gfx000-1cu": {"batch_grid": 4, "batch_tiles": {"1-16": 64}}}
    path.write_text(json.dumps(other))
    ctx = wl.Context(0)
    x, y, pair = _plot_pair(wl, ctx)
    w = 64
    rows, cols = x.size - w, y.size - w
    ref = pair.plot(w)["wlcs"].clone()  # the built-in tiling
    t0 = time.time()
    ctx.tune_plot(pair, w, cache_path=str(path))
    print(f"tune_plot {rows}x{cols}x{w}: {time.time() - t0:.1f} s", flush=True)
    data = json.loads(path.read_text())
    assert data["gfx000-1cu"] == other["gfx000-1cu"]
    entry = data[_key(torch)]
    rec = entry["plots"][f"{rows}x{cols}x{w}"]
    ms = entry["plots_ms"][f"{rows}x{cols}x{w}"]
    assert ms["tuned"] <= ms["builtin"] and ms["tuned"] > 0
    assert len(rec) == 3
    assert ctx.plot_tiling(rows, cols, w) == (tuple(rec) if rec[0] else (0, 0, 0))
    assert torch.equal(pair.plot(w)["wlcs"], ref)
    sample = [0, rows // 2, rows - 1]
    np_ref = ref[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(np_ref, oracle_mod.wlcs_rows(x, y, w, sample))
    # a second context applies the record and times nothing
    ctx2 = wl.Context(0)
    pair2 = ctx2.pair(x, y)
    t0 = time.time()
    ctx2.tune_plot(pair2, w, cache_path=str(path))
    assert time.time() - t0 < 1.0
    assert ctx2.plot_tiling(rows, cols, w) == ctx.plot_tiling(rows, cols, w)
    # wlcs_tune completes the entry with the batch knobs and keeps the record
    ctx3 = wl.Context(0)
    ctx3.tune(str(path))
    entry3 = json.loads(path.read_text())[_key(torch)]
    assert "batch_tiles" in entry3 and entry3["plots"] == entry["plots"]
    assert ctx3.plot_tiling(rows, cols, w) == ctx.plot_tiling(rows, cols, w)


def test_recorded_plot_tiling_is_applied(tmp_path, oracle_mod):
    """A cache record with a deliberate tiling (long tiles of 1024 windows for
    one leading pair, then 256) is applied to plots of that shape only; the
    strided shape (every 3rd x-window) has a record of its own."""
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    x, y, pair = _plot_pair(wl, ctx, seed=71, m=3000, n=4100)
    w = 100
    rows, cols = x.size - w, y.size - w
    srows = -(-rows // 3)
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({_key(torch): {"plots": {f"{rows}x{cols}x{w}": [1024, 256, 1],
                                                         f"{srows}x{cols}x{w}": [512, 128, 2]}}}))
    ctx.tune_plot(pair, w, cache_path=str(path))
    assert ctx.plot_tiling(rows, cols, w) == (1024, 256, 1)
    assert ctx.plot_tiling(srows, cols, w) == (0, 0, 0)  # only the asked shape is applied
    ctx.tune_plot(pair, w, hx=3, cache_path=str(path))
    assert ctx.plot_tiling(srows, cols, w) == (512, 128, 2)
    got = pair.plot(w)["wlcs"].cpu().numpy()
    np.testing.assert_array_equal(got, oracle_mod.wlcs(x, y, w))
    got = pair.plot_strided(w, 3, 1)["wlcs"].cpu().numpy()
    np.testing.assert_array_equal(got, oracle_mod.wlcs_strided(x, y, w, 3, 1))
    other = wl.Context(0)  # a context without the record: the same plots
    assert other.plot_tiling(rows, cols, w) == (0, 0, 0)
    np.testing.assert_array_equal(other.pair(x, y).plot(w)["wlcs"].cpu().numpy(), oracle_mod.wlcs(x, y, w))


@pytest.mark.parametrize("plots", [
    {"10x10x8": [100, 64, 1]},      # not a multiple of 64
    {"10x10x8": [512, 1024, 1]},    # short tile longer than the long one
    {"10x10": [512, 256, 1]},       # not rows x cols x w
    {"10x10x8": [512, 256]},        # two numbers
    [1, 2, 3],                      # not an object
])
def test_malformed_plot_records_apply_nothing(tmp_path, plots):
    import torch
    import paper_0909_2000_amd as wl
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({_key(torch): {"batch_grid": 6, "batch_tiles": {"1-16": 256}, "plots": plots}}))
    ctx = wl.Context(0)
    with pytest.raises(wl.WlcsError) as e:
        ctx.tune(str(path))
    assert e.value.status == -1
    assert ctx.batch_grid() == 0 and ctx.plot_tiling(10, 10, 8) == (0, 0, 0)


def test_tune_plot_narrow_and_empty_shapes(tmp_path, oracle_mod):
    """A plot narrower than every candidate tile records the built-in choice
    ([0, 0, 0]); an empty plot returns at once and records nothing."""
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    x, y, pair = _plot_pair(wl, ctx, seed=72, m=400, n=130)
    w = 16
    path = tmp_path / "cache.json"
    ctx.tune_plot(pair, w, cache_path=str(path))
    rows, cols = x.size - w, y.size - w
    entry = json.loads(path.read_text())[_key(torch)]
    assert entry["plots"][f"{rows}x{cols}x{w}"] == [0, 0, 0]
    assert ctx.plot_tiling(rows, cols, w) == (0, 0, 0)
    np.testing.assert_array_equal(pair.plot(w)["wlcs"].cpu().numpy(), oracle_mod.wlcs(x, y, w))
    tiny = ctx.pair(b"ACGTACGT", b"ACGTACGTAC")
    ctx.tune_plot(tiny, 8, cache_path=str(path))  # m - w = 0 windows: nothing to tune
    assert "0x2x8" not in json.loads(path.read_text())[_key(torch)]["plots"]
