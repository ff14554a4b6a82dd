"""Tuner for the tiling knobs of the seaweed kernels.

Two knobs decide how the batched launch cuts its work:

* tile per window class: the y-windows each lane covers per tile (the
  "windows per wavefront" knob: a wave combs 64 strips x 2 tiles, so it covers
  128 x tile window pairs per unit).  Longer tiles spend less of their columns
  on the w - 1 warm-up columns of every tile; shorter tiles give more units,
  which balances the queue better.
* persistent grid: resident workgroups per compute unit ("tiles per
  workgroup" follows from it: every workgroup keeps taking units until the
  queue is empty).

The tuner times real batched launches on the device for each candidate and
keeps the fastest; the single-plot tile is tuned the same way for a given
plot shape.  Results go to a JSON cache keyed by device name and compute-unit
count, and ``apply`` sets them on a context.

    python -m paper_0909_2000_amd.autotune --out paper_0909_2000_amd/tuning_gfx950.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

TILES = (256, 512, 1024, 2048, 4096, 8192)
GRIDS = (4, 6, 8, 12, 16)
CLASSES = ((1, 16), (17, 32), (33, 64), (65, 128))


def _device_key(torch) -> str:
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", p.name).split(":")[0]
    return f"{arch}-{p.multi_processor_count}cu"


def _time(torch, fn, reps=3) -> float:
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    return ms[len(ms) // 2]


def tune_batch(ctx, specs, log=print) -> dict:
    """Pick a tile per window class on the jobs of that class, then the grid
    on the whole batch.  specs: as for Context.batch (outputs preallocated)."""
    import torch
    best_tiles = {}
    for lo, hi in CLASSES:
        sub = [s for s in specs if lo <= s["w"] <= hi]
        if not sub:
            continue
        times = {}
        for t in TILES:
            ctx.set_batch_tile(lo, hi, t)
            times[t] = _time(torch, lambda: ctx.batch(sub))
        ctx.set_batch_tile(lo, hi, 0)
        tile = min(times, key=times.get)
        best_tiles[f"{lo}-{hi}"] = tile
        log(f"  w {lo}-{hi}: " + ", ".join(f"{t}:{v:.2f}ms" for t, v in times.items()) + f" -> {tile}")
    for key, tile in best_tiles.items():
        lo, hi = map(int, key.split("-"))
        ctx.set_batch_tile(lo, hi, tile)
    gtimes = {}
    for g in GRIDS:
        ctx.set_batch_grid(g)
        gtimes[g] = _time(torch, lambda: ctx.batch(specs))
    ctx.set_batch_grid(0)
    grid = min(gtimes, key=gtimes.get)
    log("  grid: " + ", ".join(f"{g}:{v:.2f}ms" for g, v in gtimes.items()) + f" -> {grid}")
    return {"batch_tiles": best_tiles, "batch_grid": grid,
            "batch_ms": {"default": None, "tuned": gtimes[grid]}}


def tune_plot(ctx, pair, w, threshold=None, log=print) -> dict:
    """Tile for single plots of this shape (applies to the w's class)."""
    import torch
    rows, cols = max(pair.m - w, 0), max(pair.n - w, 0)
    out = torch.empty((rows, cols), dtype=torch.uint8, device="cuda")
    times = {}
    for t in (0,) + TILES:  # 0 = built-in choice
        ctx.set_tile(1, 255, t) if t else ctx.set_tile(1, 255, 0)
        times[t] = _time(torch, lambda: pair.plot(w, threshold=threshold, out=out))
    ctx.set_tile(1, 255, 0)
    tile = min(times, key=times.get)
    log("  plot: " + ", ".join(f"{t or 'auto'}:{v:.2f}ms" for t, v in times.items()) + f" -> {tile or 'auto'}")
    return {"tile": tile, "ms": times}


def apply(ctx, cache: dict) -> None:
    """Set a tuning cache's knobs on a context."""
    for key, tile in cache.get("batch_tiles", {}).items():
        lo, hi = map(int, key.split("-"))
        ctx.set_batch_tile(lo, hi, int(tile))
    if cache.get("batch_grid"):
        ctx.set_batch_grid(int(cache["batch_grid"]))


def load(path: str, torch=None) -> dict | None:
    """The cache entry for this device, if the file has one."""
    if not os.path.exists(path):
        return None
    if torch is None:
        import torch
    with open(path) as f:
        data = json.load(f)
    return data.get(_device_key(torch))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "tuning_gfx950.json"))
    ap.add_argument("--pairs", type=int, default=128, help="pairs of the batch workload used")
    args = ap.parse_args()
    import torch

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import paper_0909_2000_amd as wl
    import workloads

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ctx = wl.Context(0)
    pairs = workloads.batch_config(seed=40, npairs=args.pairs)  # a tuning set, not the benchmark's
    specs = [{"pair": ctx.pair(p.x, p.y), "w": p.w} for p in pairs]
    res = ctx.batch(specs)
    for s, r in zip(specs, res):
        s["out"] = r["wlcs"]
    log(f"tuning on {len(specs)} pairs ({_device_key(torch)})")
    default_ms = _time(torch, lambda: ctx.batch(specs))
    entry = tune_batch(ctx, specs, log=log)
    entry["batch_ms"]["default"] = default_ms
    data = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            data = json.load(f)
    data[_device_key(torch)] = entry
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    log(f"default {default_ms:.2f} ms -> tuned {entry['batch_ms']['tuned']:.2f} ms; wrote {args.out}")
    print(json.dumps(entry))


if __name__ == "__main__":
    main()
