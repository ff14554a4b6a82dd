"""Tuning of the seaweed kernels' tiling knobs.

Two knobs decide how the batched launch cuts its work:

* tile per window class: the y-windows each lane covers per tile (the
  "windows per wavefront" knob: a wave combs 64 strips x 2 tiles, so it covers
  128 x tile window pairs per unit).  Longer tiles spend less of their columns
  on the w - 1 warm-up columns of every tile; shorter tiles give more units,
  which balances the queue better.
* persistent grid: resident workgroups per compute unit ("tiles per
  workgroup" follows from it: every workgroup keeps taking units until the
  queue is empty).

The tuner itself is native: ``Context.tune`` calls ``wlcs_tune``, which times
real batched launches of a seeded synthetic batch for every candidate on the
device, applies the fastest and keeps them in a JSON cache keyed by device
name and compute-unit count (this module's command line rewrites the
package's cache).  ``tune_batch`` below does that search on a caller's own
batch through the same context setters; ``tune_plot`` measures the tiling of
one plot shape (the native ``wlcs_tune_plot``); ``load`` / ``apply`` read the
cache format from Python.

    python -m paper_0909_2000_amd.autotune --out paper_0909_2000_amd/tuning_gfx950.json [--plots]
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


def tune_plot(ctx, pair, w, hx=1, cache_path=None, force=False, log=print) -> tuple:
    """Measured tiling of one plot shape (the native ``wlcs_tune_plot``): the
    fastest of a grid of two-length tilings and its neighbourhood, recorded in
    the context (and in the cache file when given).  Returns (long tile, short
    tile, long pairs), (0, 0, 0) when the built-in choice was the fastest."""
    ctx.tune_plot(pair, w, hx=hx, cache_path=cache_path, force=force)
    rows, cols = -(-max(pair.m - w, 0) // hx), max(pair.n - w, 0)
    tiling = ctx.plot_tiling(rows, cols, w)
    log(f"  plot {rows}x{cols}x{w}: {tiling if any(tiling) else 'built-in'}")
    return tiling


def apply(ctx, cache: dict) -> None:
    """Set a tuning cache entry's batch knobs on a context (its measured plot
    tilings are applied by ``Context.tune(path)``, which reads the file)."""
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
    ap.add_argument("--plots", action="store_true",
                    help="also record measured tilings of the benchmark's plot shapes (50,000^2 DNA at w = 64, "
                         "every and every 5th x-window; 30,000^2 protein at w = 128)")
    args = ap.parse_args()
    import torch

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import paper_0909_2000_amd as wl

    ctx = wl.Context(0)
    ctx.tune(args.out, force=True)
    if args.plots:
        import workloads
        for k, hx in ((2, 1), (3, 1), (2, 5)):
            p = workloads.config(k)
            pair = ctx.pair(p.x, p.y, alphabet=p.alphabet)
            tune_plot(ctx, pair, p.w, hx=hx, cache_path=args.out, force=True,
                      log=lambda msg: print(msg, file=sys.stderr, flush=True))
            pair.close()
    entry = load(args.out, torch)
    print(f"tuned on {_device_key(torch)}: {json.dumps(entry)}", file=sys.stderr, flush=True)
    print(json.dumps(entry))


if __name__ == "__main__":
    main()
