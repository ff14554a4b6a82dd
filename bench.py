"""Benchmark: alignment plot throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dna-50k-w64]

A step is one pass of the whole hot path over the workload: the windowed
seaweed plot (every strip combed, counted, stored, with the thresholded dot-plot
bitmap) of a device-resident, encoded pair.  The default workload is the DNA
pair of 50,000 x 50,000 letters with w = 64 and 20 planted homologies, bitmap at
WLCS >= 48.  Prints one JSON line on stdout; progress goes to stderr.

Beside the headline number it measures, in the same run: the plain per-window
dynamic program on the same GPU (the paper's O(m n w^2) baseline), the CPU
oracle on a bounded sample of rows on the host cores, and the kernel's
roofline position.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
TUNING_CACHE = os.path.join(ROOT, "paper_0909_2000_amd", "tuning_gfx950.json")
FIXED_RATE = 1100.0  # serving: jobs/s of the fixed-rate latency point
sys.path.insert(0, ROOT)

# HIP events over the timed region; per-cell operation count of the seaweed
# cell: the equality test, min, max and the exchange of the two labels (one
# three-input XOR)
OPS_PER_CELL = 4
# MI355X: 256 CUs x 64 lanes x 2 packed 16-bit elements x 2.4 GHz
PEAK_U16_OPS = 256 * 64 * 2 * 2.4e9
METRIC = "window-cells/s (m*n*w/s) vs plain DP on same GPU; p50/p99 job latency"

WORKLOADS = {"dna-50k-w64": 2, "dna-1k-w16": 1, "protein-30k-w128": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (Linux), or an empty string."""
    return cpu_info().get("model_name", "")


def cpu_info() -> dict:
    """The host CPU as /proc/cpuinfo and the scheduler describe it: model name,
    vendor, family/model/stepping, logical CPUs, the CPUs this process may run
    on, and OMP_NUM_THREADS."""
    info = {}
    keys = {"model name": "model_name", "vendor_id": "vendor", "cpu family": "family", "model": "model",
            "stepping": "stepping"}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # the first CPU's block is enough
                k, _, v = line.partition(":")
                k = k.strip()
                if k in keys:
                    info[keys[k]] = v.strip()
    except OSError:
        pass
    info["nproc"] = os.cpu_count()
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["affinity"] = None
    info["omp_num_threads"] = os.environ.get("OMP_NUM_THREADS")
    return info


def measured_traffic(workload: str, cells: float = 0.0):
    """HBM bytes per launch of the timed kernel, from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs, each scaled by what the same counter read for
    a plain 1 GiB device copy; None when the kernel sources changed since.
    The detail also carries the VALU counters of the same kernel: wave
    instructions x 64 lanes per cell (4 instructions per two cells is 2.0),
    and, from the counter run's own launch time and GRBM_COUNT, the shader
    clock and the SIMD cycles per wave64 VALU instruction."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"seaweed_counters_{workload.replace('-planted', '')}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)
    h = hashlib.sha1()
    for fn in d["digest_files"]:
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != d["kernel_digest"]:
        return None, {"stale": True, "source": os.path.relpath(path, ROOT)}
    fetch = sum(d["fetch_kib_per_dispatch"]) / len(d["fetch_kib_per_dispatch"]) * 1024
    write = sum(d["write_kib_per_dispatch"]) / len(d["write_kib_per_dispatch"]) * 1024
    f_scale = d["copy_fetch_kib"] * 1024 / d["copy_bytes"]
    w_scale = d["copy_write_kib"] * 1024 / d["copy_bytes"]
    detail = {"read_bytes": fetch / f_scale, "write_bytes": write / w_scale,
              "fetch_scale": f_scale, "write_scale": w_scale,
              "source": os.path.relpath(path, ROOT)}
    vc = d.get("valu_counters_per_dispatch")
    if vc and cells:
        mean = lambda k: sum(vc[k]) / len(vc[k])
        insts = mean("SQ_INSTS_VALU")
        detail["valu"] = {"lane_instructions_per_cell": insts * 64 / cells,
                          "instructions_per_launch": insts,
                          "salu_per_valu": mean("SQ_INSTS_SALU") / insts}
        ns = d.get("valu_run_kernel_ns")
        if ns and "GRBM_COUNT" in vc:
            # the counter run's last launch (the first runs while the clock
            # ramps up); GRBM_COUNT is summed over the 8 XCDs, each XCD's
            # count runs at the shader clock
            cyc = vc["GRBM_COUNT"][-1] / 8
            detail["valu"].update({
                "counter_run_launch_ms": ns[-1] / 1e6,
                "clock_ghz": cyc / ns[-1],
                # SIMD cycles per wave64 VALU instruction, every other cycle
                # included (1,024 SIMDs)
                "simd_cycles_per_valu_instruction": cyc / (vc["SQ_INSTS_VALU"][-1] / 1024),
                "cu_busy_share": vc["SQ_BUSY_CU_CYCLES"][-1] / 256 / cyc,
                # the counter's accounting: one quad-cycle per wave64 instruction
                "valu_quad_cycles_per_instruction": vc["SQ_ACTIVE_INST_VALU"][-1] / vc["SQ_INSTS_VALU"][-1]})
    return detail["read_bytes"] + detail["write_bytes"], detail


# kernel sources whose digest the counter summary records (a summary of
# other sources is stale and its bytes are not reported)
COUNTER_DIGEST_FILES = ["paper_0909_2000_amd/csrc/seaweed.hip", "paper_0909_2000_amd/csrc/seaweed_unit.hpp",
                        "paper_0909_2000_amd/csrc/packed.hpp", "paper_0909_2000_amd/csrc/kernels.hpp"]


def write_counters(prof_dir: str, workload: str, commands: list) -> str:
    """Summarise rocprofv3 runs of this benchmark into
    profiles/seaweed_counters_<workload>.json: the timed kernel's FETCH_SIZE
    and WRITE_SIZE per dispatch (runs bytes_FETCH_SIZE and bytes_WRITE_SIZE,
    made with --calib-copy) beside the same counters of the plain 1 GiB copy,
    and its VALU and clock counters with the launch times of that run
    (valu_<workload>).  No GPU is used."""
    import csv
    import hashlib

    def dispatches(sub, pick):
        rows = list(csv.DictReader(open(os.path.join(prof_dir, sub, "run_counter_collection.csv"))))
        per = {}
        for r in rows:
            e = per.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})
            e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        return pick([per[k] for k in sorted(per)])

    def timed_kernel(ds):  # the plot kernel of the run: its dispatches, in order
        plot = [d for d in ds if "seaweed_kernel" in d["name"]]
        name = max(plot, key=lambda d: d.get("SQ_INSTS_VALU", d.get("FETCH_SIZE", d.get("WRITE_SIZE", 0))))["name"]
        return [d for d in plot if d["name"] == name]

    def copy_kernel(ds):  # the largest device copy of the run (the 1 GiB calibration copy)
        return [max((d for d in ds if "copyBuffer" in d["name"]),
                    key=lambda d: d.get("FETCH_SIZE", d.get("WRITE_SIZE", 0.0)))]

    fetch = dispatches("bytes_FETCH_SIZE", timed_kernel)
    write = dispatches("bytes_WRITE_SIZE", timed_kernel)
    cf = dispatches("bytes_FETCH_SIZE", copy_kernel)[0]
    cw = dispatches("bytes_WRITE_SIZE", copy_kernel)[0]
    valu = dispatches(f"valu_{workload}", timed_kernel)
    trace = list(csv.DictReader(open(os.path.join(prof_dir, f"valu_{workload}", "run_kernel_trace.csv"))))
    ns = [int(t["End_Timestamp"]) - int(t["Start_Timestamp"]) for t in trace
          if t["Kernel_Name"] == valu[0]["name"]]
    h = hashlib.sha1()
    for fn in COUNTER_DIGEST_FILES:
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(f.read())
    name = valu[0]["name"]
    short = name[name.index("seaweed_kernel"):name.index(">") + 1] if ">" in name else name
    counters = sorted(k for k in valu[0] if k != "name")
    out = {"kernel": short, "workload": workload, "kernel_digest": h.hexdigest(),
           "digest_files": COUNTER_DIGEST_FILES,
           "fetch_kib_per_dispatch": [d["FETCH_SIZE"] for d in fetch],
           "write_kib_per_dispatch": [d["WRITE_SIZE"] for d in write],
           "copy_bytes": 1 << 30, "copy_fetch_kib": cf["FETCH_SIZE"], "copy_write_kib": cw["WRITE_SIZE"],
           "valu_counters_per_dispatch": {k: [d[k] for d in valu] for k in counters},
           "valu_run_kernel_ns": ns, "commands": commands}
    path = os.path.join(ROOT, "profiles", f"seaweed_counters_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dna-50k-w64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-dp", action="store_true", help="skip the GPU DP baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU sample time")
    ap.add_argument("--tile", type=int, default=0, help="override the seaweed tile (windows)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-pair measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serving-jobs", type=int, default=2000)
    ap.add_argument("--serving-load", type=float, default=0.7, help="arrival rate / measured capacity")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serving HBM budget")
    ap.add_argument("--serving-repeats", type=int, default=3,
                    help="runs of the headline serving point (the spread of p50/p99 is reported)")
    ap.add_argument("--serving-child", action="store_true",
                    help="internal: run only the serving leg, after a line on stdin, and print its JSON")
    ap.add_argument("--row-align", type=int, default=64,
                    help="row stride of the timed plot rounded up to this many bytes")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other single-pair configurations (1k DNA w16, 30k protein w128)")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the alignment-score plots shaped like the paper's experiments")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--write-counters", metavar="DIR",
                    help="write profiles/seaweed_counters_<workload>.json from the rocprofv3 runs under DIR "
                         "(bytes_FETCH_SIZE, bytes_WRITE_SIZE, valu_<workload>) and exit; no GPU")
    ap.add_argument("--counter-commands", metavar="FILE",
                    help="with --write-counters: a text file of the rocprofv3 commands, one a line")
    args = ap.parse_args()

    if args.write_counters:
        cmds = []
        if args.counter_commands:
            with open(args.counter_commands) as f:
                cmds = [ln.strip() for ln in f if ln.strip()]
        print(write_counters(args.write_counters, args.workload, cmds))
        return
    if args.serving_child:
        serving_child(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    # The serving leg runs in a child process of its own, started here before
    # this process touches the GPU: it waits until the headline plot is done,
    # then serves with a device context that nothing else in its process has
    # used (measured after the other legs in this process, its latencies read
    # 30-40% higher).
    child = None
    if not args.no_serving:
        cmd = [sys.executable, os.path.abspath(__file__), "--serving-child",
               "--serving-jobs", str(args.serving_jobs), "--serving-load", str(args.serving_load),
               "--budget-gib", str(args.budget_gib), "--serving-repeats", str(args.serving_repeats)]
        child = subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)

    import numpy as np
    import torch

    import paper_0909_2000_amd as wl
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = workloads.config(WORKLOADS[args.workload])
    m, n, w = p.m, p.n, p.w
    rows, cols = m - w, n - w
    log(f"workload {p.name}: m={m} n={n} w={w} -> {rows}x{cols} plot")

    ctx = wl.Context(0)
    # the library's tuning cache: the batch knobs and the tilings that
    # wlcs_tune_plot measured for plot shapes (applied without timing when
    # this device has an entry; other shapes keep the built-in tile model)
    ctx.tune(TUNING_CACHE)
    if args.tile:
        ctx.set_tile(1, 255, args.tile)
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    pair = ctx.pair(p.x, p.y, alphabet=p.alphabet)
    torch.cuda.synchronize()
    encode_ms = (time.perf_counter() - t0) * 1e3
    # plot rows padded to whole 64-byte sectors (a pitched layout; the plot
    # itself is out[:, :cols])
    ld = (cols + args.row_align - 1) // args.row_align * args.row_align
    out = torch.empty((rows, ld), dtype=torch.uint8, device=dev)[:, :cols]
    thr = p.threshold
    bm = torch.empty((rows, (cols + 63) // 64), dtype=torch.int64, device=dev) if thr else None

    def step():
        pair.plot(w, threshold=thr, out=out, bitmap_out=bm, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # timed region: K steps, HIP events on the launch stream around each one
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    ms_per_step = wall * 1e3 / args.steps
    nominal = float(m) * n * w
    value = nominal / (ms_per_step / 1e3)
    log(f"seaweed: {ms_per_step:.3f} ms/step, {value:.3e} window-cells/s")

    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB read + 1 GiB written")

    avg_kernel_ms = float(np.mean(kern_ms))
    cells = float(rows) * n * w  # cells the method combs: m-w strips of w x n
    achieved = cells * OPS_PER_CELL / (avg_kernel_ms / 1e3)
    traffic, traffic_detail = measured_traffic(p.name, cells)
    algo_bytes = float(m + n) * 2 + float(rows) * cols + (float(rows) * ((cols + 63) // 64) * 8 if thr else 0)
    # the device's sustained packed-16-bit rate, measured by the library's
    # probe of independent v_pk_max_u16 chains, beside the published peak
    # (about 28 ms a run: shorter runs read low while the clock ramps up)
    measured_peak = max(ctx.measure_valu_peak(8000) for _ in range(2))
    log(f"measured packed-u16 VALU peak: {measured_peak / 1e12:.1f} TOP/s "
        f"(published {PEAK_U16_OPS / 1e12:.1f})")
    # the library's issue-rate probe: wave64 VALU instructions per second per
    # SIMD at one to four resident waves per SIMD, for packed 16-bit and plain
    # 32-bit streams and for the seaweed cell's own dependency chain (and the
    # same chain with the letter comparison as a 32-bit XOR)
    issue = {kind: [ctx.measure_valu_issue(kind, k) for k in (1, 2, 3, 4)]
             for kind in ("pk16", "b32", "bitop3", "cell", "cell_xor", "cell_two_xor")}
    log("VALU issue probe (M instructions/s per SIMD, 1..4 waves): " +
        "; ".join(f"{k} " + " ".join(f"{r / 1e6:.0f}" for r in v) for k, v in issue.items()))
    launch_s = avg_kernel_ms / 1e3
    if traffic_detail is not None and "write_bytes" in traffic_detail:
        traffic_detail["write_TB_per_s"] = traffic_detail["write_bytes"] / launch_s / 1e12
        traffic_detail["read_TB_per_s"] = traffic_detail["read_bytes"] / launch_s / 1e12
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_U16_OPS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_U16_OPS, "traffic": traffic,
                "traffic_detail": traffic_detail, "algorithmic_bytes": algo_bytes,
                "algorithmic_output_TB_per_s": algo_bytes / launch_s / 1e12,
                "measured_peak": measured_peak / 1e12, "frac_of_measured_peak": achieved / measured_peak,
                "peak_probe": "wlcs_measure_valu_peak: independent v_pk_max_u16 chains on every SIMD",
                "ops_per_cell": OPS_PER_CELL, "cells_per_launch": cells,
                "avg_launch_ms": avg_kernel_ms,
                "valu_issue_probe_instr_per_s_per_simd": {k: [float(r) for r in v] for k, v in issue.items()}}
    valu = (traffic_detail or {}).get("valu")
    if valu and "instructions_per_launch" in valu:
        # the timed kernel's own issue rate: its (deterministic) VALU
        # instruction count over this run's launch time, per SIMD
        simds = 4 * torch.cuda.get_device_properties(dev).multi_processor_count
        roofline["valu_instr_per_s_per_simd"] = valu["instructions_per_launch"] / simds / launch_s

    # serving right after the headline plot: measured after the heavier legs
    # below, its latencies read 30-40% higher (the legs are independent)
    serving = None
    if child is not None:
        child.stdin.write("go\n")
        child.stdin.close()
        line = child.stdout.read()
        if child.wait() != 0:
            raise RuntimeError(f"the serving child exited with {child.returncode}")
        serving = json.loads(line.strip().splitlines()[-1])
        log(f"serving: p50 {serving['at_load']['p50_s'] * 1e3:.1f} ms, p99 "
            f"{serving['at_load']['p99_s'] * 1e3:.1f} ms at {serving['rate_jobs_per_s']:.0f} jobs/s")
        sp = serving["sparse"]
        log(f"serving with dot lists: p50 {sp['at_load']['p50_s'] * 1e3:.1f} ms, p99 "
            f"{sp['at_load']['p99_s'] * 1e3:.1f} ms at {sp['rate_jobs_per_s']:.0f} jobs/s")

    # rows of the timed plot kept for the consistency checks below
    sample_rows = np.array([0, rows // 3, rows - 1])
    sea_rows = out[torch.as_tensor(sample_rows, device=dev)].cpu().numpy()

    cpu, parity = None, None
    if not args.no_cpu:
        # the oracle as it stands, on whole rows of the same plot, sized to
        # about cpu-seconds of host time; the rows it computes are also the
        # parity check of the timed plot
        import oracle
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        oracle.wlcs_rows(p.x, p.y, w, [rows // 2], nthreads=1)
        one_row = time.perf_counter() - t0
        nrows = max(threads, int(args.cpu_seconds * threads / max(one_row, 1e-3)))
        nrows = min(nrows, rows)
        ids = np.linspace(0, rows - 1, nrows).astype(np.int64)
        t0 = time.perf_counter()
        want = oracle.wlcs_rows(p.x, p.y, w, ids, nthreads=threads)
        cpu_s = time.perf_counter() - t0
        parity = bool(np.array_equal(out[torch.as_tensor(ids, device=dev)].cpu().numpy(), want))
        # the oracle's loop-interchanged build (the same recurrence, 64
        # y-windows side by side) on the same rows, for context
        t0 = time.perf_counter()
        want_b = oracle.wlcs_batch(p.x, p.y, w, rows=ids, nthreads=threads)
        batch_s = time.perf_counter() - t0
        info = cpu_info()
        cpu = {"value": nrows * float(n) * w / cpu_s, "unit": "window-cells/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{nrows} of {rows} plot rows (x-windows spread evenly), each against all "
                         f"{cols} y-windows, plain per-window DP, {cpu_s:.1f} s",
               "one_core_value": float(n) * w / one_row, "cpu_model": info.get("model_name", ""),
               "cpu": info,
               "o_batch_value": nrows * float(n) * w / batch_s,
               "o_batch_equal": bool(np.array_equal(want_b, want))}
        log(f"CPU oracle: {cpu['value']:.3e} window-cells/s on {threads} threads "
            f"(O-batch {cpu['o_batch_value']:.3e}); timed plot equals it on those {nrows} rows: {parity}")

    dp = None
    if not args.no_dp:
        # plain per-window DP on the same GPU, the same plot (one untimed run
        # on a slice first, then one timed full run)
        small = ctx.pair(p.x[: 64 + w], p.y, alphabet=p.alphabet)
        small.plot_dp(w, out=out[:64])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pair.plot_dp(w, threshold=thr, out=out, bitmap_out=bm, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        dp_ms = a.elapsed_time(b)
        dp_same = bool(np.array_equal(out[torch.as_tensor(sample_rows, device=dev)].cpu().numpy(), sea_rows))
        dp = {"value": nominal / (dp_ms / 1e3), "unit": "window-cells/s", "ms": dp_ms,
              "speedup_seaweed_over_dp": dp_ms / ms_per_step, "equals_seaweed_on_sampled_rows": dp_same}
        log(f"GPU DP: {dp_ms:.1f} ms, seaweed speedup {dp_ms / ms_per_step:.1f}x")
        # bit-parallel LCS per window pair (the BLCS comparison of Section 4)
        pair.plot_blcs(w, out=out[:64])  # warm-up on a slice
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pair.plot_blcs(w, threshold=thr, out=out, bitmap_out=bm, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        blcs_ms = a.elapsed_time(b)
        dp["blcs"] = {"value": nominal / (blcs_ms / 1e3), "ms": blcs_ms,
                      "speedup_seaweed_over_blcs": blcs_ms / ms_per_step,
                      "equals_seaweed_on_sampled_rows":
                          bool(np.array_equal(out[torch.as_tensor(sample_rows, device=dev)].cpu().numpy(), sea_rows))}
        log(f"GPU BLCS: {blcs_ms:.1f} ms, seaweed speedup {blcs_ms / ms_per_step:.1f}x")

    others = None
    if not args.no_configs:
        others = {}
        for k in (1, 3):
            if WORKLOADS[args.workload] == k:
                continue  # already the headline workload
            others[workloads.config(k).name] = bench_config(ctx, torch, workloads, k)
            log(f"config {k}: {others[workloads.config(k).name]}")

    wide = None
    if not args.no_configs:
        wide = bench_wide(ctx, torch, workloads)
        log("windows of 129..255 letters (30,000 x 30,000 protein): " + ", ".join(
            f"w={w} {v['ms']:.2f} ms ({v['roofline_frac']:.2f})" for w, v in wide["plots"].items()))

    paper_shapes = None
    if not args.no_paper_shapes:
        paper_shapes = bench_paper_shapes(ctx, torch, workloads)
        for k, v in paper_shapes.items():
            log(f"{k}: {v['ms']:.1f} ms (paper: Sea-8 {v['paper_sea8_s']} s on 1 core, MPI "
                f"{v['paper_mpi_s']} s on {v['paper_mpi_cores']} cores)")

    batched = None
    if not args.no_batch:
        batched = bench_batch(ctx, torch, workloads)
        log(f"batched: {batched['value']:.3e} window-cells/s over {batched['pairs']} pairs "
            f"({batched['ms']:.1f} ms; graph replay {batched['graph_ms']:.1f} ms)")

    step5 = None
    if not args.no_configs:
        step5 = bench_step5(ctx, torch, workloads)
        log(f"step 5 (paper's vertical step): {step5['ms']:.2f} ms, {step5['dots']} dots, "
            f"DP {step5['dp_ms']:.1f} ms ({step5['speedup_over_dp']:.0f}x)")

    dots_filter = None
    if not args.no_configs:
        dots_filter = bench_dots_filter(ctx, torch, workloads)
        log("dot list at WLCS >= 48, every strip: {:.2f} ms; probe filter: {}".format(
            dots_filter["plain_ms"], ", ".join(f"h={h} {v['ms']:.2f} ms" for h, v in dots_filter["filtered"].items())))

    rec = {
        "metric": METRIC, "value": value, "unit": "window-cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": p.name, "m": m, "n": n, "w": w, "rows": rows, "cols": cols, "ld": ld,
                   "threshold": thr, "outputs": "uint8 plot + bitmap" if thr else "uint8 plot",
                   "parallelism": "single GPU",
                   "tiling": dict(zip(("long_tile", "short_tile", "long_pairs"), ctx.plot_tiling(rows, cols, w)),
                                  source="measured (tuning cache)" if any(ctx.plot_tiling(rows, cols, w))
                                  else "built-in tile model")},
        "roofline": roofline, "cpu_baseline": cpu, "gpu_dp_baseline": dp,
        "other_configs": others, "wide_windows": wide, "paper_shaped_score_plots": paper_shapes,
        "batched": batched, "serving": serving, "step5_lcs_plot": step5, "dot_list_filter": dots_filter,
        "encode_ms": encode_ms, "parity_sampled_rows": parity,
        "kernel_ms": {"min": float(np.min(kern_ms)), "median": float(np.median(kern_ms)),
                      "max": float(np.max(kern_ms))},
    }
    print(json.dumps(rec), flush=True)
    pair.close()
    ctx.close()


def bench_batch(ctx, torch, workloads, reps=3):
    """256 DNA pairs of uneven m, n and w in persistent launches (eager and
    graph-replayed), outputs preallocated, pairs resident."""
    import numpy as np
    pairs = workloads.batch_config()
    specs = [{"pair": ctx.pair(p.x, p.y), "w": p.w} for p in pairs]
    # the built-in batch knobs first (the context has the cache applied)
    ctx.set_batch_grid(0)
    ctx.set_batch_tile(1, 128, 0)
    res = ctx.batch(specs)  # allocates the outputs once (and warms up)
    for sp, r in zip(specs, res):
        sp["out"] = r["wlcs"]
    default_ms = float(np.median([_timed_once(torch, lambda: ctx.batch(specs)) for _ in range(3)]))
    # the library's tuner: applies this device's entry of the committed cache
    # (or times the candidates and adds an entry when the device has none)
    ctx.tune(TUNING_CACHE)
    tuning = {"batch_tiles": {f"{lo}-{hi}": ctx.batch_tile(hi) for lo, hi in ((1, 16), (17, 32), (33, 64), (65, 128))},
              "batch_grid": ctx.batch_grid()}
    graph = ctx.batch_graph(specs)
    graph.launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def timed(fn):
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms))

    eager_ms = timed(lambda: ctx.batch(specs))
    graph_ms = timed(lambda: graph.launch())
    nominal = sum(float(p.m) * p.n * p.w for p in pairs)
    graph.close()
    out = {"pairs": len(pairs), "window_cells": nominal, "ms": eager_ms, "graph_ms": graph_ms,
           "tuned": True, "untuned_ms": default_ms, "tuning": tuning,
           "value": nominal / (eager_ms / 1e3), "graph_value": nominal / (graph_ms / 1e3),
           "unit": "window-cells/s", "workload": "256 iid DNA pairs, m,n ~ U[1000,20000], w ~ {16,32,64,128}"}
    del specs, res
    torch.cuda.empty_cache()
    return out


def bench_config(ctx, torch, workloads, k, steps=10):
    """Seaweed plot and GPU DP on another single-pair configuration; the two
    GPU plots are compared whole (the oracle's parity at these sizes is the
    test suite's)."""
    import numpy as np
    p = workloads.config(k)
    rows, cols = p.m - p.w, p.n - p.w
    pair = ctx.pair(p.x, p.y, alphabet=p.alphabet)
    out = torch.empty((rows, cols), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        pair.plot(p.w, out=out)
    ms = float(np.median([_timed_once(torch, lambda: pair.plot(p.w, out=out)) for _ in range(steps)]))
    dp_out = torch.empty_like(out)
    dp_ms = _timed_once(torch, lambda: pair.plot_dp(p.w, out=dp_out))
    dp_same = bool(torch.equal(out, dp_out))
    pair.plot_blcs(p.w, out=dp_out)  # warm-up
    blcs_ms = _timed_once(torch, lambda: pair.plot_blcs(p.w, out=dp_out))
    nominal = float(p.m) * p.n * p.w
    cells = float(rows) * p.n * p.w
    res = {"m": p.m, "n": p.n, "w": p.w, "ms": ms, "value": nominal / (ms / 1e3),
           "unit": "window-cells/s", "roofline_frac": cells * OPS_PER_CELL / (ms / 1e3) / PEAK_U16_OPS,
           "dp_ms": dp_ms, "dp_value": nominal / (dp_ms / 1e3), "speedup_over_dp": dp_ms / ms,
           "dp_equals_seaweed": dp_same, "blcs_ms": blcs_ms, "speedup_over_blcs": blcs_ms / ms,
           "blcs_equals_seaweed": bool(torch.equal(out, dp_out))}
    if ms < 0.5:
        # a launch-bound plot: also time it captured in a HIP graph, 100 plots
        # per replay (the plot call enqueues kernels only: no allocation, no
        # memset), the per-plot time taken over the replay
        reps = 100
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            pair.plot(p.w, out=out, stream=cap)  # warm-up on the capture stream
            cap.synchronize()
            with torch.cuda.graph(graph, stream=cap):
                for _ in range(reps):
                    pair.plot(p.w, out=out, stream=cap)
        torch.cuda.current_stream().wait_stream(cap)
        graph.replay()
        torch.cuda.synchronize()
        g_ms = float(np.median([_timed_once(torch, graph.replay) for _ in range(5)])) / reps
        graph_same = bool(torch.equal(out, dp_out))
        res.update({"graph_ms_per_plot": g_ms, "graph_value": nominal / (g_ms / 1e3),
                    "graph_roofline_frac": cells * OPS_PER_CELL / (g_ms / 1e3) / PEAK_U16_OPS,
                    "graph_equals_blcs": graph_same})
        del graph
    pair.close()
    del out, dp_out
    torch.cuda.empty_cache()
    return res


def bench_wide(ctx, torch, workloads, widths=(150, 200, 255), steps=5):
    """Plain plots with windows of 129..255 letters (the 256-row class, a
    chain of four waves per strip) on the 30,000 x 30,000 protein pair; at
    w = 200 the plot is compared whole with the GPU BLCS baseline's."""
    import numpy as np
    p = workloads.config(3)
    pair = ctx.pair(p.x, p.y, alphabet=p.alphabet)
    plots = {}
    blcs = None
    for w in widths:
        rows, cols = p.m - w, p.n - w
        out = torch.empty((rows, cols), dtype=torch.uint8, device="cuda")
        pair.plot(w, out=out)
        ms = float(np.median([_timed_once(torch, lambda: pair.plot(w, out=out)) for _ in range(steps)]))
        cells = float(rows) * p.n * w
        plots[w] = {"ms": ms, "value": float(p.m) * p.n * w / (ms / 1e3), "unit": "window-cells/s",
                    "roofline_frac": cells * OPS_PER_CELL / (ms / 1e3) / PEAK_U16_OPS}
        if w == 200:
            ref = torch.empty_like(out)
            pair.plot_blcs(w, out=ref)
            blcs_ms = _timed_once(torch, lambda: pair.plot_blcs(w, out=ref))
            blcs = {"w": w, "ms": blcs_ms, "speedup_seaweed_over_blcs": blcs_ms / ms,
                    "equals_seaweed": bool(torch.equal(out, ref))}
            del ref
        del out
        torch.cuda.empty_cache()
    pair.close()
    return {"workload": f"{p.name}, windows {', '.join(str(w) for w in widths)}", "plots": plots, "blcs": blcs}


# The paper's experiments (Section 4, Table 1): alignment-score plots with
# w = 100 (window 200 after the blow-up) and a vertical step of 5 on four
# biological pairs.  The sequences are not available; iid DNA of the same
# lengths stands in (the seaweed method's time does not depend on content).
# (m, n, Sea-16 1 core s, Sea-8 1 core s, fastest MPI run s, its cores)
PAPER_SHAPES = {
    "berti-2712x2305": (2712, 2305, 10.8, 3.8, 1.3, 4),
    "jimmy-15kx97k": (15000, 97000, 1026.0, 368.0, 11.0, 64),
    "henry-80kx80k": (80000, 80000, 4514.0, 1614.0, 23.0, 64),
}


def bench_paper_shapes(ctx, torch, workloads):
    """Alignment-score plots at the paper's experimental shapes, timed with
    HIP events (strings uploaded, blown up and encoded inside each call)."""
    import numpy as np
    out = {}
    for name, (m, n, sea16, sea8, mpi, mpi_cores) in PAPER_SHAPES.items():
        g = workloads.rng(500 + m % 97)
        x, y = workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)
        w, step = 100, 5
        res = ctx.score_plot(x, y, w, step=step)  # allocates and warms up
        S = res["score"]
        ms = float(np.median([_timed_once(torch, lambda: ctx.score_plot(x, y, w, step=step, out=S))
                              for _ in range(7)]))
        cells = float(S.shape[0]) * (2 * n) * (2 * w)
        out[name] = {"m": m, "n": n, "w": w, "step": step, "rows": S.shape[0], "cols": S.shape[1],
                     "ms": ms, "blown_up_cells_per_s": cells / (ms / 1e3),
                     "paper_sea16_s": sea16, "paper_sea8_s": sea8, "paper_mpi_s": mpi,
                     "paper_mpi_cores": mpi_cores,
                     "data": "iid uniform DNA of the paper's lengths (datasets not available)"}
        del res, S
    torch.cuda.empty_cache()
    return out


def _timed_once(torch, fn):
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def serving_child(args):
    """The serving leg alone (a child process of the benchmark): waits for a
    line on stdin, serves, prints one JSON line on stdout."""
    if sys.stdin.readline().strip() != "go":
        return  # the parent ended before the serving leg (its end of the pipe closed)
    import torch

    import workloads
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rep = bench_serving(None, torch, workloads, args)
    rep["process"] = "a child of bench.py that had not used the GPU before the serving leg"
    print(json.dumps(rep), flush=True)


def bench_serving(ctx, torch, workloads, args):
    """Poisson stream of DNA/protein jobs (bitmap + indel outputs): capacity
    with every job queued at once, then latency at a fraction of it."""
    from paper_0909_2000_amd import serve
    jobs = workloads.serving_jobs(rate=1.0, njobs=args.serving_jobs)
    budget = int(args.budget_gib * (1 << 30))

    def run(rate_scale, all_at_once=False, dots=False, d2h=False):
        reqs = serve.requests_from_workload(jobs, rate_scale=rate_scale, dots=dots)
        if all_at_once:
            for r in reqs:
                r.arrival = 0.0
        ex = serve.GpuExecutor(0, streams=4, d2h_bitmaps=d2h)  # its own context, latency tiles
        srv = serve.Server(ex, budget_bytes=budget, max_jobs=256, max_batch=64, keep_results=False)
        rep = srv.run(reqs)
        torch.cuda.synchronize()
        return rep  # the output memory stays cached for the next run (same streams)

    run(1.0, all_at_once=True)  # warm-up (untimed): the executor streams' memory, staging slots
    sat = run(1.0, all_at_once=True)
    capacity = sat["jobs_per_s"]
    rate = args.serving_load * capacity
    # arrivals were drawn at 1 job/s: compress them to `rate`; the headline
    # point is run several times and the median run is reported, with the
    # spread of its p50 and p99
    reps = [run(rate) for _ in range(max(1, args.serving_repeats))]
    order = sorted(range(len(reps)), key=lambda k: reps[k]["p99_s"])
    at = reps[order[len(order) // 2]]
    at["repeats"] = {"p50_s": [r["p50_s"] for r in reps], "p99_s": [r["p99_s"] for r in reps],
                     "jobs_per_s": [r["jobs_per_s"] for r in reps]}
    log(f"serving at {args.serving_load:.2f} x capacity, {len(reps)} runs: p99 "
        + ", ".join(f"{r['p99_s'] * 1e3:.1f}" for r in reps) + " ms")
    # a fixed arrival rate, comparable whatever the capacity
    fixed = run(FIXED_RATE)
    log(f"serving at {FIXED_RATE:.0f} jobs/s: p50 {fixed['p50_s'] * 1e3:.1f} ms, p99 {fixed['p99_s'] * 1e3:.1f} ms")
    sweep = {}
    for load in (0.25, 0.5, 0.9):
        r = run(load * capacity)
        sweep[str(load)] = {"rate_jobs_per_s": load * capacity, "p50_s": r["p50_s"], "p99_s": r["p99_s"],
                            "jobs_per_s": r["jobs_per_s"]}
        log(f"serving at {load:.2f} x capacity: p50 {r['p50_s'] * 1e3:.1f} ms, p99 {r['p99_s'] * 1e3:.1f} ms")
    # the same stream with dot lists (window starts, WLCS, indel distance of
    # every pair at or above the threshold) in place of the dense outputs
    sat_s = run(1.0, all_at_once=True, dots=True)
    rate_s = args.serving_load * sat_s["jobs_per_s"]
    at_s = run(rate_s, dots=True)
    # last (it pins host memory for every job's bitmap): each job's latency
    # running until its bitmap is in host memory
    at_d2h = run(rate, d2h=True)
    log(f"serving with bitmap D2H: p50 {at_d2h['p50_s'] * 1e3:.1f} ms, p99 {at_d2h['p99_s'] * 1e3:.1f} ms")
    torch.cuda.empty_cache()
    return {"jobs": len(jobs), "capacity_jobs_per_s": capacity, "saturated": sat,
            "load": args.serving_load, "rate_jobs_per_s": rate, "at_load": at, "load_sweep": sweep,
            "at_load_with_bitmap_d2h": at_d2h,
            "at_fixed_rate": {"rate_jobs_per_s": FIXED_RATE, "p50_s": fixed["p50_s"], "p99_s": fixed["p99_s"],
                              "jobs_per_s": fixed["jobs_per_s"]},
            "budget_gib": args.budget_gib,
            "workload": "Poisson arrivals; DNA/protein 1:1; m,n log-uniform [500,50000]; "
                        "w ~ {16,32,64,128}; outputs bitmap (T=ceil(3w/4)) + uint16 indel",
            "batch_tiles": {f"{lo}-{hi}": t for (lo, hi), t in serve.LATENCY_TILES.items()},
            "batch_grid": serve.LATENCY_GRID,
            "sparse": {"capacity_jobs_per_s": sat_s["jobs_per_s"], "saturated": sat_s,
                       "rate_jobs_per_s": rate_s, "at_load": at_s,
                       "outputs": "dot list (12-byte records: i, j, WLCS, indel) at T=ceil(3w/4), "
                                  "first capacity max(4096, windows/64) per job, jobs with more "
                                  "dots rerun with an exact list"}}


def bench_dots_filter(ctx, torch, workloads, reps=5):
    """The 50,000 x 50,000 DNA pair's dot list at WLCS >= 48 (every window
    pair, w = 64): the plain dot list of every strip, then the exact probe
    filter at several probe steps (only every h-th strip combed, the rows in
    reach of the threshold evaluated one by one); every filtered list is
    compared with the plain one."""
    import numpy as np
    import paper_0909_2000_amd as wl
    p = workloads.config(2)
    pair = ctx.pair(p.x, p.y)
    cap = 4 << 20
    dots = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    count = torch.empty(1, dtype=torch.int64, device="cuda")

    def plain():
        pair.plot_strided(p.w, 1, 1, threshold=p.threshold, want_plot=False, dots_out=dots, count_out=count)

    plain()
    torch.cuda.synchronize()
    plain_ms = float(np.median([_timed_once(torch, plain) for _ in range(reps)]))
    want, n_want = wl.dot_records({"dots": dots, "dot_count": count})
    out = {"m": p.m, "n": p.n, "w": p.w, "threshold": p.threshold, "dots": n_want, "plain_ms": plain_ms,
           "filtered": {}}
    for h in (2, 4, 6, 8, 12):
        def filt():
            pair.dots_filtered(p.w, p.threshold, probe_step=h, dots_out=dots, count_out=count)
        filt()
        torch.cuda.synchronize()
        ms = float(np.median([_timed_once(torch, filt) for _ in range(reps)]))
        got, n_got = wl.dot_records({"dots": dots, "dot_count": count})
        out["filtered"][str(h)] = {"ms": ms, "speedup": plain_ms / ms,
                                   "equal": bool(n_got == n_want and np.array_equal(got, want))}
    pair.close()
    del dots
    torch.cuda.empty_cache()
    return out


def bench_step5(ctx, torch, workloads, reps=5):
    """The 50,000 x 50,000 DNA pair, w = 64, at the paper's vertical step of
    5 (every fifth x-window against every y-window, Section 3's step size):
    seaweed plot with the dot list at WLCS >= 48, and the plain per-window DP
    with the same step on the same GPU; the two plots are compared whole and
    the dot list with the plot's entries at or above the threshold on sampled
    rows."""
    import numpy as np
    p = workloads.config(2)
    w, hx = p.w, 5
    pair = ctx.pair(p.x, p.y)
    rows = -(-(p.m - w) // hx)
    cols = p.n - w
    out = torch.empty((rows, cols), dtype=torch.uint8, device="cuda")
    dots = torch.empty((1 << 20, 3), dtype=torch.int32, device="cuda")
    count = torch.empty(1, dtype=torch.int64, device="cuda")

    def sea():
        pair.plot_strided(w, hx, 1, threshold=p.threshold, out=out, dots_out=dots, count_out=count)

    sea()
    torch.cuda.synchronize()
    ms = float(np.median([_timed_once(torch, sea) for _ in range(reps)]))
    res = {"wlcs": out, "dots": dots, "dot_count": count}
    import paper_0909_2000_amd as wl
    recs, n_dots = wl.dot_records(res)
    sample = np.array([0, rows // 2, rows - 1])
    plot_rows = out[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    dots_ok = all({int(j) for j in np.nonzero(row >= p.threshold)[0]} ==
                  {int(d["j"]) for d in recs[recs["i"] == r * hx]} for r, row in zip(sample, plot_rows))
    dp_out = torch.empty_like(out)
    dp_ms = _timed_once(torch, lambda: pair.plot_dp_strided(w, hx, 1, out=dp_out, want_plot=True))
    dp_ok = bool(torch.equal(dp_out, out))
    pair.close()
    cells = float(rows) * p.n * w  # x-windows compared x n x w
    del out, dp_out, dots
    torch.cuda.empty_cache()
    return {"m": p.m, "n": p.n, "w": w, "hx": hx, "rows": rows, "cols": cols, "ms": ms,
            "window_cells_per_s": cells / (ms / 1e3), "dots": n_dots, "dots_match_plot_rows": dots_ok, "dp_ms": dp_ms, "speedup_over_dp": dp_ms / ms,
            "dp_equals_seaweed": dp_ok,
            "outputs": "uint8 plot of every 5th x-window + dot list at WLCS >= 48"}


if __name__ == "__main__":
    main()
