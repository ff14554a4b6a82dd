"""Write per-row digests of the full alignment plots of the 50,000 x 50,000 DNA
pair (w = 64, bitmap at WLCS >= 48) and the 30,000 x 30,000 protein pair
(w = 128), computed by the oracle.

    python tests/golden/make_plot_digests.py [--threads N]

Takes about five minutes on eight cores.  The plots come from the oracle's
O-batch (the plain dynamic program of every window pair, evaluated for 64
neighbouring y-windows at once; pinned equal to the scalar oracle entry by
entry in tests/test_oracle.py), a block of rows at a time.  For each pair:

* plot_rows_<name>.u64: one 8-byte BLAKE2b digest of each plot row (the row's
  bytes, cols of them), little-endian, in row order;
* plot_digests.json: the workload, the shape, the SHA-256 of the whole plot
  (rows concatenated), of the digest file, and for the DNA pair the SHA-256 of
  the thresholded bitmap (the oracle's dot_bitmap layout, row by row).

Only the oracle and the seeded input generators are used.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

BLOCK = 2048  # rows per oracle call


def row_digest(row: np.ndarray) -> bytes:
    return hashlib.blake2b(row.tobytes(), digest_size=8).digest()


def digest_plot(cfg: int, threads: int) -> dict:
    p = workloads.config(cfg)
    rows, cols = p.m - p.w, p.n - p.w
    plot_sha = hashlib.sha256()
    bm_sha = hashlib.sha256() if p.threshold else None
    digests = bytearray()
    t0 = time.time()
    for r0 in range(0, rows, BLOCK):
        ids = np.arange(r0, min(rows, r0 + BLOCK), dtype=np.int64)
        block = oracle.wlcs_batch(p.x, p.y, p.w, rows=ids, nthreads=threads)
        for row in block:
            digests += row_digest(row)
            plot_sha.update(row.tobytes())
        if bm_sha is not None:
            bm_sha.update(np.ascontiguousarray(oracle.dot_bitmap(block, p.threshold)).tobytes())
        done = r0 + ids.size
        print(f"{p.name}: {done}/{rows} rows, {time.time() - t0:.0f} s", flush=True)
    fname = f"plot_rows_{p.name}.u64"
    with open(os.path.join(HERE, fname), "wb") as f:
        f.write(bytes(digests))
    rec = {"workload": p.name, "config": cfg, "m": p.m, "n": p.n, "w": p.w, "rows": rows, "cols": cols,
           "row_digest": "blake2b-64 of each row's bytes, little-endian u64 per row",
           "row_digests_file": fname, "row_digests_sha256": hashlib.sha256(bytes(digests)).hexdigest(),
           "plot_sha256": plot_sha.hexdigest()}
    if bm_sha is not None:
        rec["threshold"] = p.threshold
        rec["bitmap_sha256"] = bm_sha.hexdigest()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None)
    args = ap.parse_args()
    threads = args.threads or len(os.sched_getaffinity(0))
    recs = [digest_plot(2, threads), digest_plot(3, threads)]
    with open(os.path.join(HERE, "plot_digests.json"), "w") as f:
        json.dump({"generator": "tests/golden/make_plot_digests.py (oracle O-batch)", "plots": recs}, f,
                  indent=1)
        f.write("\n")
    print("written", [r["row_digests_file"] for r in recs])


if __name__ == "__main__":
    main()
