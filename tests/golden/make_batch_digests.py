"""Write the oracle's digest of every plot of the batched configuration (256
DNA pairs, m and n uniform in [1,000, 20,000], w from {16, 32, 64, 128}, seed
4).

    python tests/golden/make_batch_digests.py [--threads N]

About 25 minutes on eight cores.  Each plot comes from the oracle's O-batch
(pinned equal to the plain dynamic program); batch_plots.txt holds one line
per pair: its index, w, rows, columns and the BLAKE2b-64 digest (hex) of the
plot's bytes, row-major.  Only the oracle and the seeded input generators are
used.
"""
import argparse
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None)
    args = ap.parse_args()
    threads = args.threads or len(os.sched_getaffinity(0))
    lines = ["# batched configuration (256 DNA pairs, seed 4): oracle plots",
             "# pair w rows cols blake2b-64(plot bytes, row-major)"]
    t0 = time.time()
    for k, p in enumerate(workloads.batch_config()):
        plot = oracle.wlcs_batch(p.x, p.y, p.w, nthreads=threads)
        d = hashlib.blake2b(plot.tobytes(), digest_size=8).hexdigest()
        lines.append(f"{k} {p.w} {plot.shape[0]} {plot.shape[1]} {d}")
        print(f"pair {k}: w={p.w} {plot.shape}, {time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "batch_plots.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("written", len(lines) - 2, "plots")


if __name__ == "__main__":
    main()
