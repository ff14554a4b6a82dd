"""Write the oracle's digests of every job of the 2,000-job serving stream whose
strings satisfy m * n <= 1e7 (the stream of the serving configuration: seed 5,
DNA and protein, m and n log-uniform in [500, 50,000], w in {16, 32, 64, 128};
the jobs do not depend on the arrival rate).

    python tests/golden/make_serving_digests.py [--threads N]

About two minutes on eight cores.  Each plot comes from the oracle's O-batch
(pinned equal to the plain dynamic program); the file serving_small_jobs.txt
holds one line per job: its index, w, rows, columns and the BLAKE2b-64 digest
(hex) of the plot's bytes, row-major.  Only the oracle and the seeded input
generators are used.
"""
import argparse
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

LIMIT = 10_000_000  # m * n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None)
    args = ap.parse_args()
    threads = args.threads or len(os.sched_getaffinity(0))
    jobs = workloads.serving_jobs(rate=1.0, njobs=2000)
    lines = ["# serving stream (2,000 jobs, seed 5): jobs with m * n <= 1e7, oracle plots",
             "# jid w rows cols blake2b-64(plot bytes, row-major)"]
    for j in jobs:
        p = j.pair
        if p.m * p.n > LIMIT:
            continue
        plot = oracle.wlcs_batch(p.x, p.y, p.w, nthreads=threads)
        d = hashlib.blake2b(plot.tobytes(), digest_size=8).hexdigest()
        lines.append(f"{j.jid} {p.w} {plot.shape[0]} {plot.shape[1]} {d}")
    with open(os.path.join(HERE, "serving_small_jobs.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"written {len(lines) - 2} jobs")


if __name__ == "__main__":
    main()
