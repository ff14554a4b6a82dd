"""GPU: the whole 2,000-job serving stream, every job checked as it completes.

The serving configuration's stream (seed 5: DNA and protein, m and n
log-uniform in [500, 50,000], w in {16, 32, 64, 128}, bitmap at ceil(3w/4) and
indel distance) runs through the serving loop as the benchmark runs it (HBM
budget of 64 GiB, four executor streams, continuous batching, arrivals at
1,200 jobs/s so batches overlap).  As each job completes, before its outputs
are released:

* every job with m * n <= 1e7 (636 of them): the plot recovered from its
  indel distances (WLCS = w - indel / 2) equals the oracle's, by the per-job
  digests in tests/golden/serving_small_jobs.txt (written by
  tests/golden/make_serving_digests.py from the oracle alone), and its bitmap
  equals the thresholded plot;
* a seeded sample of 520 jobs of every size: its bitmap and indel distances
  equal the job run alone on the device, on a stream of its own, from the
  same resident strings;
* 20 seeded jobs among the larger ones: two seeded rows of each plot (from
  its indel distances) equal the oracle's rows of that job.
"""
import hashlib
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _small_digests():
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "serving_small_jobs.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            jid, w, rows, cols, d = line.split()
            out[int(jid)] = (int(w), int(rows), int(cols), d)
    return out


def _bitmap_of(plot: np.ndarray, thr: int) -> np.ndarray:
    rows, cols = plot.shape
    words = (cols + 63) // 64
    bits = np.zeros((rows, words * 64), dtype=np.uint8)
    bits[:, :cols] = plot >= thr
    return np.packbits(bits, axis=1, bitorder="little").view("<u8").reshape(rows, words)


def test_every_job_of_the_serving_stream(oracle_mod):
    import torch
    from paper_0909_2000_amd import serve

    small = _small_digests()
    assert len(small) == 636
    jobs = workloads.serving_jobs(rate=1.0, njobs=2000)
    reqs = serve.requests_from_workload(jobs, rate_scale=1200.0)
    sample = set(int(k) for k in workloads.rng(5050).choice(len(reqs), 520, replace=False))
    g = workloads.rng(5060)
    large = sorted(r.jid for r in reqs if r.jid not in small)
    rows_checked = {int(j): None for j in g.choice(large, 20, replace=False)}
    alone_stream = torch.cuda.Stream()
    seen = {"oracle": 0, "alone": 0, "oracle_rows": 0}
    bad = []

    def on_done(req, res):
        bm, ind = res["bitmap"], res["indel"]
        if req.jid in small:
            w, rows, cols, want = small[req.jid]
            assert (w, rows, cols) == (req.w, ind.shape[0], ind.shape[1]), req.jid
            d = ind.cpu().numpy().view(np.uint16)
            plot = (req.w - d // 2).astype(np.uint8)
            if (hashlib.blake2b(plot.tobytes(), digest_size=8).hexdigest() != want or
                    not np.array_equal(bm.cpu().numpy().view("<u8"), _bitmap_of(plot, req.threshold))):
                bad.append(("oracle", req.jid))
            seen["oracle"] += 1
        if req.jid in rows_checked:
            d = ind.cpu().numpy().view(np.uint16)
            picks = np.sort(workloads.rng(5070 + req.jid).choice(d.shape[0], 2, replace=False))
            want = oracle_mod.wlcs_rows(req.x, req.y, req.w, picks)
            if not np.array_equal((req.w - d[picks] // 2).astype(np.uint8), want):
                bad.append(("oracle rows", req.jid))
            seen["oracle_rows"] += 1
        if req.jid in sample:
            pair = res["_pair"]  # the job's own resident strings
            alone = pair.plot(req.w, threshold=req.threshold, indel=True, want_plot=False, stream=alone_stream)
            alone_stream.synchronize()
            if not (torch.equal(alone["bitmap"], bm) and torch.equal(alone["indel"], ind)):
                bad.append(("alone", req.jid))
            seen["alone"] += 1
            del alone

    ex = serve.GpuExecutor(0, streams=4)
    srv = serve.Server(ex, budget_bytes=64 << 30, max_jobs=256, max_batch=64, keep_results=False,
                       on_done=on_done)
    print("serving stream: 2000 jobs at 1,200 jobs/s", flush=True)
    rep = srv.run(reqs)
    torch.cuda.synchronize()
    print("report", rep, "checked", seen, flush=True)
    assert rep["rejected"] == 0 and rep["overlapped_launches"] > 0
    assert seen == {"oracle": 636, "alone": 520, "oracle_rows": 20}
    assert not bad, bad[:20]
