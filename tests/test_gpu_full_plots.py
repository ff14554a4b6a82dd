"""GPU: whole-matrix parity on the full-size plots.

The 50,000 x 50,000 DNA plot at w = 64 (with its bitmap at WLCS >= 48) and
the 30,000 x 30,000 protein plot at w = 128 are computed on the device in the
launch configuration the benchmark times (the tuning cache's measured
tilings, rows padded to 64-byte sectors), and every row is compared with the
oracle's: tests/golden/plot_digests.json and the plot_rows_*.u64 files hold
one 8-byte BLAKE2b digest per row of the oracle's plot, the SHA-256 of the
whole plot and of the bitmap, written by tests/golden/make_plot_digests.py
from the oracle alone.  The DNA plot is also checked with the library's
built-in tiling model.  Any differing row is reported by index."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")
TUNING_CACHE = os.path.join(ROOT, "paper_0909_2000_amd", "tuning_gfx950.json")


def _golden(name):
    with open(os.path.join(GOLD, "plot_digests.json")) as f:
        recs = {r["workload"]: r for r in json.load(f)["plots"]}
    rec = recs[name]
    with open(os.path.join(GOLD, rec["row_digests_file"]), "rb") as f:
        raw = f.read()
    assert hashlib.sha256(raw).hexdigest() == rec["row_digests_sha256"]
    return rec, raw


@pytest.mark.parametrize("cfg,tiling", [(2, "measured"), (2, "model"), (3, "measured")])
def test_full_plot_rows_equal_the_oracle(cfg, tiling):
    import torch
    import paper_0909_2000_amd as wl
    p = workloads.config(cfg)
    rec, raw = _golden(p.name)
    rows, cols = p.m - p.w, p.n - p.w
    assert (rec["rows"], rec["cols"], rec["w"]) == (rows, cols, p.w)
    print(f"full plot {p.name} ({tiling} tiling): {rows} x {cols}", flush=True)
    dev = torch.device("cuda", 0)
    ctx = wl.Context(0)
    if tiling == "measured":
        ctx.tune(TUNING_CACHE)
    pair = ctx.pair(p.x, p.y, alphabet=p.alphabet)
    ld = (cols + 63) // 64 * 64
    out = torch.empty((rows, ld), dtype=torch.uint8, device=dev)[:, :cols]
    thr = p.threshold
    bm = torch.empty((rows, (cols + 63) // 64), dtype=torch.int64, device=dev) if thr else None
    pair.plot(p.w, threshold=thr, out=out, bitmap_out=bm)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    del out
    want = np.frombuffer(raw, dtype="<u8")
    got = np.empty(rows, dtype="<u8")
    whole = hashlib.sha256()
    for r in range(rows):
        b = host[r].tobytes()
        got[r] = int.from_bytes(hashlib.blake2b(b, digest_size=8).digest(), "little")
        whole.update(b)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} rows differ from the oracle, first {bad[:10].tolist()}"
    assert whole.hexdigest() == rec["plot_sha256"]
    if thr:
        assert thr == rec["threshold"]
        assert hashlib.sha256(np.ascontiguousarray(bm.cpu().numpy()).tobytes()).hexdigest() == rec["bitmap_sha256"]
    pair.close()
    ctx.close()
