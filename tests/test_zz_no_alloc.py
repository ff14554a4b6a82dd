"""GPU: the allocation-free batch (wlcs_batch_noalloc) against wlcs_batch.

Two calls in a row on one stream, the second with fewer and shorter jobs, so
that a table entry, work counter or dot counter left in the device's fixed
scratch by the first call would show.  Each call mixes every window class
(exact and padded, one above 128 that leaves for a single-plot launch),
bitmaps, indel distances, x/y steps and dot lists; every output must equal
what wlcs_batch writes for the same jobs, and the small jobs' plots equal the
oracle.  A batch too large for the scratch is refused before anything is
enqueued."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ESCRATCH = -7


def _mix(ctx, g, njobs, lo, hi):
    ws = (16, 12, 32, 20, 64, 40, 128, 100, 200)
    pairs, specs = [], []
    for k in range(njobs):
        w = ws[k % len(ws)]
        m, n = int(g.integers(lo, hi)) + w, int(g.integers(lo, hi)) + w
        alpha = workloads.DNA if k % 3 else workloads.PROTEIN
        x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
        if n > 400 and m > 260:
            y[100:100 + 200] = x[50:250]  # a homology, so thresholds have dots
        pairs.append((x, y, alpha, ctx.pair(x, y, alphabet=alpha)))
        thr = (3 * w) // 4
        kind = k % 4
        # a list that holds every window pair: never cut short (which dots a
        # full list keeps depends on the order the units finish in)
        cap = max(1, (m - w) * (n - w))
        if kind == 0:
            specs.append({"pair": pairs[-1][3], "w": w, "threshold": thr, "indel": True})
        elif kind == 1:
            specs.append({"pair": pairs[-1][3], "w": w})
        elif kind == 2 and w <= 128:
            specs.append({"pair": pairs[-1][3], "w": w, "hx": 2, "hy": 3, "threshold": thr,
                          "dot_cap": cap})
        else:
            specs.append({"pair": pairs[-1][3], "w": w, "threshold": thr, "dot_cap": cap,
                          "want_plot": False})
    return pairs, specs


def _host(res):
    out = {}
    for key, v in res.items():
        if key in ("dots", "dot_count") or v is None:
            continue
        out[key] = v.cpu().numpy()
    if "dot_count" in res:
        import paper_0909_2000_amd as wl
        recs, count = wl.dot_records(res)  # sorted by window starts (each pair at most once)
        out["dots"] = recs.view(np.uint8)
        out["count"] = count
    return out


def test_noalloc_batch_equals_batch(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    g = workloads.rng(4400)
    stream = torch.cuda.current_stream()
    for call, (njobs, lo, hi) in enumerate([(36, 200, 2500), (9, 40, 700)]):
        print(f"noalloc call {call}: {njobs} jobs", flush=True)
        pairs, specs = _mix(ctx, g, njobs, lo, hi)
        ref = ctx.batch(specs, stream=stream)
        got = ctx.batch_noalloc(specs, stream=stream)
        torch.cuda.synchronize()
        for k, (r, o) in enumerate(zip(ref, got)):
            hr, ho = _host(r), _host(o)
            assert hr.keys() == ho.keys(), k
            for key in hr:
                if key == "count":
                    assert hr[key] == ho[key], (k, key)
                    assert hr[key] <= specs[k]["dot_cap"]
                else:
                    np.testing.assert_array_equal(ho[key], hr[key], err_msg=f"job {k} {key}")
        # the small jobs' dense plots against the oracle as well
        for k, (sp, o) in enumerate(zip(specs, got)):
            x, y, alpha, _ = pairs[k]
            if "wlcs" in o and o["wlcs"] is not None and sp.get("hx", 1) == 1 and x.size * y.size <= 4e6:
                np.testing.assert_array_equal(o["wlcs"].cpu().numpy(), oracle_mod.wlcs(x, y, sp["w"]),
                                              err_msg=f"job {k}")


def test_noalloc_batch_refuses_a_table_beyond_the_scratch():
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    g = workloads.rng(4500)
    x, y = workloads.iid(g, 300, workloads.DNA), workloads.iid(g, 300, workloads.DNA)
    pair = ctx.pair(x, y)
    n = 6200  # one table entry of 184 bytes each: more than the 1 MiB scratch
    counts = torch.full((n,), -5, dtype=torch.int64, device="cuda")
    specs = [{"pair": pair, "w": 16, "threshold": 12, "dot_cap": 0, "want_plot": False,
              "count_out": counts[k:k + 1]} for k in range(n)]
    torch.cuda.synchronize()
    with pytest.raises(wl.WlcsError) as e:
        ctx.batch_noalloc(specs)
    assert e.value.status == ESCRATCH
    torch.cuda.synchronize()
    assert (counts.cpu().numpy() == -5).all()  # nothing was enqueued
    # the same jobs fit a plain batch (its table is allocated per call)
    ctx.batch(specs)
    torch.cuda.synchronize()
    assert (counts.cpu().numpy() >= 0).all()
