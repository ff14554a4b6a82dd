"""GPU: plots captured in a HIP graph and replayed.

A pair plot, a strided plot and a sparse dot list enqueue kernels only (no
allocation, no memset: counters are cleared by a small kernel), so a caller
can capture a run of them once and replay it.  Each replay here is checked
against the oracle, with the outputs overwritten and other plots run eagerly
between the replays, so that a replay which leaned on state left by the
capture (or by an earlier replay) fails."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_oracle(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    dev = torch.device("cuda", 0)
    ctx = wl.Context(0)
    g = workloads.rng(2024)
    xa, ya = workloads.iid(g, 2100, workloads.DNA), workloads.iid(g, 1700, workloads.DNA)
    xb, yb = workloads.iid(g, 900, workloads.PROTEIN), workloads.iid(g, 1000, workloads.PROTEIN)
    xc, yc = workloads.iid(g, 1300, workloads.DNA), workloads.iid(g, 1200, workloads.DNA)
    yc[300:500] = xc[600:800]  # a homology, so the dot list is not empty
    wa, wb, (wc, hx, hy) = 64, 100, (32, 2, 3)
    want_a = oracle_mod.wlcs(xa, ya, wa)
    want_b = oracle_mod.wlcs(xb, yb, wb)
    want_c = oracle_mod.wlcs_strided(xc, yc, wc, hx, hy)
    thr_a, thr_c = int(np.quantile(want_a, 0.99)), int(np.quantile(want_c, 0.99))
    dots_c = oracle_mod.dot_list(want_c, wc, thr_c, hx, hy)
    assert dots_c.size > 0

    pa = ctx.pair(xa, ya)
    pb = ctx.pair(xb, yb, alphabet=workloads.PROTEIN)
    pc = ctx.pair(xc, yc)
    out_a = torch.empty(want_a.shape, dtype=torch.uint8, device=dev)
    bm_a = torch.empty((want_a.shape[0], (want_a.shape[1] + 63) // 64), dtype=torch.int64, device=dev)
    ind_a = torch.empty(want_a.shape, dtype=torch.int16, device=dev)
    out_b = torch.empty(want_b.shape, dtype=torch.uint8, device=dev)
    out_c = torch.empty(want_c.shape, dtype=torch.uint8, device=dev)
    dots = torch.empty((dots_c.size + 8, 3), dtype=torch.int32, device=dev)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    outs = (out_a, bm_a, ind_a, out_b, out_c, dots, count)

    def enqueue(stream):
        pa.plot(wa, threshold=thr_a, indel=True, out=out_a, bitmap_out=bm_a, indel_out=ind_a, stream=stream)
        pb.plot(wb, out=out_b, stream=stream)
        return pc.plot_strided(wc, hx, hy, threshold=thr_c, out=out_c, dots_out=dots, count_out=count,
                               stream=stream)

    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        enqueue(cap)  # eager warm-up on the capture stream
        cap.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=cap):
            res_c = enqueue(cap)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()

    other = ctx.pair(workloads.iid(g, 800, workloads.DNA), workloads.iid(g, 900, workloads.DNA))
    for rep in range(3):
        print(f"replay {rep}", flush=True)
        for t in outs:  # garbage in every output, eagerly, outside the graph
            t.fill_(-1 if t.dtype != torch.uint8 else 0xA5)
        other.plot(32, threshold=20, indel=True)  # unrelated eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out_a.cpu().numpy(), want_a)
        np.testing.assert_array_equal(bm_a.cpu().numpy().view("<u8"), oracle_mod.dot_bitmap(want_a, thr_a))
        np.testing.assert_array_equal(ind_a.cpu().numpy().view(np.uint16), oracle_mod.indel(want_a, wa))
        np.testing.assert_array_equal(out_b.cpu().numpy(), want_b)
        np.testing.assert_array_equal(out_c.cpu().numpy(), want_c)
        got, n = wl.dot_records(res_c)
        assert n == dots_c.size
        np.testing.assert_array_equal(got.view(np.uint8), dots_c.view(np.uint8))
    del graph
