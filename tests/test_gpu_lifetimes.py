"""GPU: a resident pair released while a plot on another stream still reads it.

The pair's codes are freed in stream order on its creation stream; the
library records an event on every other stream that reads them and makes the
creation stream wait for it before the free.  Here a plot of the pair is
queued on stream B behind long plots, the pair is released at once, and a new
pair of the same sizes is made on the creation stream A: in A's order its
codes take the freed memory, so without the wait its encoding would overwrite
the first pair's codes before B's plot reads them.  Both plots must equal the
oracle."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_pair_released_while_another_stream_reads_it(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    dev = torch.device("cuda", 0)
    ctx = wl.Context(0)
    g = workloads.rng(3100)
    w = 32
    x, y = workloads.iid(g, 1500, workloads.DNA), workloads.iid(g, 2600, workloads.DNA)
    x2, y2 = workloads.iid(g, 1500, workloads.DNA), workloads.iid(g, 2600, workloads.DNA)
    want, want2 = oracle_mod.wlcs(x, y, w), oracle_mod.wlcs(x2, y2, w)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    bx, by = workloads.iid(g, 40000, workloads.DNA), workloads.iid(g, 40000, workloads.DNA)
    with torch.cuda.stream(b):
        big = ctx.pair(bx, by, stream=b)
        big_out = torch.empty((40000 - 64, 40000 - 64), dtype=torch.uint8, device=dev)
        out = torch.empty(want.shape, dtype=torch.uint8, device=dev)
    p = ctx.pair(x, y, stream=a)
    a.synchronize()
    b.synchronize()
    for rep in range(2):
        print(f"release under a queued plot, round {rep}", flush=True)
        out.fill_(0xA5)
        torch.cuda.synchronize()
        for _ in range(3):  # some 20 ms of work ahead on b
            big.plot(64, out=big_out, stream=b)
        p.plot(w, out=out, stream=b)
        p.close()  # while b has not reached the plot
        p = ctx.pair(x2, y2, stream=a)  # same sizes: reuses the freed codes in a's order
        b.synchronize()
        a.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        res = p.plot(w, stream=a)
        a.synchronize()
        np.testing.assert_array_equal(res["wlcs"].cpu().numpy(), want2)
        x, y, x2, y2, want, want2 = x2, y2, x, y, want2, want
    p.close()
    big.close()
    torch.cuda.synchronize()
