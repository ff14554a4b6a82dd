"""GPU: staging slots of a context (pinned host buffer + device buffer per
slot, made as needed up to 256, reused once the encode that read them ran).

Pairs are created back to back, more of them than the context keeps slots,
on a stream kept busy by long plots, so slots are still pending when later
pairs need them; every pair's codes must still be right (its plots equal the
oracle).  Strings longer than a slot's first size make it grow."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_more_pairs_in_flight_than_staging_slots(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    ctx = wl.Context(0)
    s = torch.cuda.Stream()
    g = workloads.rng(90)
    bx, by = workloads.iid(g, 50_000, workloads.DNA), workloads.iid(g, 50_000, workloads.DNA)
    big = ctx.pair(bx, by, stream=s)
    out = torch.empty((50_000 - 64, 50_000 - 64), dtype=torch.uint8, device="cuda")
    for _ in range(2):  # about 20 ms of work ahead of the pairs on the same stream
        big.plot(64, out=out, stream=s)
    strings = []
    for k in range(300):
        m, n = int(g.integers(40, 300)), int(g.integers(40, 300))
        strings.append((workloads.iid(g, m, workloads.DNA), workloads.iid(g, n, workloads.DNA)))
    print("creating 300 pairs behind two long plots", flush=True)
    pairs = [ctx.pair(x, y, stream=s) for x, y in strings]
    # a pair longer than the slots' first size (1 MiB of letters) makes a slot grow
    lx = workloads.iid(g, 700_000, workloads.DNA)
    ly = workloads.iid(g, 600_000, workloads.DNA)
    long_pair = ctx.pair(lx, ly, stream=s)
    torch.cuda.synchronize()  # the plots below run on the default stream, which reads them back
    for k in list(range(0, 300, 29)) + [255, 256, 299]:
        x, y = strings[k]
        got = pairs[k].plot(16)["wlcs"].cpu().numpy()
        np.testing.assert_array_equal(got, oracle_mod.wlcs(x, y, 16), err_msg=f"pair {k}")
    got = long_pair.plot_strided(32, 5000, 1000)["wlcs"].cpu().numpy()
    np.testing.assert_array_equal(got, oracle_mod.wlcs_strided(lx, ly, 32, 5000, 1000))
