"""GPU parity of the bit-parallel LCS baseline (the BLCS method the paper
compares against in Section 4) with the oracle, through the C ABI
(wlcs_plot_blcs, wlcs_pair_plot_blcs): every window length from 1 to 255
(one to eight 32-bit words, partial last words), DNA and protein, ragged
shapes, the full-range flag, the epilogues, and the 50,000 x 50,000 DNA
pair on sampled rows."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CASES = []
for w in (1, 5, 16, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 200, 255):
    CASES.append((w, w + 1, w + 1))
    CASES.append((w, w + 70, w + 300))  # several chunks of y-windows, ragged strip block


@pytest.mark.parametrize("w,m,n", CASES)
def test_blcs_vs_oracle(oracle_mod, w, m, n):
    import paper_0909_2000_amd as wl
    g = workloads.rng(7000 + 3 * w + m)
    alpha = workloads.PROTEIN if w % 2 else workloads.DNA
    x, y = workloads.iid(g, m, alpha), workloads.iid(g, n, alpha)
    print(f"blcs w={w} m={m} n={n}", flush=True)
    ctx = wl.Context(0)
    got = ctx.plot_blcs(x, y, w, alphabet=alpha)["wlcs"].cpu().numpy()
    np.testing.assert_array_equal(got, oracle_mod.wlcs(x, y, w))


def test_blcs_full_range_and_epilogues(oracle_mod):
    import paper_0909_2000_amd as wl
    g = workloads.rng(71)
    x = workloads.iid(g, 400, workloads.DNA)
    y = np.concatenate([workloads.iid(g, 150, workloads.DNA), x[100:300], workloads.iid(g, 100, workloads.DNA)])
    w, thr = 40, 30
    ctx = wl.Context(0)
    pair = ctx.pair(x, y)
    res = pair.plot_blcs(w, threshold=thr, indel=True, full_range=True)
    want = oracle_mod.wlcs(x, y, w, full_range=True)
    np.testing.assert_array_equal(res["wlcs"].cpu().numpy(), want)
    np.testing.assert_array_equal(res["bitmap"].cpu().numpy().view("<u8"), oracle_mod.dot_bitmap(want, thr))
    np.testing.assert_array_equal(res["indel"].cpu().numpy().view(np.uint16), oracle_mod.indel(want, w))
    # epilogues only (no plot requested)
    res2 = pair.plot_blcs(w, threshold=thr, want_plot=False, full_range=True)
    np.testing.assert_array_equal(res2["bitmap"].cpu().numpy().view("<u8"), oracle_mod.dot_bitmap(want, thr))


def test_blcs_largest_alphabet(oracle_mod):
    import paper_0909_2000_amd as wl
    g = workloads.rng(72)
    alpha = bytes(range(40, 103))  # 63 letters: the largest mask table in LDS
    x, y = workloads.iid(g, 300, alpha), workloads.iid(g, 280, alpha)
    ctx = wl.Context(0)
    for w in (30, 200):
        np.testing.assert_array_equal(ctx.plot_blcs(x, y, w, alphabet=alpha)["wlcs"].cpu().numpy(),
                                      oracle_mod.wlcs(x, y, w))


def test_blcs_full_size_sampled(oracle_mod):
    import torch
    import paper_0909_2000_amd as wl
    p = workloads.config(2)
    ctx = wl.Context(0)
    pair = ctx.pair(p.x, p.y)
    print("blcs full size 50k x 50k w=64", flush=True)
    out = pair.plot_blcs(p.w)["wlcs"]
    torch.cuda.synchronize()
    rows = out.shape[0]
    sample = np.array([0, rows // 2, rows - 1])
    np.testing.assert_array_equal(out[torch.as_tensor(sample, device="cuda")].cpu().numpy(),
                                  oracle_mod.wlcs_rows(p.x, p.y, p.w, sample))
