"""The compiled kernels keep the register budget they were designed for.

The build writes the compiler's resource report of every kernel
(paper_0909_2000_amd/kernel_resources.json).  A kernel whose label and code
arrays no longer fit its registers runs from scratch memory many times
slower (a 256-row class once went from 9 ms to 220 ms that way) and still
gives the right answers, so only this check sees it: no kernel may use more
than a few spill slots of scratch, and the combing kernels run at least at
the waves per SIMD their launch bounds ask for."""
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT = os.path.join(ROOT, "paper_0909_2000_amd", "kernel_resources.json")
MAX_SCRATCH = 128  # bytes per lane: a few spilled temporaries, never an array


@pytest.fixture(scope="module")
def report():
    if not os.path.exists(REPORT):
        pytest.skip("library not built (the build writes the resource report)")
    with open(REPORT) as f:
        rep = json.load(f)
    assert rep, "empty resource report"
    return rep


def _general_waves(wc):
    return 4 if wc <= 32 else 3 if wc <= 64 else 2 if wc <= 128 else 1


def _dl_waves(wc):
    return 3 if wc <= 64 else 2 if wc <= 128 else 1


def test_no_kernel_runs_from_scratch(report):
    bad = {k: v["scratch_bytes"] for k, v in report.items() if v.get("scratch_bytes", 0) > MAX_SCRATCH}
    assert not bad, f"kernels with scratch arrays: {bad}"


def test_combing_kernels_keep_their_occupancy(report):
    seen = set()
    for name, v in report.items():
        occ = v["waves_per_simd"]
        m = re.search(r"14seaweed_kernelILi(\d+)ELb([01])ELi(\d)ELb([01])ELb([01])E", name)
        if m:
            wc, dl = int(m.group(1)), m.group(5) == "1"
            want = _dl_waves(wc) if dl else _general_waves(wc)
            assert occ >= want, (name, occ, want)
            seen.add("dl" if dl else f"general{wc}")
            continue
        m = re.search(r"20seaweed_kernel_splitILi(\d+)E", name)
        if m:
            want = 3 if int(m.group(1)) <= 208 else 2
            assert occ >= want, (name, occ, want)
            seen.add("dl_split")
            continue
        if "21seaweed_kernel_rsplit" in name:
            assert occ >= 3, (name, occ)
            seen.add("rsplit")
            continue
        if "19seaweed_kernel_wide" in name:
            assert occ >= 3 and v.get("agprs", 0) == 0, (name, occ)
            seen.add("wide")
            continue
        m = re.search(r"12batch_kernelILi(\d)E", name)
        if m:
            want = 4 if m.group(1) == "0" else 3
            assert occ >= want, (name, occ, want)
            seen.add(f"batch{m.group(1)}")
            continue
        if "18batch_kernel_split" in name:
            assert occ >= 3, (name, occ)
            seen.add("batch_split")
    assert seen >= {"dl", "general16", "general32", "general64", "wide", "dl_split", "rsplit",
                    "batch0", "batch1", "batch_split"}, seen


def test_no_single_wave_kernel_for_the_256_row_class(report):
    """The 256-row class runs as a chain of four waves per strip;
    no kernel holds a whole 256-row strip in one wave (that needs the
    accumulation registers, at one wave per SIMD)."""
    assert not [k for k in report if "14seaweed_kernelILi256E" in k]
    assert len([k for k in report if "19seaweed_kernel_wide" in k]) == 2  # plain and strided / sparse
