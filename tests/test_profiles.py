"""The committed rocprofv3 summaries stay current and their commands runnable.

The counter file feeds the bench line's measured HBM traffic and VALU detail
only while the kernel sources still hash to the digest recorded with it; the
summaries' commands use committed files and options bench.py still has.
"""
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _bench_options():
    with open(os.path.join(ROOT, "bench.py")) as f:
        return set(re.findall(r'add_argument\(\s*"(--[a-z0-9-]+)"', f.read()))


def _logical_lines(text):
    """Lines with backslash continuations joined, as the shell reads them."""
    return re.sub(r"\\\n\s*", " ", text).splitlines()


def _include_closure(src):
    """The file and every header it reaches by quoted includes."""
    seen, todo = set(), [src]
    while todo:
        rel = todo.pop()
        if rel in seen:
            continue
        seen.add(rel)
        with open(os.path.join(ROOT, rel)) as f:
            for inc in re.findall(r'^\s*#include\s+"([^"]+)"', f.read(), re.M):
                todo.append(os.path.join(os.path.dirname(rel), inc))
    return seen


def test_counter_file_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    files = glob.glob(os.path.join(PROFILES, "seaweed_counters_*.json"))
    assert files
    for path in files:
        with open(path) as f:
            d = json.load(f)
        for fn in d["digest_files"]:
            assert os.path.exists(os.path.join(ROOT, fn)), fn
        traffic, detail = bench.measured_traffic(d["workload"], 1.0)
        # stale: re-take the FETCH_SIZE, WRITE_SIZE and VALU runs its summary
        # lists, then bench.py --write-counters
        assert traffic is not None, detail
        # two counter runs of the same launch agree, and the plain copy that
        # scales them was counted
        assert len(d["fetch_kib_per_dispatch"]) >= 2 and len(d["write_kib_per_dispatch"]) >= 2
        w = d["write_kib_per_dispatch"]
        assert max(w) / min(w) < 1.01
        assert d["copy_write_kib"] > 0 and d["copy_fetch_kib"] > 0
        # the digest covers every source the kernel is built from: its file
        # and the headers it includes, directly or through each other
        assert d["digest_files"] == bench.COUNTER_DIGEST_FILES
        assert set(d["digest_files"]) == _include_closure(d["digest_files"][0])
        # the VALU run's launch time and GRBM_COUNT belong to one launch: they
        # give a shader clock the chip can run at, with its CUs busy
        assert 1.5 < detail["valu"]["clock_ghz"] < 2.5
        assert 0.9 < detail["valu"]["cu_busy_share"] <= 1.0


def test_summary_commands_use_committed_files_and_existing_options():
    options = _bench_options()
    assert {"--steps", "--warmup", "--write-counters"} <= options
    mds = sorted(glob.glob(os.path.join(PROFILES, "*.md")))
    assert mds
    for md in mds:
        with open(md) as f:
            text = f.read()
        name = os.path.basename(md)
        assert "_work/" not in text, name
        seen = 0
        for line in _logical_lines(text):
            for head in ("bench.py", 'BASE="'):
                if head in line:
                    tail = line.split(head, 1)[1].split("#", 1)[0]
                    for opt in re.findall(r"(?<![\w-])--[a-z0-9][a-z0-9-]*", tail):
                        assert opt in options, f"{name}: bench.py has no {opt}"
                        seen += 1
        assert seen, f"{name} names no bench.py command"
