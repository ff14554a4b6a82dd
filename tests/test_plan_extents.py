"""CPU: the batch planner and the kernels' unit decode stay inside every buffer.

``tests/native/plan_extents.cpp`` builds the library's host runtime into a
program with AddressSanitizer and UndefinedBehaviorSanitizer (host code only,
g++; no GPU) and, for random job mixes, follows every unit the batched and
single-plot launches would run: the tile pair and strip block each ticket or
workgroup decodes to, the x and y codes it reads, and the plot, bitmap,
indel, strided and dot outputs it writes.  Every read must lie inside the
pair's code arrays, every write inside the caller's buffers, and every plot
entry and bitmap word of every strip block must be written by exactly one
unit.  The mixes cover last-pair table entries, full-range plots, x and y
steps, dot lists with and without records, empty jobs, batch tiles up to
32,768 windows and windows above 128 (single-plot launches with two-length
tilings); the benchmark's plot shapes run with the built-in tilings.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "plan_extents.cpp")
ROCM = "/opt/rocm"


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_extents")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", SRC, "-o", exe,
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_units_stay_in_bounds(harness, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([harness, str(seed), "60"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout
