"""CPU: the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/oracle_sanitize.c links oracle/wlcs_oracle.c with the sanitizers
and calls every entry point on seeded random strings (windows 1..255, empty
and single-window plots, the full range, thread counts up to 9): the plain
plot, O-batch, selected rows, single entries, strided sub-grids, the textbook
table and the score plot must agree, bad arguments must be refused, and no
access may leave its buffer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    out = str(tmp_path_factory.mktemp("osan") / "oracle_sanitize")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-pthread",
                    os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"),
                    os.path.join(ROOT, "oracle", "wlcs_oracle.c"), "-o", out],
                   check=True, capture_output=True, text=True)
    return out


@pytest.mark.parametrize("seed", [11, 12])
def test_oracle_entry_points_under_sanitizers(exe, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(seed), "25"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout
