"""Build the gfx950 library libwlcs.so in place (hipcc, no torch involved).

    python -m paper_0909_2000_amd.build [--verbose]
"""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwlcs.so")
SOURCES = ["api.cpp", "tune.cpp", "seaweed.hip", "dp.hip", "batch.hip", "blcs.hip", "filter.hip", "probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result",
    # packed FP32 instructions stay off (integer kernels, but keep the whole
    # library on the safe side of that feature)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# the compiler's per-kernel resource report (registers, scratch, occupancy)
REPORT = os.path.join(HERE, "kernel_resources.json")
_REMARK = re.compile(r"remark: +(Function Name|VGPRs|AGPRs|SGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]): (\S+)")
_KEYS = {"VGPRs": "vgprs", "AGPRs": "agprs", "SGPRs": "sgprs", "ScratchSize [bytes/lane]": "scratch_bytes",
         "Occupancy [waves/SIMD]": "waves_per_simd", "LDS Size [bytes/block]": "lds_bytes"}


def parse_resources(text: str) -> dict:
    """Kernel (mangled name) -> its resource figures, from the compiler's
    kernel-resource-usage remarks."""
    kernels, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = kernels.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val)
    return kernels


def build(verbose: bool = False, extra: list | None = None, out: str = LIB) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-Rpass-analysis=kernel-resource-usage", *(extra or []), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libwlcs.so")
    other = "\n".join(ln for ln in r.stderr.splitlines()
                      if "kernel-resource-usage" not in ln and ln.strip())
    if verbose and other:
        sys.stderr.write(other + "\n")
    os.replace(tmp, out)
    if out == LIB:
        with open(REPORT + ".tmp", "w") as f:
            json.dump(parse_resources(r.stderr), f, indent=1, sort_keys=True)
        os.replace(REPORT + ".tmp", REPORT)
    return out


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
    print(LIB)
