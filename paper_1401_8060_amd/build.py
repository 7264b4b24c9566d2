"""Build libstt.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libstt.so")
SOURCES = ["stt_api.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are left to no one: the compiler may not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; libstt needs ROCm to build")
    return p


# The issue-rate probe (vector-ALU rates of the scorers' instructions), a measurement aid of its
# own: bench.py --issue-rates loads it; nothing on the search path does.
PROBE_LIB = os.path.join(PKG, "libstt_probe.so")
PROBE_SOURCES = ["probe_issue.hip"]


def _hipcc_shared(sources: list[str], out: str, verbose: bool, extra: list[str] | None) -> str:
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, *(extra or []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    _hipcc_shared(PROBE_SOURCES, PROBE_LIB, verbose, extra)
    return _hipcc_shared(SOURCES, LIB, verbose, extra)


if __name__ == "__main__":
    print(build(verbose=True))
