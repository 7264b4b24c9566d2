"""Compile the oracle's C sources into ``oracle/libstt_oracle.so`` with gcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["stt_oracle.c", "stt_oracle_ext.c"]


def lib_path() -> str:
    """The built library; STT_ORACLE_LIB names another build of these sources instead (the tests'
    planted-mistake copies)."""
    return os.environ.get("STT_ORACLE_LIB") or os.path.join(HERE, "libstt_oracle.so")


def build(verbose: bool = False) -> str:
    out = lib_path()
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out
