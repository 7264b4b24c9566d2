"""CPU oracle for the seedless-clustering track search (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. It wraps ``stt_oracle.c`` (plain single-threaded
FP64 C, compiled with gcc) through ctypes and shares no code with the HIP
library in ``paper_1401_8060_amd``.
"""
from .oracle import *  # noqa: F401,F403
from .build import build, lib_path  # noqa: F401
from . import mapform, significance  # noqa: F401,E402
