"""The oracle sharded by template range over host cores (test infrastructure only).

The oracle stays single-threaded: each worker thread runs the unchanged C function on its own
contiguous range of template indices and writes its own slice of the output. ctypes releases the
GIL for the duration of a foreign call, so the ranges run in parallel on separate cores. Template
j is a pure function of (seed, stream, j), so the sharded scores equal one call over the whole
range element for element.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import oracle as _o

MAX_THREADS = 16  # the host share of one GPU on the boxes this runs on


def host_threads() -> int:
    """Cores this process may run on (its affinity mask), at most MAX_THREADS; the environment
    variable STT_ORACLE_THREADS overrides."""
    env = os.environ.get("STT_ORACLE_THREADS")
    if env:
        return max(1, int(env))
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, MAX_THREADS))


def smt_active() -> bool | None:
    """Whether simultaneous multithreading is on (None where the kernel does not say)."""
    try:
        with open("/sys/devices/system/cpu/smt/active") as fh:
            return fh.read().strip() == "1"
    except OSError:
        return None


def _ranges(first: int, n: int, threads: int):
    pieces = max(1, min(n, threads * 8))  # several pieces per thread even out uneven templates
    edges = [first + (n * k) // pieces for k in range(pieces + 1)]
    return [(a, b) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def score_gen(m: "_o.Map", seed: int, stream: int, L: int, D: int, first: int, n: int,
              norm: int = _o.NORM_SQRT_N, threads: int | None = None) -> np.ndarray:
    """Scores of generated templates first .. first+n-1 (as oracle.score_gen), over `threads`
    worker threads."""
    threads = threads or host_threads()
    z = np.zeros(n, dtype=np.float64)
    if n == 0:
        return z
    lib = _o.lib()
    import ctypes as C

    def run(rng):
        a, b = rng
        out = z[a - first:b - first]
        if lib.orc_score_gen(C.byref(m.c), seed, stream, L, D, a, b - a, norm, out.ctypes.data) != 0:
            raise ValueError("invalid parameters")

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, _ranges(first, n, threads)))
    return z


def score_tm_gen(m: "_o.Map", seed: int, stream: int, L: int, D: int, first: int, n: int,
                 norm: int = _o.NORM_SQRT_N, threads: int | None = None) -> np.ndarray:
    """Scores of generated free-t_mid templates first .. first+n-1, over worker threads."""
    threads = threads or host_threads()
    z = np.zeros(n, dtype=np.float64)
    if n == 0:
        return z
    lib = _o.lib()
    import ctypes as C

    def run(rng):
        a, b = rng
        idx = np.arange(a, b, dtype=np.uint64)
        out = z[a - first:b - first]
        if lib.orc_score_tm_gen_idx(C.byref(m.c), seed, stream, L, D, idx.ctypes.data, idx.size, norm,
                                    out.ctypes.data) != 0:
            raise ValueError("invalid parameters")

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, _ranges(first, n, threads)))
    return z
