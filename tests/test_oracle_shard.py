"""The oracle sharded by template range over host threads equals one call over the whole range,
element for element (template j is a pure function of (seed, stream, j))."""
from __future__ import annotations

import numpy as np

import synth

D10MS = 2684355


def test_sharded_scores_equal_one_call(orc):
    from oracle import shard
    Y, s = synth.noise_map(200, 150, seed=7, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    for first, n, th in ((0, 5003, 4), (123457, 999, 3), (17, 1, 8), (5, 0, 2)):
        want = orc.score_gen(m, 4, 2, 10, D10MS, first, n)
        got = shard.score_gen(m, 4, 2, 10, D10MS, first, n, threads=th)
        assert np.array_equal(got, want)
    idx = np.arange(100, 1300, dtype=np.uint64)
    want = orc.score_tm_gen_idx(m, 4, 2, 10, D10MS, idx)
    assert np.array_equal(shard.score_tm_gen(m, 4, 2, 10, D10MS, 100, 1200, threads=5), want)


def test_host_threads_is_bounded():
    from oracle import shard
    assert 1 <= shard.host_threads() <= shard.MAX_THREADS
