"""Pins of the significance oracle (per-map maxima of background maps -> false-alarm probability
and the FAP < alpha threshold), checked against values fixed by the IEEE format and by hand:

* the high word of a best key is the order-preserving image of the FP32 score: 0x80000000 is
  +0, 0xBF800000 is 1.0, 0x407FFFFF is -1.0, 0x007FFFFF is -inf;
* hand-worked counts with ties, -inf and empty keys;
* a ladder of distinct scores 1 .. 1000: FAP and thresholds by counting;
* i.i.d. Gumbel maxima: the empirical FAP follows the exact survival function within a few
  binomial standard deviations.
"""
from __future__ import annotations

import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def sg():
    from oracle import significance
    return significance


def _key(hi: int, j: int = 0) -> int:
    return (hi << 32) | (0xFFFFFFFF - j)


def _key_of(z: float, j: int = 0) -> int:
    bits = int(np.float32(z).view(np.uint32))
    hi = bits ^ 0x80000000 if not bits & 0x80000000 else (~bits) & 0xFFFFFFFF
    return _key(hi, j)


def test_key_high_word_constants(sg):
    assert sg.key_score(_key(0x80000000)) == 0.0
    assert sg.key_score(_key(0xBF800000, 7)) == 1.0
    assert sg.key_score(_key(0x407FFFFF)) == -1.0
    assert sg.key_score(_key(0x007FFFFF)) == -math.inf
    assert sg.key_score(0) == -math.inf
    z = np.sort(np.random.default_rng(3).standard_normal(200).astype(np.float32))
    assert [sg.key_score(_key_of(float(v))) for v in z] == [float(v) for v in z]


def test_counts_by_hand(sg):
    ref = [_key_of(2.0), _key_of(1.0), _key_of(1.0, 5), _key_of(-3.0), _key(0x007FFFFF), 0]
    q = [_key_of(1.0), _key_of(2.5), _key_of(-3.0), _key(0x007FFFFF), 0, _key_of(-10.0)]
    # ties count as louder; -inf beats an empty key; an empty query is beaten by everything
    assert sg.count_louder(ref, q) == [3, 0, 4, 5, 6, 4]


def test_ladder_fap_and_threshold(sg):
    bg = [_key_of(float(v), v) for v in range(1, 1001)]
    assert sg.fap(bg, [_key_of(995.5), _key_of(1000.0), _key_of(1001.0), _key_of(0.5)]) == [0.005, 0.001, 0.0, 1.0]
    assert sg.threshold(bg, 0.001) == 1000.0
    assert sg.threshold(bg, 0.01) == 991.0
    assert sg.threshold(bg, 1e-6) == 1000.0  # fewer maps than 1/alpha: the loudest one
    assert sg.threshold(bg, 1.0) == 1.0
    assert sg.threshold(bg, 0.0025) == 998.0  # alpha n = 2.5: the 3rd largest
    # the threshold separates by FAP: at it FAP >= alpha, just above it FAP < alpha
    for alpha in (0.0025, 0.0137, 0.3333):
        zt = sg.threshold(bg, alpha)
        above = float(np.nextafter(np.float32(zt), np.float32(np.inf)))
        assert sg.fap(bg, [_key_of(above)])[0] < alpha <= sg.fap(bg, [_key_of(zt)])[0]


def test_gumbel_maxima_fap(sg):
    rng = np.random.default_rng(11)
    n = 20000
    bg = [_key_of(float(v), i) for i, v in enumerate(rng.gumbel(size=n).astype(np.float32))]
    zs = [0.0, 1.0, 2.0, 3.0, 4.0]
    got = sg.fap(bg, [_key_of(z) for z in zs])
    for z, f in zip(zs, got):
        p = 1.0 - math.exp(-math.exp(-z))
        assert abs(f - p) <= 5 * math.sqrt(p * (1 - p) / n) + 1 / n
