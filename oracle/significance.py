"""Oracle of the significance stage (test infrastructure only).

Plain Python over FP32 scores. The search records the maximum statistic of every map (Sec. V),
so background maps (time slides) give a sample of the per-map maximum in noise. A foreground
map's false-alarm probability is the fraction of background maxima at least as loud as its own,
and the detection threshold for FAP < alpha (0.1 % in Sec. IV) is the ceil(alpha n_bg)-th largest
background maximum: a foreground value strictly above it has fewer than alpha n_bg louder
background maps.

Scores are read from the 64-bit best keys of the scorer (score in the high word as ordered
FP32 bits, so a NaN score was already stored as -inf); an empty key (0) is quieter than every
score. The comparison is on the FP32 value, the precision the keys carry.
"""
from __future__ import annotations

import math
import struct


def key_score(key: int) -> float:
    """The FP32 score in a best key; -inf for an empty key (0)."""
    if key == 0:
        return -math.inf
    hi = (key >> 32) & 0xFFFFFFFF
    bits = hi ^ 0x80000000 if hi & 0x80000000 else (~hi) & 0xFFFFFFFF  # undo the order-preserving map
    return struct.unpack("<f", struct.pack("<I", bits))[0]


def _louder_or_equal(kr: int, kq: int) -> bool:
    """Reference at least as loud as the query; an empty key is quieter than any score (-inf
    included) and as loud as another empty key."""
    if kq == 0:
        return True
    if kr == 0:
        return False
    return key_score(kr) >= key_score(kq)


def count_louder(ref_keys, q_keys) -> list[int]:
    """For each query key, how many reference keys are at least as loud."""
    ref = [int(k) for k in ref_keys]
    return [sum(1 for r in ref if _louder_or_equal(r, int(q))) for q in q_keys]


def fap(bg_keys, fg_keys) -> list[float]:
    """Empirical false-alarm probability of each foreground maximum against the background."""
    n = len(bg_keys)
    return [c / n for c in count_louder(bg_keys, fg_keys)]


def threshold(bg_keys, alpha: float) -> float:
    """The ceil(alpha n_bg)-th largest background score (at least the largest one); an empty
    key counts as -inf here."""
    z = sorted((key_score(int(k)) for k in bg_keys), reverse=True)
    m = max(1, math.ceil(alpha * len(z)))
    return z[m - 1]
