"""Pins of the sky-patch delay prior (Sec. VI: draw the delay from a patch of sky instead of the
isotropic prior), checked on the draw itself:

* every field but the delay is the isotropic draw's, and the delay is that draw's moved by the
  patch centre (the same random word, so the shift is exact);
* delays stay in [c - D, c + D], both ends are reached, and the histogram is flat;
* a patch of zero width (D = 0) is a fixed delay: the targeted search of Eq. 5 at that delay.
"""
from __future__ import annotations

import numpy as np
import pytest

D10MS = 2684355


def test_patch_moves_only_the_delay(orc):
    a = orc.draw_many(3, 1, 100, 5000, 500, 200, 10, D10MS)
    for c in (0, 123456, -D10MS // 2, (1 << 30) - 1 - D10MS):
        b = orc.draw_patch_many(3, 1, 100, 5000, 500, 200, 10, D10MS, c)
        for name in ("t0", "t2", "f0", "f1", "f2"):
            assert np.array_equal(a[name], b[name])
        assert np.array_equal(b["dtau"].astype(np.int64), a["dtau"].astype(np.int64) + c)


def test_patch_range_and_flatness(orc):
    D, c = 40, -700
    b = orc.draw_patch_many(9, 0, 0, 40_000, 100, 50, 10, D, c)
    d = b["dtau"].astype(np.int64)
    assert d.min() == c - D and d.max() == c + D
    h = np.bincount(d - (c - D), minlength=2 * D + 1)
    chi2 = ((h - h.mean()) ** 2 / h.mean()).sum()
    assert chi2 < 2 * D + 1 + 6 * np.sqrt(2 * (2 * D + 1))  # 80 degrees of freedom


def test_zero_width_patch_is_a_fixed_delay(orc):
    b = orc.draw_patch_many(4, 2, 0, 1000, 200, 64, 10, 0, 8051)
    assert (b["dtau"] == 8051).all()
    with pytest.raises(ValueError):
        orc.draw_patch_many(4, 2, 0, 10, 200, 64, 10, D10MS, (1 << 30) - D10MS)
