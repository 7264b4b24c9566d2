"""Pins of the oracle's delay-maximised statistic (a reading of "phase-maximised": the maximum
of Eq. 8 over a grid of delays per template), checked without the oracle's per-pixel loop.

* Constant-row templates: every pixel has the same frequency f, so Eq. 8 is
  Re[e^{2 pi i f dtau} * sum(p)] / sqrt(N) -- one complex sum and one exponential per delay,
  with the phase taken exactly from integers.
* Conjugating the map mirrors the statistic in the delay (S*(dtau) = S(-dtau)), so the maximum
  over a grid equals the maximum over the reversed, negated grid on the conjugate map.
* The reported delay index attains the maximum, and the maximum dominates every grid member.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth

D10MS = 2684355


def _const_row_track(t0, t2, fq8, dtau=0):
    return np.array([(t0, t2, fq8, fq8, fq8, dtau)], dtype=[("t0", "<i4"), ("t2", "<i4"), ("f0", "<u4"),
                                                              ("f1", "<u4"), ("f2", "<u4"), ("dtau", "<i4")])


def _closed_form(Y, s, t0, t2, row, fq4_lo, dfq4, delays):
    p = (Y[t0:t2 + 1, row].astype(np.complex128) / s[t0:t2 + 1, row].astype(np.float64)).sum()
    fq4 = fq4_lo + row * dfq4
    z = []
    for d in delays:
        turns = ((fq4 * int(d)) % 2 ** 32) / 2 ** 32  # (fq4/16 Hz)(d 2^-28 s), exact before the division
        z.append((np.exp(2j * math.pi * turns) * p).real / math.sqrt(t2 - t0 + 1))
    return np.array(z)


@pytest.mark.parametrize("d0,step,nt", [(-D10MS, 2 * D10MS // 7, 8), (-1000, 250, 9), (12345, 0, 1), (0, 97, 33),
                                        (7, 0, 5)])  # step 0: all delays tie, the lowest index wins
def test_constant_row_closed_form(orc, d0, step, nt):
    T, F = 64, 40
    Y, s = synth.noise_map(T, F, seed=91, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s, fq4_lo=1600, dfq4=16)
    rng = np.random.default_rng(7)
    for _ in range(20):
        t0 = int(rng.integers(0, T - 12))
        t2 = int(rng.integers(t0 + 1, T))
        row = int(rng.integers(0, F))
        fq8 = row * 256 + int(rng.integers(0, 256))  # any point inside the row keeps the row
        z, mm = orc.score_maxdelay_list(m, _const_row_track(t0, t2, fq8, dtau=777), d0, step, nt)
        want = _closed_form(Y, s, t0, t2, row, 1600, 16, [d0 + k * step for k in range(nt)])
        assert z[0] == pytest.approx(want.max(), abs=1e-12)
        assert mm[0] == int(np.argmax(want))  # first maximum = lowest index


def test_conjugate_map_mirrors_the_delay(orc):
    T, F = 80, 50
    Y, s = synth.noise_map(T, F, seed=92, sigma=("loguniform", 0.5, 2.0))
    m, mc = orc.Map(Y, s), orc.Map(np.conj(Y), s)
    idx = np.arange(200, dtype=np.uint64)
    d0, step, nt = -D10MS, 2 * D10MS // 10, 11
    z, mm = orc.score_maxdelay_gen_idx(m, 5, 0, 10, D10MS, idx, d0, step, nt)
    d0r = -(d0 + (nt - 1) * step)  # the negated grid, in increasing order
    zc, mc_idx = orc.score_maxdelay_gen_idx(mc, 5, 0, 10, D10MS, idx, d0r, step, nt)
    assert np.allclose(z, zc, rtol=0, atol=1e-12)
    # the maximising delay maps to its mirror (index nt-1-m) unless two grid delays tie
    assert (mc_idx == nt - 1 - mm).mean() > 0.99


def test_reported_delay_attains_the_maximum(orc):
    T, F = 120, 64
    Y, s = synth.noise_map(T, F, seed=93, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    idx = np.arange(300, dtype=np.uint64)
    d0, step, nt = -D10MS, 2 * D10MS // 15, 16
    z, mm = orc.score_maxdelay_gen_idx(m, 6, 2, 10, D10MS, idx, d0, step, nt)
    tr = np.concatenate([orc.draw_many(6, 2, int(j), 1, T, F, 10, D10MS) for j in idx])
    for k in range(nt):
        zk, _ = orc.score_maxdelay_list(m, tr, d0 + k * step, 0, 1)
        assert (z >= zk).all()
        hit = mm == k
        assert np.array_equal(z[hit], zk[hit])
    # one delay equal to the template's own reproduces the plain statistic
    own = tr["dtau"][:10]
    for i in range(10):
        zi, _ = orc.score_maxdelay_list(m, tr[i:i + 1], int(own[i]), 0, 1)
        assert zi[0] == orc.score_list(m, tr[i:i + 1])[0]


def test_invalid_template_and_bad_grid(orc):
    Y, s = synth.noise_map(30, 20, seed=94, sigma="unit")
    m = orc.Map(Y, s)
    z, mm = orc.score_maxdelay_list(m, _const_row_track(5, 5, 10), -100, 10, 4)  # t2 <= t0: invalid
    assert math.isnan(z[0]) and mm[0] == -1
    with pytest.raises(ValueError):
        orc.score_maxdelay_list(m, _const_row_track(0, 9, 10), 2 ** 30 - 5, 10, 4)  # leaves the delay range
    with pytest.raises(ValueError):
        orc.score_maxdelay_list(m, _const_row_track(0, 9, 10), 0, 10, 0)
