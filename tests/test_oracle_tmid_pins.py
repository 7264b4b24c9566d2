"""Pins of the oracle's free-t_mid templates (Eq. 6 with all six random numbers), checked
without its integer formula:

* rows from a 50-digit evaluation of the definition itself -- the root xi(t) of the time
  Bezier in [0, 1], then the frequency Bezier at xi -- with exact rational arithmetic wherever
  the value is rational (a perfect-square discriminant), so exact row boundaries are decided
  exactly;
* t_mid at the midpoint reduces to the plain rasteriser; the end rows are floor(f0/256) and
  floor(f2/256); reversing time (and the control points) reverses the rows;
* the draw keeps the plain template's fields and puts t1 uniformly in [t0, t2].
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

D10MS = 2684355

mpmath = pytest.importorskip("mpmath")


def _row_reference(t0, t1, t2, f0, f1, f2, t, dps=50):
    """floor(f(xi)/256) at column t, from the definition: a xi^2 + b xi + (t0 - t) = 0, xi in [0, 1]."""
    a, b, c = t0 - 2 * t1 + t2, 2 * (t1 - t0), t0 - t
    def freq(xi):
        return (1 - xi) ** 2 * f0 + 2 * xi * (1 - xi) * f1 + xi ** 2 * f2
    if a == 0:
        return math.floor(freq(Fraction(-c, b)) / 256)
    D = b * b - 4 * a * c
    s = math.isqrt(D)
    if s * s == D:  # rational root: exact
        xi = Fraction(-b + s, 2 * a)
        return math.floor(freq(xi) / 256)
    with mpmath.workdps(dps):
        xi = (-b + mpmath.sqrt(D)) / (2 * a)
        v = freq(xi) / 256
        r = int(mpmath.floor(v))
        # an irrational value (U + V sqrt(D))/W keeps a distance of at least 1/(W (|U| + |V| sqrt(D) + W))
        # from every integer: above 1e-32 for T <= 2896 and F <= 32767, far above the working precision
        assert abs(v - mpmath.nint(v)) > mpmath.mpf("1e-40")
    return r


def test_rows_against_the_definition(orc):
    rng = np.random.default_rng(31)
    F = 40
    for it in range(400):
        T = int(rng.integers(2, 60))
        t0 = int(rng.integers(0, T - 1))
        t2 = int(rng.integers(t0 + 1, T))
        t1 = int(rng.integers(t0, t2 + 1)) if it % 5 else (t0 if it % 10 else t2)  # include both extremes
        f = [int(x) for x in rng.integers(0, F * 256, 3)]
        if it % 7 == 0:
            f = [256 * int(x) for x in rng.integers(0, F, 3)]  # row boundaries hit exactly
        tr = np.array([(t0, t1, t2, f[0], f[1], f[2], 0)], dtype=orc.TRACK_TM_DTYPE)
        got = orc.rows_tm(tr, F)
        want = [_row_reference(t0, t1, t2, f[0], f[1], f[2], t) for t in range(t0, t2 + 1)]
        assert got.tolist() == want, (t0, t1, t2, f)


def test_rows_against_the_definition_at_full_size(orc):
    """The same definition at the sizes the kernels run: T up to 2896 columns, F up to 32767 rows,
    sampled columns of long templates (60-digit evaluation), including near-linear time (t1 close to
    the midpoint, where the elimination's integers are largest relative to the row) and both ends."""
    rng = np.random.default_rng(34)
    for it in range(240):
        T = int(rng.choice([1000, 2000, 2896]))
        F = int(rng.choice([1000, 2000, 32767]))
        t0 = int(rng.integers(0, T // 3))
        t2 = int(rng.integers(max(t0 + 2, T - T // 3), T))
        mid = (t0 + t2) // 2
        if it % 4 == 0:
            t1 = mid + int(rng.integers(-2, 3))  # a = t0 - 2 t1 + t2 within a few units of 0
        else:
            t1 = int(rng.integers(t0, t2 + 1))
        t1 = min(max(t1, t0), t2)
        f = [int(x) for x in rng.integers(0, F * 256, 3)]
        if it % 6 == 0:
            f = [256 * int(x) for x in rng.integers(0, F, 3)]
        tr = np.array([(t0, t1, t2, f[0], f[1], f[2], 0)], dtype=orc.TRACK_TM_DTYPE)
        got = orc.rows_tm(tr, F)
        cols = np.unique(np.concatenate([[t0, t0 + 1, t2 - 1, t2], rng.integers(t0, t2 + 1, 24)]))
        for t in cols:
            want = _row_reference(t0, t1, t2, f[0], f[1], f[2], int(t), dps=60)
            assert int(got[t - t0]) == want, (T, F, t0, t1, t2, f, int(t))


def test_midpoint_reduces_to_plain_rasteriser_and_end_rows(orc):
    rng = np.random.default_rng(32)
    F, T = 300, 2896
    for _ in range(300):
        t0 = int(rng.integers(0, T - 2))
        t2 = t0 + 2 * int(rng.integers(1, (T - 1 - t0) // 2 + 1))
        f = [int(x) for x in rng.integers(0, F * 256, 3)]
        tm = np.array([(t0, (t0 + t2) // 2, t2, *f, 0)], dtype=orc.TRACK_TM_DTYPE)
        plain = np.array([(t0, t2, *f, 0)], dtype=orc.TRACK_DTYPE)
        assert orc.rows_tm(tm, F).tolist() == orc.rows(plain[0], F).tolist()
        t1 = int(rng.integers(t0, t2 + 1))
        tm["t1"] = t1
        r = orc.rows_tm(tm, F)
        assert r[0] == f[0] >> 8 and r[-1] == f[2] >> 8
        assert ((r >= 0) & (r < F)).all()


def test_time_reversal_reverses_rows(orc):
    rng = np.random.default_rng(33)
    F, T = 128, 700
    for _ in range(200):
        t0 = int(rng.integers(0, T - 2))
        t2 = int(rng.integers(t0 + 1, T))
        t1 = int(rng.integers(t0, t2 + 1))
        f = [int(x) for x in rng.integers(0, F * 256, 3)]
        fwd = np.array([(t0, t1, t2, f[0], f[1], f[2], 0)], dtype=orc.TRACK_TM_DTYPE)
        rev = np.array([(T - 1 - t2, T - 1 - t1, T - 1 - t0, f[2], f[1], f[0], 0)], dtype=orc.TRACK_TM_DTYPE)
        assert orc.rows_tm(rev, F).tolist() == orc.rows_tm(fwd, F)[::-1].tolist()


def test_draw_keeps_plain_fields_and_t1_is_uniform(orc):
    T, F, L = 400, 100, 10
    tm = orc.draw_tm_many(12, 3, 5000, 20000, T, F, L, D10MS)
    pl = orc.draw_many(12, 3, 5000, 20000, T, F, L, D10MS)
    for name in ("t0", "t2", "f0", "f1", "f2", "dtau"):
        assert np.array_equal(tm[name], pl[name])
    assert ((tm["t1"] >= tm["t0"]) & (tm["t1"] <= tm["t2"])).all()
    u = (tm["t1"] - tm["t0"] + 0.5) / (tm["t2"] - tm["t0"] + 1)  # position of t1 in [t0, t2]
    h, _ = np.histogram(u, bins=10, range=(0, 1))
    chi2 = ((h - h.mean()) ** 2 / h.mean()).sum()
    assert chi2 < 40  # 9 degrees of freedom; a biased draw lands far above


def test_score_midpoint_equals_plain_score(orc):
    import synth
    T, F = 120, 80
    Y, s = synth.noise_map(T, F, seed=95, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    pl = orc.draw_many(7, 0, 0, 300, T, F, 10, D10MS)
    pl = pl[(pl["t0"] + pl["t2"]) % 2 == 0]
    tm = np.zeros(pl.size, dtype=orc.TRACK_TM_DTYPE)
    for name in ("t0", "t2", "f0", "f1", "f2", "dtau"):
        tm[name] = pl[name]
    tm["t1"] = (pl["t0"] + pl["t2"]) // 2
    assert np.array_equal(orc.score_tm_list(m, tm), orc.score_list(m, pl))
