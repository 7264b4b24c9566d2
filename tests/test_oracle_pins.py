"""Pins of the CPU oracle against things other than itself.

Each test ties one part of the oracle to the paper's closed forms and printed
numbers, to exact rational arithmetic, to a library routine, or to a brute
force evaluation by a different route, chosen so that a dropped term, a wrong
sign, a wrong index or a transposed operand fails at least one of them.
"""
from __future__ import annotations

import math
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
UNIT = Fraction(1, 2 ** 28)  # seconds per delay unit


def _golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return rows


# --------------------------------------------------------------------------- RNG

def test_philox_matches_rocrand_block_function(orc, rocrand_philox):
    sel = np.random.default_rng(20140131)  # picks test counters only
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6,
             [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0]]
    cases += sel.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64).tolist()
    text = "\n".join(" ".join(f"{int(v):x}" for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_philox], input=text, capture_output=True, text=True,
                         check=True).stdout.strip().split("\n")
    assert len(out) == len(cases)
    for c, line in zip(cases, out):
        want = [int(w, 16) for w in line.split()]
        got = orc.philox4x32_10(c[:4], c[4:]).tolist()
        assert got == want, (c, got, want)


# --------------------------------------------------------------------------- template draw

@pytest.mark.parametrize("T,L", [(10, 10), (11, 10), (12, 10), (30, 2), (100, 10), (57, 7)])
def test_unrank_enumerates_every_valid_extent_once(orc, T, L):
    valid = {(a, b) for a in range(T) for b in range(T) if b - a + 1 >= L}
    P = orc.npairs(T, L)
    assert P == len(valid)
    got = [orc.unrank(k, L) for k in range(P)]
    assert set(got) == valid and len(got) == len(valid)
    # ordered by end column, then start column
    assert got == sorted(got, key=lambda ab: (ab[1], ab[0]))


def test_unrank_large_k_brackets(orc):
    L = 10
    for k in [2 ** 31 - 1, 2 ** 32 + 12345, 4_194_303, 8_386_560 - 1]:
        t0, t2 = orc.unrank(k, L)
        e = t2 - L + 1
        assert e * (e + 1) // 2 <= k < (e + 1) * (e + 2) // 2
        assert t0 == k - e * (e + 1) // 2


def test_draw_is_uniform_on_its_ranges(orc):
    from scipy.stats import chisquare
    T, F, L, D = 14, 3, 10, 3  # 15 extents, 768 frequency codes, 7 delays
    n = 60000
    tr = orc.draw_many(7, 0, 0, n, T, F, L, D)
    N = tr["t2"] - tr["t0"] + 1
    assert (N >= L).all() and (tr["t0"] >= 0).all() and (tr["t2"] < T).all()
    for f in ("f0", "f1", "f2"):
        assert (tr[f] < F * 256).all()
    assert (np.abs(tr["dtau"]) <= D).all()
    pair_id = tr["t0"] * T + tr["t2"]
    _, counts = np.unique(pair_id, return_counts=True)
    assert counts.size == orc.npairs(T, L)
    assert chisquare(counts).pvalue > 1e-4
    for f in ("f0", "f1", "f2"):
        assert chisquare(np.bincount(tr[f] // 32, minlength=24)).pvalue > 1e-4
    assert chisquare(np.bincount(tr["dtau"] + D, minlength=2 * D + 1)).pvalue > 1e-4
    # the six numbers come from different words: no correlation between them
    cols = np.stack([tr["t0"], tr["f0"], tr["f1"], tr["f2"], tr["dtau"]]).astype(np.float64)
    cc = np.corrcoef(cols)
    assert np.abs(cc[np.triu_indices(5, 1)]).max() < 0.03


def test_draw_depends_on_seed_stream_and_index(orc):
    a = orc.draw(1, 0, 5, 100, 128, 10, 1000)
    assert a.tolist() != orc.draw(2, 0, 5, 100, 128, 10, 1000).tolist()
    assert a.tolist() != orc.draw(1, 1, 5, 100, 128, 10, 1000).tolist()
    assert a.tolist() != orc.draw(1, 0, 6, 100, 128, 10, 1000).tolist()
    assert a.tolist() == orc.draw(1, 0, 5, 100, 128, 10, 1000).tolist()


# --------------------------------------------------------------------------- rasteriser (Eq. 6)

def _bezier_rows_exact(t0, t2, f0, f1, f2):
    """Eq. 6 in exact rationals with t_mid at the midpoint; one sample per column."""
    P0 = (Fraction(t0), Fraction(f0, 256))
    P1 = (Fraction(t0 + t2, 2), Fraction(f1, 256))
    P2 = (Fraction(t2), Fraction(f2, 256))
    D = t2 - t0
    rows = []
    for k in range(D + 1):
        xi = Fraction(k, D)
        w0, w1, w2 = (1 - xi) ** 2, 2 * (1 - xi) * xi, xi ** 2
        t = w0 * P0[0] + w1 * P1[0] + w2 * P2[0]
        f = w0 * P0[1] + w1 * P1[1] + w2 * P2[1]
        assert t == t0 + k  # the k-th sample lands on column t0+k
        rows.append(math.floor(f))
    return rows


def _trk(t0, t2, f0, f1, f2, dtau=0):
    import oracle
    return np.array((t0, t2, f0, f1, f2, dtau), dtype=oracle.TRACK_DTYPE)


def test_rows_match_exact_rationals_exhaustive_small(orc):
    F = 3
    grid = [0, 1, 127, 255, 256, 257, 383, 511, 512, 700, 767]
    for D in range(1, 9):
        for f0 in grid:
            for f1 in grid:
                for f2 in grid[::2]:
                    want = _bezier_rows_exact(5, 5 + D, f0, f1, f2)
                    got = orc.rows(_trk(5, 5 + D, f0, f1, f2), F).tolist()
                    assert got == want, (D, f0, f1, f2)


def test_rows_match_exact_rationals_random_large(orc):
    sel = np.random.default_rng(6)
    for _ in range(12):
        F = int(sel.integers(1, 32768))
        D = int(sel.integers(1, 2896))
        f = sel.integers(0, F * 256, size=3)
        want = _bezier_rows_exact(0, D, *map(int, f))
        got = orc.rows(_trk(0, D, *map(int, f)), F).tolist()
        assert got == want
        assert min(got) >= 0 and max(got) < F


def test_rows_special_cases(orc):
    F = 50
    # constant frequency -> constant row
    assert set(orc.rows(_trk(0, 40, 1234, 1234, 1234), F).tolist()) == {1234 // 256}
    # middle point on the chord -> floor of the straight line
    r = orc.rows(_trk(0, 30, 256 * 3, (256 * 3 + 256 * 40) // 2, 256 * 40), F)
    line = [math.floor(Fraction(256 * 3) / 256 + Fraction(k, 30) * Fraction(256 * 37, 256)) for k in range(31)]
    assert r.tolist() == line
    # reversing time and the control points reverses the rows
    a = orc.rows(_trk(3, 61, 5000, 100, 9000), F)
    b = orc.rows(_trk(3, 61, 9000, 100, 5000), F)
    assert a.tolist() == b[::-1].tolist()


# --------------------------------------------------------------------------- phase and statistic

def _flat_map(T, F, sigma=1.0):
    Y = np.zeros((T, F), dtype=np.complex64)
    s = np.full((T, F), sigma, dtype=np.float32)
    return Y, s


def _inject_track(Y, s, cols, rows, amp, fq4_lo, dfq4, dtau0):
    """p += amp * exp(-2 pi i f dtau0) at the pixels (matched to a template of delay dtau0)."""
    fq4 = fq4_lo + rows.astype(np.int64) * dfq4
    turns = -(fq4 * dtau0).astype(np.float64) / 2.0 ** 32  # f dtau0 in turns, exact product
    synth.add_pixels(Y, s, cols, rows, amp, turns)


def test_score_matches_eq8_in_50_digit_arithmetic(orc):
    import mpmath
    mpmath.mp.dps = 50
    Y, s = synth.noise_map(40, 64, seed=11, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s, fq4_lo=1600, dfq4=16)
    for j in range(20):
        tr = orc.draw(3, 0, j, 40, 64, 10, orc.dtau_units(0.01))
        rows = _bezier_rows_exact(int(tr["t0"]), int(tr["t2"]), int(tr["f0"]), int(tr["f1"]), int(tr["f2"]))
        acc = mpmath.mpf(0)
        for k, r in enumerate(rows):
            t = int(tr["t0"]) + k
            f = Fraction(1600 + 16 * r, 16)  # Hz
            ft = f * int(tr["dtau"]) * UNIT   # turns, exact (not reduced)
            ang = 2 * mpmath.pi * mpmath.mpf(ft.numerator) / ft.denominator
            pre = mpmath.mpf(float(Y[t, r].real)) / mpmath.mpf(float(s[t, r]))
            pim = mpmath.mpf(float(Y[t, r].imag)) / mpmath.mpf(float(s[t, r]))
            acc += mpmath.cos(ang) * pre - mpmath.sin(ang) * pim
        want = float(acc / mpmath.sqrt(len(rows)))
        assert orc.score(m, tr) == pytest.approx(want, abs=1e-12)
        want_n = float(acc / len(rows))
        assert orc.score(m, tr, norm=orc.NORM_N) == pytest.approx(want_n, abs=1e-12)


def test_zero_delay_reduces_to_eq5_real_sum(orc):
    Y, s = synth.noise_map(60, 32, seed=4, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    p = Y.astype(np.complex128) / s.astype(np.float64)
    for j in range(30):
        tr = orc.draw(9, 0, j, 60, 32, 10, 0)
        assert int(tr["dtau"]) == 0
        r = orc.rows(tr, 32)
        cols = np.arange(int(tr["t0"]), int(tr["t2"]) + 1)
        rho = p[cols, r].real
        assert orc.score(m, tr, norm=orc.NORM_N) == pytest.approx(rho.mean(), abs=1e-13)
        assert orc.score(m, tr) == pytest.approx(rho.sum() / math.sqrt(rho.size), abs=1e-13)


def test_mismatch_ratio_eq3_constant_row(orc):
    """Eq. 3: a delay error dtau - dtau0 keeps cos(2 pi f (dtau - dtau0)) of the SNR."""
    T, F = 50, 200
    r0 = 37
    f_hz = 100 + r0
    Y, s = _flat_map(T, F, sigma=0.7)
    dtau0 = 123457
    tr0 = _trk(2, 45, r0 * 256 + 100, r0 * 256 + 7, r0 * 256 + 255, dtau0)
    cols = np.arange(2, 46)
    rows = np.full(cols.size, r0)
    _inject_track(Y, s, cols, rows, 0.25, 1600, 16, dtau0)
    m = orc.Map(Y, s)
    z0 = orc.score(m, tr0)
    assert z0 == pytest.approx(0.25 * math.sqrt(cols.size), rel=1e-6)
    for dd in [-900000, -33333, -1, 1, 5000, 77777, 2684355]:
        tr = tr0.copy()
        tr["dtau"] = dtau0 + dd
        want = math.cos(2 * math.pi * f_hz * dd * 2.0 ** -28)
        assert orc.score(m, tr) / z0 == pytest.approx(want, abs=2e-6)


def test_mismatch_ratio_eq3_curved_track(orc):
    T, F = 80, 300
    tr0 = _trk(5, 70, 20 * 256, 250 * 256, 90 * 256 + 17, 555555)
    rows = orc.rows(tr0, F)
    cols = np.arange(5, 71)
    Y, s = _flat_map(T, F)
    _inject_track(Y, s, cols, rows, 1.0, 1600, 16, 555555)
    m = orc.Map(Y, s)
    z0 = orc.score(m, tr0)
    f = 100.0 + rows
    for dd in [-400000, 12345, 1000000]:
        tr = tr0.copy()
        tr["dtau"] = 555555 + dd
        want = np.mean(np.cos(2 * math.pi * f * dd * 2.0 ** -28))
        assert orc.score(m, tr) / z0 == pytest.approx(want, abs=2e-6)


@pytest.mark.parametrize("f_hz,R,printed_us", _golden("paper_eq4_tolerance.txt"))
def test_eq4_tolerance_reproduces_printed_values(orc, f_hz, R, printed_us):
    """Solve ratio(dtau) = R on the oracle's statistic; it must round to the paper's value."""
    row = int(f_hz) - 100
    F = row + 1
    Y, s = _flat_map(20, F)
    cols = np.arange(0, 20)
    _inject_track(Y, s, cols, np.full(20, row), 1.0, 1600, 16, 0)
    m = orc.Map(Y, s)
    tr = _trk(0, 19, row * 256, row * 256, row * 256, 0)
    z0 = orc.score(m, tr)

    def ratio(d):
        t = tr.copy()
        t["dtau"] = d
        return orc.score(m, t) / z0

    lo, hi = 0, int(0.25 / f_hz / 2.0 ** -28)  # ratio goes 1 -> 0 on [0, quarter period]
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ratio(mid) > R:
            lo = mid
        else:
            hi = mid
    dtau_us = hi * 2.0 ** -28 * 1e6
    # exact to the delay grid: within one 2^-28 s unit of arccos(R) / (2 pi f)
    assert dtau_us == pytest.approx(math.acos(R) / (2 * math.pi * f_hz) * 1e6, abs=2.0 ** -28 * 1e6)
    digits = 2 - int(math.floor(math.log10(printed_us))) - 1
    assert round(dtau_us, digits) == pytest.approx(printed_us)
    # past a half period the signal comes back negative (delta = pi -> ratio -1)
    assert ratio(int(round(0.5 / f_hz / 2.0 ** -28))) == pytest.approx(-1.0, abs=1e-5)


@pytest.mark.parametrize("dtau_max_s,stripe_hz", _golden("paper_stripes.txt"))
def test_stripes_have_quarter_period_bandwidth(orc, dtau_max_s, stripe_hz):
    """A real-positive map seen through delay dtau: sign alternates every 1/(2 dtau) Hz,
    with a peak-to-null width of 1/(4 dtau) (25 Hz at 10 ms)."""
    F = 160
    T = 12
    Y = np.ones((T, F), dtype=np.complex64)
    s = np.ones((T, F), dtype=np.float32)
    m = orc.Map(Y, s)
    D = orc.dtau_units(dtau_max_s)
    z = np.array([orc.score(m, _trk(0, T - 1, r * 256, r * 256, r * 256, D)) for r in range(F)])
    f = 100 + np.arange(F)
    assert z[0] == pytest.approx(math.sqrt(T), rel=1e-5)  # 100 Hz * 10 ms = 1 turn: peak
    nulls = f[np.abs(z) < 1e-4]
    assert nulls[0] - 100 == pytest.approx(stripe_hz)
    assert np.allclose(np.diff(nulls), 2 * stripe_hz)
    sign = np.sign(z[np.abs(z) > 1e-3])
    assert (np.diff(sign) != 0).sum() == len(nulls)


def test_matched_injection_scores_exactly_its_amplitude(orc):
    T, F = 120, 90
    D = orc.dtau_units(0.01)
    Yn, s = synth.noise_map(T, F, seed=21, sigma=("loguniform", 0.5, 2.0))
    for j in range(5):
        tr = orc.draw(21, 3, j, T, F, 10, D)
        rows = orc.rows(tr, F)
        cols = np.arange(int(tr["t0"]), int(tr["t2"]) + 1)
        amp = 8.0 / math.sqrt(cols.size)
        Ys = np.zeros_like(Yn)
        _inject_track(Ys, s, cols, rows, amp, 1600, 16, int(tr["dtau"]))
        assert orc.score(orc.Map(Ys, s), tr) == pytest.approx(8.0, abs=2e-5)
        Yb = Yn.copy()
        _inject_track(Yb, s, cols, rows, amp, 1600, 16, int(tr["dtau"]))
        dz = orc.score(orc.Map(Yb, s), tr) - orc.score(orc.Map(Yn, s), tr)
        assert dz == pytest.approx(8.0, abs=5e-5)


def test_scorer_symmetries(orc):
    T, F = 70, 40
    D = orc.dtau_units(0.01)
    Y1, s = synth.noise_map(T, F, seed=31, sigma=("loguniform", 0.5, 2.0))
    Y2, _ = synth.noise_map(T, F, seed=32)
    m1, m2 = orc.Map(Y1, s), orc.Map(Y2, s)
    m12 = orc.Map(Y1.astype(np.complex128) + Y2, s)
    mc = orc.Map(np.conj(Y1), s)
    msc = orc.Map(Y1.astype(np.complex128) * 3.5, s.astype(np.float64) * 3.5)
    Yr, sr = Y1[::-1].copy(), s[::-1].copy()
    mr = orc.Map(Yr, sr)
    for j in range(40):
        tr = orc.draw(5, 0, j, T, F, 10, D)
        z1 = orc.score(m1, tr)
        # linear in Y
        assert orc.score(m12, tr) == pytest.approx(z1 + orc.score(m2, tr), abs=1e-9)
        # (Y, sigma) -> (cY, c sigma) leaves p unchanged
        assert orc.score(msc, tr) == pytest.approx(z1, abs=1e-12)
        # conjugate map seen with the opposite delay
        tc = tr.copy()
        tc["dtau"] = -tr["dtau"]
        assert orc.score(mc, tc) == pytest.approx(z1, abs=1e-12)
        # time reversal: same pixels, reversed order
        trr = _trk(T - 1 - int(tr["t2"]), T - 1 - int(tr["t0"]), int(tr["f2"]), int(tr["f1"]),
                   int(tr["f0"]), int(tr["dtau"]))
        assert orc.score(mr, trr) == pytest.approx(z1, abs=1e-12)


def test_null_distribution_is_standard_normal(orc):
    """Noise only: for a data-independent template the statistic is exactly N(0,1) (1/sqrt N)."""
    from scipy.stats import kstest
    T, F, M = 30, 16, 4096
    tr = _trk(3, 27, 2 * 256 + 9, 15 * 256, 7 * 256 + 200, 1500000)
    zs, zn = [], []
    for k in range(M):
        Y, s = synth.noise_map(T, F, seed=777, sigma=("loguniform", 0.5, 2.0), stream=k)
        m = orc.Map(Y, s)
        zs.append(orc.score(m, tr))
        zn.append(orc.score(m, tr, norm=orc.NORM_N))
    zs, zn = np.array(zs), np.array(zn)
    assert kstest(zs, "norm").pvalue > 1e-3
    assert abs(zs.mean()) < 4 / math.sqrt(M)
    assert abs(zs.var() - 1) < 5 * math.sqrt(2 / M)
    assert np.allclose(zn * math.sqrt(25), zs, atol=1e-12)


def test_brute_force_linear_algebra_route(orc):
    """Tiny map, every template of a grid: oracle scores vs a dense pixel-membership
    matrix built from exact rationals and multiplied into the phase-rotated map."""
    T, F, L = 12, 4, 10
    D = 2684355
    Y, s = synth.noise_map(T, F, seed=41, sigma=("loguniform", 0.5, 2.0))
    p = (Y.astype(np.complex128) / s.astype(np.float64)).reshape(-1)
    fgrid = [0, 200, 300, 511, 700, 1023]
    tracks = []
    for e in range(T - L + 1):
        for a in range(e + 1):
            for f0 in fgrid:
                for f1 in fgrid:
                    for f2 in fgrid:
                        for dt in (-D, -D // 3, 0, D // 2):
                            tracks.append((a, e + L - 1, f0, f1, f2, dt))
    import oracle
    tr = np.array(tracks, dtype=oracle.TRACK_DTYPE)
    z = orc.score_list(orc.Map(Y, s), tr)
    # membership matrix and per-template phase from exact rationals
    cache = {}
    want = np.empty(len(tracks))
    for i, (t0, t2, f0, f1, f2, dt) in enumerate(tracks):
        key = (t0, t2, f0, f1, f2)
        if key not in cache:
            cache[key] = _bezier_rows_exact(t0, t2, f0, f1, f2)
        rr = cache[key]
        idx = np.array([(t0 + k) * F + r for k, r in enumerate(rr)])
        f = Fraction(1) * (100 + np.array(rr))
        ph = np.array([float((Fraction(int(fk)) * dt * UNIT) % 1) for fk in f])
        want[i] = (np.exp(2j * np.pi * ph) * p[idx]).real.sum() / math.sqrt(len(rr))
    assert np.allclose(z, want, atol=1e-12, rtol=0)
    assert orc.argmax(z) == int(np.argmax(want))


def test_argmax_rules(orc):
    nan = float("nan")
    assert orc.argmax(np.array([1.0, 3.0, nan, 3.0, 2.0])) == 1
    assert orc.argmax(np.array([nan, nan])) == -1
    assert orc.argmax(np.array([-0.0, 0.0])) == 0
    assert orc.argmax(np.array([nan, -np.inf, -5.0])) == 2
    z = np.random.default_rng(1).standard_normal(1000)
    assert orc.argmax(z) == int(np.argmax(z))
