"""Pins of the oracle's extensions (top-K, FP16 storage, smooth SNR and its
gradient, refinement) against library routines, closed forms and invariants."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth

D10MS = 2684355


def _trk(orc, t0, t2, f0, f1, f2, dtau=0):
    return np.array((t0, t2, f0, f1, f2, dtau), dtype=orc.TRACK_DTYPE)


# --------------------------------------------------------------------------- top-K

def test_topk_matches_a_library_sort(orc):
    sel = np.random.default_rng(5)
    z = sel.standard_normal(50_000).round(2)  # many exact ties
    z[sel.choice(z.size, 300, replace=False)] = np.nan
    for K in (0, 1, 7, 1024, 50_000):
        got = orc.topk(z, K)
        key = np.where(np.isnan(z), -np.inf, z)
        want = np.lexsort((np.arange(z.size), -key))[:K]  # score descending, then index ascending
        assert np.array_equal(got, want)


# --------------------------------------------------------------------------- FP16 storage

def test_fp16_storage_within_half_ulp(orc):
    """Magnitude within half a binary16 ulp (relative 2^-11) or the subnormal step, argument within
    half of 2^-16 turn, of the FP64 p; the exponent puts the largest magnitude in (2^14, 2^15]."""
    Y, s = synth.noise_map(60, 50, seed=3, sigma=("loguniform", 0.5, 2.0))
    Y[10, 7] = np.complex64(1000.0 * s[10, 7])  # a loud pixel sets the exponent
    q, e, deq = orc.quantize_p16(Y, s)
    p = Y.astype(np.complex128) / s.astype(np.float64)
    assert 2.0 ** 14 < np.abs(deq).max() / 2.0 ** e <= 2.0 ** 15
    mag16 = q[..., 1].view(np.float16).astype(np.float64) * 2.0 ** e
    # the FP32 division that forms p adds at most 2^-24 relative
    lim = np.maximum(np.abs(p) * 2.0 ** -11, 2.0 ** (e - 25)) + np.abs(p) * 2.0 ** -23
    assert (np.abs(mag16 - np.abs(p)) <= lim).all()
    d_turn = (q[..., 0].astype(np.float64) / 65536.0 - np.angle(p) / (2 * np.pi) + 0.5) % 1.0 - 0.5
    assert (np.abs(d_turn) <= 2.0 ** -17 + 2.0 ** -22).all()
    assert np.allclose(deq, mag16 * np.exp(2j * np.pi * q[..., 0] / 65536.0), rtol=0, atol=1e-12 * 2.0 ** e)


def test_fp16_storage_exact_cases(orc):
    """Worked values: magnitudes that binary16 holds exactly are kept; the four axis directions and
    the diagonals take exact arguments (0, 1/8, 1/4, 1/2, 3/4 turn); ties of the magnitude go to
    even; the exponent is ceil(log2 max|p|) - 15 (a power-of-two maximum is its own ceiling)."""
    one = np.ones((1, 9), dtype=np.float32)
    Y = np.array([[4.0, 4j, -4.0, -4j, 3 + 3j, 2.0, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 0.0]],
                 dtype=np.complex64)
    q, e, deq = orc.quantize_p16(Y, one)
    assert e == 3 - 15  # max |p| = 3 sqrt(2) = 4.24: ceil(log2) = 3
    mag = q[0, :, 1].view(np.float16).astype(np.float64) * 2.0 ** e
    assert list(q[0, :5, 0]) == [0, 16384, 32768, 49152, 8192]
    assert mag[0] == mag[1] == mag[2] == mag[3] == 4.0 and mag[5] == 2.0
    # 3 sqrt(2) * 2^12 = 17378.9: binary16 steps by 16 there, to 17376
    assert mag[4] * 2.0 ** -e == 17376.0
    # 1 + 2^-11 scaled by 2^12 is 4098, halfway between the neighbours 4096 (even) and 4100: 4096;
    # 1 + 3 2^-11 is 4102, halfway between 4100 and 4104 (even): 4104
    assert mag[6] == 1.0 and mag[7] * 2.0 ** -e == 4104.0
    assert q[0, 8, 0] == 0 and mag[8] == 0.0 and deq[0, 8] == 0
    # an exact power of two as the maximum is its own ceiling: max |p| = 8 gives e = 3 - 15
    _, e8, _ = orc.quantize_p16(np.array([[8.0, 1.0]], np.complex64), np.ones((1, 2), np.float32))
    assert e8 == 3 - 15
    # a map of zeros: exponent 0, everything zero
    q0, e0, d0 = orc.quantize_p16(np.zeros((2, 3), np.complex64), np.ones((2, 3), np.float32))
    assert e0 == 0 and not q0.any() and not d0.any()


# --------------------------------------------------------------------------- smooth SNR

def test_smooth_equals_plain_score_on_pixel_centres(orc):
    """A template whose samples sit on column integers and row centres: z~ = the plain Eq. 8 score."""
    T, F = 80, 60
    Y, s = synth.noise_map(T, F, seed=8, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    for (t0, t2, r, dtau) in [(5, 70, 17, 1234567), (0, 79, 0, -D10MS), (30, 39, 59, 0), (3, 50, 33, 7)]:
        K = t2 - t0 + 1
        th = [t0, t2, r + 0.5, r + 0.5, r + 0.5, dtau * 2.0 ** -28 * 1e3]
        zs, _ = orc.smooth(m, th, K)
        zp = orc.score(m, _trk(orc, t0, t2, r * 256 + 128, r * 256 + 128, r * 256 + 128, dtau))
        assert zs == pytest.approx(zp, abs=1e-10)
    # straight line with an integer slope of rows per column: samples on centres too
    t0, t2, r0, slope = 10, 40, 5, 1
    th = [t0, t2, r0 + 0.5, r0 + 0.5 + slope * (t2 - t0) / 2, r0 + 0.5 + slope * (t2 - t0), 0.25]
    zs, _ = orc.smooth(m, th, t2 - t0 + 1)
    rows = r0 + slope * np.arange(t2 - t0 + 1)
    p = Y.astype(np.complex128) / s
    f = 100.0 + rows
    want = (np.exp(2j * np.pi * f * 0.25e-3) * p[np.arange(t0, t2 + 1), rows]).real.sum() / math.sqrt(rows.size)
    assert zs == pytest.approx(want, abs=1e-10)


def _clear_of_grid(theta, K, T, F, margin):
    xi = np.arange(K) / (K - 1)
    t = theta[0] + xi * (theta[1] - theta[0])
    f = (1 - xi) ** 2 * theta[2] + 2 * xi * (1 - xi) * theta[3] + xi ** 2 * theta[4] - 0.5
    inside = (t > margin).all() and (t < T - 1 - margin).all() and (f > margin).all() and (f < F - 1 - margin).all()
    dist = min(np.abs(t - np.round(t)).min(), np.abs(f - np.round(f)).min())
    return inside and dist > margin


def test_smooth_gradient_matches_central_differences(orc):
    """Away from grid lines z~ is linear in each position coordinate, so a central
    difference with h = 1e-3 is exact to rounding; the delay direction is smooth (O(h^2))."""
    T, F = 120, 90
    Y, s = synth.noise_map(T, F, seed=9, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    sel = np.random.default_rng(10)
    h = 1e-3
    done = 0
    while done < 25:
        K = int(sel.integers(10, 60))
        a = sel.uniform(2, T - 40)
        th = np.array([a, a + sel.uniform(K, 35 + K), *sel.uniform(3, F - 3, 3), sel.uniform(-10, 10)])
        if th[1] > T - 3 or not _clear_of_grid(th, K, T, F, 4 * h):
            continue
        z, g = orc.smooth(m, th, K)
        for q in range(6):
            e = np.zeros(6)
            e[q] = h
            fd = (orc.smooth(m, th + e, K, grad=False)[0] - orc.smooth(m, th - e, K, grad=False)[0]) / (2 * h)
            tol = 1e-8 if q < 5 else 1e-4 * max(1.0, abs(g[q]))
            assert fd == pytest.approx(g[q], abs=tol), (q, th, K)
        done += 1


def test_delay_derivative_follows_eq3(orc):
    """Matched injection on a constant-row track: z~(dtau) = a sqrt(K) cos(2 pi f (dtau - dtau0)),
    so dz~/d(dtau) = -a sqrt(K) 2 pi f sin(2 pi f (dtau - dtau0)) (Eq. 3 differentiated)."""
    T, F, r = 60, 40, 23
    f_hz = 100 + r
    Y = np.zeros((T, F), dtype=np.complex64)
    s = np.full((T, F), 1.3, dtype=np.float32)
    dt0_ms = 2.5
    cols = np.arange(4, 54)
    synth.add_pixels(Y, s, cols, np.full(cols.size, r), 0.5, -f_hz * dt0_ms * 1e-3)
    m = orc.Map(Y, s)
    K = cols.size
    for d_ms in (-3.0, 0.1, 1.7, 2.5, 6.0):
        z, g = orc.smooth(m, [4, 53, r + 0.5, r + 0.5, r + 0.5, d_ms], K)
        ang = 2 * math.pi * f_hz * (d_ms - dt0_ms) * 1e-3
        assert z == pytest.approx(0.5 * math.sqrt(K) * math.cos(ang), abs=1e-6)
        want = -0.5 * math.sqrt(K) * 2 * math.pi * f_hz * math.sin(ang) * 1e-3
        assert g[5] == pytest.approx(want, abs=1e-6)
        assert np.allclose(g[2:5] * 0, 0)


def test_clamped_coordinates_have_zero_gradient(orc):
    T, F = 40, 30
    Y, s = synth.noise_map(T, F, seed=2)
    m = orc.Map(Y, s)
    # the whole template before the map in time and above it in frequency
    z, g = orc.smooth(m, [-20.3, -5.1, 40.2, 45.0, 50.5, 0.3], 12)
    assert g[0] == 0 and g[1] == 0 and g[2] == 0 and g[3] == 0 and g[4] == 0


# --------------------------------------------------------------------------- refinement

def test_refine_keeps_best_and_respects_constraints(orc):
    T, F, L = 200, 120, 10
    Y, s = synth.noise_map(T, F, seed=11, sigma=("loguniform", 0.5, 2.0))
    m = orc.Map(Y, s)
    sel = np.random.default_rng(12)
    for _ in range(10):
        K = int(sel.integers(10, 80))
        th0 = np.array([sel.uniform(0, 100), 0, *sel.uniform(0, F, 3), sel.uniform(-10, 10)])
        th0[1] = th0[0] + K + sel.uniform(0, 20)
        z0, _ = orc.smooth(m, th0, K)
        th, z = orc.refine(m, th0, K, 50, L, 10.0)
        assert z >= z0 - 1e-12
        assert z == pytest.approx(orc.smooth(m, th, K)[0], abs=1e-12)
        assert 0 <= th[0] and th[1] <= T - 1 and th[1] - th[0] >= L - 1 - 1e-9
        assert (th[2:5] >= 0).all() and (th[2:5] < F).all() and abs(th[5]) <= 10.0


def test_refine_climbs_to_a_nearby_injection(orc):
    """Noise-free map with one injected straight track; a start 1-1.5 px and 1 ms away climbs
    to within a pixel and 0.1 ms of the generating line and 95% of its smooth SNR."""
    T, F = 100, 80
    Y = np.zeros((T, F), dtype=np.complex64)
    s = np.ones((T, F), dtype=np.float32)
    t0, t2, r0, r2, dt0 = 20, 79, 30.5, 50.5, 2.0
    k = np.arange(t2 - t0 + 1)
    rows = np.floor(r0 + (r2 - r0) * k / (t2 - t0)).astype(int)
    synth.add_pixels(Y, s, t0 + k, rows, 1.0, -(100.0 + rows) * dt0 * 1e-3)
    m = orc.Map(Y, s)
    K = t2 - t0 + 1
    th0 = [t0 + 1.5, t2 - 1.0, r0 + 1.5, 0.5 * (r0 + r2) - 1.0, r2 + 1.2, dt0 + 1.0]
    z0, _ = orc.smooth(m, th0, K)
    z_true, _ = orc.smooth(m, [t0, t2, r0, 0.5 * (r0 + r2), r2, dt0], K)  # the generating line
    th, z = orc.refine(m, th0, K, 50, 10, 10.0)
    assert z > z0 + 2.0 and z > 0.95 * z_true
    assert abs(th[5] - dt0) < 0.1
    assert np.abs(th[2:5] - [r0, 0.5 * (r0 + r2), r2]).max() < 1.0


def test_theta_to_track_rounding(orc):
    tr = orc.theta_to_track([3.5, 12.49, 1.999, 0.0, 7.99999, 1.0], T=20, F=8, L=10, dtau_max=D10MS)
    assert (int(tr["t0"]), int(tr["t2"])) == (4, 13)  # half up, then widened to L = 10 pixels
    assert (int(tr["f0"]), int(tr["f1"]), int(tr["f2"])) == (511, 0, 2047)
    assert int(tr["dtau"]) == round(1e-3 * 2 ** 28)
    tr = orc.theta_to_track([15.2, 19.0, -1, 9, 3, 50.0], T=20, F=8, L=10, dtau_max=D10MS)
    assert (int(tr["t0"]), int(tr["t2"])) == (10, 19) and int(tr["dtau"]) == D10MS
    assert int(tr["f0"]) == 0 and int(tr["f1"]) == 8 * 256 - 1
