"""Pins of the map-formation oracle (cross-power ft-map from two strain streams), each checked
against something other than the oracle's own formula:

* the column spectra against a direct DFT summed term by term (no FFT);
* an integer-bin tone through the periodic Hann window: the closed form A M dt / 4 at its bin,
  -A M dt / 8 at the two neighbours, zero elsewhere, with the column's phase advancing by half a
  cycle per bin index per column (hop M / 2);
* a tone reaching J tau seconds after I: Y at its bin is real-positive after Eq. 8's phase factor
  e^{2 pi i f tau}, with the closed-form magnitude (pins the conjugate on I and the sign);
* white noise of variance s^2: mean column power 2 s^2 dt (the one-sided PSD), which fixes the
  DFT normalisation and the window's 3/8;
* the neighbour mean on profiles with hand-worked means, including the edges;
* slides: swapping the detectors conjugates the map and reverses the slide; one detector with
  itself at slide 0 gives a real map equal to its column power;
* in noise, Y / sigma has unit-variance real and imaginary parts when P' averages many columns;
* end to end with the scorer's oracle: a delayed tone burst scores high at zero lag with Eq. 8's
  delay and vanishes under slides longer than the burst.
"""
from __future__ import annotations

import cmath
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def mf():
    from oracle import mapform
    return mapform


def test_spectra_against_direct_dft(mf):
    M, fs, T = 16, 8.0, 5
    x = synth.white_strain((T + 1) * M // 2, seed=11)
    got = mf.column_spectra(x, fs, M, T, 0, M // 2)
    for t in range(T):
        for k in range(M // 2):
            acc = 0j
            for n in range(M):
                w = math.sin(math.pi * n / M) ** 2
                acc += w * float(x[t * M // 2 + n]) * cmath.exp(-2j * math.pi * k * n / M)
            assert abs(got[t, k] - acc / fs) < 1e-12


def test_integer_bin_tone_closed_form(mf):
    M, fs, k0, A, ph, T = 64, 64.0, 5, 1.5, 0.1, 7
    x = np.zeros((T + 1) * M // 2, dtype=np.float32)
    synth.add_tone(x, fs, k0 * fs / M, A, phase_turns=ph)
    # the FP32 samples carry a rounding error of ~1e-7 A
    spec = mf.column_spectra(x, fs, M, T, 0, M // 2)
    dt = 1.0 / fs
    for t in range(T):
        e = cmath.exp(2j * math.pi * (ph + k0 * t / 2))  # phase of the tone at sample t M / 2
        assert abs(spec[t, k0] - A * M * dt / 4 * e) < 1e-6
        assert abs(spec[t, k0 - 1] + A * M * dt / 8 * e) < 1e-6
        assert abs(spec[t, k0 + 1] + A * M * dt / 8 * e) < 1e-6
        others = np.delete(spec[t], [k0 - 1, k0, k0 + 1])
        assert np.abs(others).max() < 1e-6


def test_delayed_tone_phase_and_magnitude(mf):
    M, fs, k0, A, T = 128, 1024.0, 20, 0.8, 9
    f0 = k0 * fs / M
    tau = 3.7e-4
    xi = np.zeros((T + 1) * M // 2, dtype=np.float32)
    xj = np.zeros_like(xi)
    synth.add_tone(xi, fs, f0, A, phase_turns=0.3)
    synth.add_tone(xj, fs, f0, A, phase_turns=0.3, delay_s=tau)
    si = mf.column_spectra(xi, fs, M, T, 0, M // 2)
    sj = mf.column_spectra(xj, fs, M, T, 0, M // 2)
    Y, _ = mf.form_map(si, np.ones(si.shape), sj, np.ones(sj.shape), fs, M, 0)
    nrm = M / fs * 3 / 8
    want = 2 / nrm * (A * M / fs / 4) ** 2
    for t in range(T):
        z = cmath.exp(2j * math.pi * f0 * tau) * Y[t, k0]
        assert abs(z.imag) < 1e-5 * want and abs(z.real - want) < 1e-5 * want


def test_white_noise_power_is_the_one_sided_psd(mf):
    M, fs, s, T = 128, 512.0, 2.0, 400
    x = synth.white_strain((T + 1) * M // 2, seed=12, std=s)
    pw = mf.column_power(mf.column_spectra(x, fs, M, T, 2, 60), fs, M)
    want = 2 * s * s / fs
    # 24000 exponential variates, pairwise correlated through the overlap: well within 3 %
    assert abs(pw.mean() / want - 1) < 0.03


def test_neighbour_mean_hand_worked(mf):
    T, nb = 20, 3
    pw = np.arange(T, dtype=np.float64)[:, None] * np.ones((1, 2))
    got = mf.neighbour_mean(pw, nb)[:, 0]
    want = {0: 3.0, 1: 4.0, 2: 15 / 4, 3: 19 / 5, 16: 76 / 5, 17: 61 / 4, 18: 15.0, 19: 16.0}
    for t in range(T):
        assert got[t] == pytest.approx(want.get(t, float(t)), abs=1e-12), t
    c = np.full((T, 3), 2.5)
    assert np.array_equal(mf.neighbour_mean(c, nb), c)
    with pytest.raises(ValueError):
        mf.neighbour_mean(np.ones((2, 1)), 4)  # no column two away


def test_slide_symmetries(mf):
    M, fs, T, nb = 64, 256.0, 24, 3
    xi = synth.white_strain((T + 1) * M // 2, seed=13)
    xj = synth.white_strain((T + 1) * M // 2, seed=13, stream=1)
    si, sj = mf.column_spectra(xi, fs, M, T, 3, 20), mf.column_spectra(xj, fs, M, T, 3, 20)
    pi, pj = mf.psd(si, fs, M, nb), mf.psd(sj, fs, M, nb)
    for s in (0, 1, 5, 23):
        Y, sg = mf.form_map(si, pi, sj, pj, fs, M, s)
        Yr, sgr = mf.form_map(sj, pj, si, pi, fs, M, -s)
        roll = (np.arange(T) + s) % T
        assert np.allclose(Y, np.conj(Yr[roll]), rtol=1e-14, atol=0)
        assert np.allclose(sg, sgr[roll], rtol=1e-14, atol=0)
        Y2, _ = mf.form_map(si, pi, sj, pj, fs, M, s + T)
        assert np.array_equal(Y, Y2)
    Y0, s0 = mf.form_map(si, pi, si, pi, fs, M, 0)
    assert np.all(np.abs(Y0.imag) <= 1e-14 * Y0.real)  # zero up to the product's rounding
    assert np.allclose(Y0.real, mf.column_power(si, fs, M), rtol=1e-14, atol=0)
    assert np.allclose(s0, pi / math.sqrt(2), rtol=1e-14, atol=0)


def test_unit_variance_in_noise(mf):
    M, fs, T, nb = 128, 512.0, 600, 60
    n = (T + 1) * M // 2
    maps = mf.form_maps(synth.white_strain(n, seed=14), synth.white_strain(n, seed=14, stream=1, std=3.0),
                        fs, M, T, 4, 50, nb, [0])
    p = maps[0][0] / maps[0][1]
    # P' from ~120 columns per detector inflates the variance by only ~2 %
    for part in (p.real, p.imag):
        assert 0.95 < part.var() < 1.10
        assert abs(part.mean()) < 0.03


def test_delayed_burst_found_at_zero_lag_only(orc, mf):
    """Noise plus a 40 s tone burst that reaches J 2.5 ms after I: Eq. 8 along the burst's row with
    the true delay scores high on the zero-lag map and near zero on maps slid by more than the
    burst (a stationary tone would stay coherent under a slide; a transient does not)."""
    fs, M, T, nb, k_lo, F = 256.0, 256, 300, 4, 20, 60
    n = (T + 1) * M // 2
    xi, xj = synth.white_strain(n, seed=15), synth.white_strain(n, seed=15, stream=1)
    k0, tau = 41, 0.0025
    f0 = k0 * fs / M
    for x, d in ((xi, 0.0), (xj, tau)):
        synth.add_tone(x, fs, f0, 0.5, phase_turns=0.2, delay_s=d, t_start_s=50.0, t_stop_s=90.0)
    maps = mf.form_maps(xi, xj, fs, M, T, k_lo, F, nb, [0, 100, 200])
    dtau = round(tau / orc.DTAU_UNIT_S)
    row = k0 - k_lo
    # columns 101 .. 177 (0.5 s apart, 1 s long) lie inside the burst
    track = np.array([(101, 177, row * 256 + 128, row * 256 + 128, row * 256 + 128, dtau)], dtype=orc.TRACK_DTYPE)
    z = [orc.score_list(orc.Map(Y.astype(np.complex64), s.astype(np.float32), fq4_lo=int(16 * k_lo * fs / M),
                                dfq4=int(16 * fs / M)), track)[0] for Y, s in maps]
    assert z[0] > 10 and abs(z[1]) < 4 and abs(z[2]) < 4
