"""Oracle of the cross-power map formation (test infrastructure only).

Plain numpy in FP64, one step per function, in the order the paper forms its complex
SNR spectrogram (Sec. II, Eq. 7, and the formalism appendix):

1. the strain of each detector is cut into columns of M samples that overlap by half,
   each weighted by a Hann window (Sec. IV: 50 %-overlapping Hann windows) and
   Fourier-transformed: s~(t; f_k) = dt * sum_n w[n] s[t M/2 + n] exp(-2 pi i k n / M);
2. the auto-power of each column is (2 / Nrm) |s~|^2 with Nrm = M dt <w^2> (the DFT
   normalisation, corrected for the window's mean square <w^2> = 3/8), and P'(t; f), the
   power "in the segments neighbouring t", is its mean over the columns 2 .. nb + 1 away on
   either side (the columns 1 away share half their samples with t and are skipped);
3. the cross-power estimator and its standard deviation follow the appendix with the
   direction filter Q set to 1 (the direction enters later, through Eq. 8's phase factor):
   Y = (2 / Nrm) s~_I^* s~_J and sigma = sqrt(P'_I P'_J / 2), so that Y / sigma is twice the
   paper's lambda s~_I^* s~_J and has unit-variance real and imaginary parts in noise;
4. a time slide by ``shift`` columns pairs column t of I with column (t + shift) mod T of J
   (J's spectrum and its P' travel together).

Readings (the paper states none of these numbers): the periodic Hann window
w[n] = sin^2(pi n / M); non-wrapping columns t = 0 .. T-1 starting at t M / 2; circular
slides within the T analysed columns. The FFT is numpy's (a library primitive for step 1).
"""
from __future__ import annotations

import numpy as np

HANN_MEAN_SQUARE = 3.0 / 8.0  # mean of sin^4(pi n / M) over n = 0 .. M-1, for M >= 3


def hann(M: int) -> np.ndarray:
    """Periodic Hann window w[n] = sin^2(pi n / M), n = 0 .. M-1."""
    n = np.arange(M, dtype=np.float64)
    return np.sin(np.pi * n / M) ** 2


def n_columns_max(n_samples: int, M: int) -> int:
    """Largest T with every column inside the stream: (T + 1) M / 2 <= n_samples."""
    return max(0, 2 * n_samples // M - 1)


def column_spectra(strain: np.ndarray, fs: float, M: int, T: int, k_lo: int, F: int) -> np.ndarray:
    """s~(t; k) for columns t < T and bins k_lo .. k_lo+F-1, complex128 [T][F] (step 1)."""
    if M < 8 or M & (M - 1):
        raise ValueError("M must be a power of two >= 8")
    if not (0 <= k_lo and k_lo + F <= M // 2 and F >= 1):
        raise ValueError("bins must lie in [0, M/2)")
    if T < 1 or (T + 1) * (M // 2) > strain.size:
        raise ValueError("columns run past the end of the strain")
    x = np.asarray(strain, dtype=np.float64)
    w = hann(M)
    dt = 1.0 / fs
    out = np.empty((T, F), dtype=np.complex128)
    for t in range(T):
        seg = x[t * (M // 2): t * (M // 2) + M] * w
        out[t] = dt * np.fft.rfft(seg)[k_lo:k_lo + F]
    return out


def norm_const(fs: float, M: int) -> float:
    """Nrm = M dt <w^2>: the DFT normalisation of the appendix for a Hann-windowed column."""
    return M / fs * HANN_MEAN_SQUARE


def column_power(spec: np.ndarray, fs: float, M: int) -> np.ndarray:
    """(2 / Nrm) |s~|^2 per column and bin (step 2, before averaging)."""
    return 2.0 / norm_const(fs, M) * np.abs(spec) ** 2


def neighbour_mean(pw: np.ndarray, nb: int) -> np.ndarray:
    """P'(t) = mean of pw(t') over 2 <= |t' - t| <= nb + 1, 0 <= t' < T (step 2)."""
    T = pw.shape[0]
    if nb < 1:
        raise ValueError("nb must be >= 1")
    out = np.empty_like(pw, dtype=np.float64)
    for t in range(T):
        nbrs = [u for u in range(t - nb - 1, t + nb + 2) if abs(u - t) >= 2 and 0 <= u < T]
        if not nbrs:
            raise ValueError("a column has no neighbour (T too small)")
        out[t] = pw[nbrs].mean(axis=0)
    return out


def psd(spec: np.ndarray, fs: float, M: int, nb: int) -> np.ndarray:
    """P'(t; f) of one detector from its column spectra."""
    return neighbour_mean(column_power(spec, fs, M), nb)


def form_map(spec_i: np.ndarray, psd_i: np.ndarray, spec_j: np.ndarray, psd_j: np.ndarray,
             fs: float, M: int, shift: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """(Y, sigma) of the slide by ``shift`` columns (steps 3 and 4), complex128 / float64 [T][F]."""
    T = spec_i.shape[0]
    tj = (np.arange(T) + shift) % T
    Y = 2.0 / norm_const(fs, M) * np.conj(spec_i) * spec_j[tj]
    sigma = np.sqrt(psd_i * psd_j[tj] / 2.0)
    return Y, sigma


def form_maps(strain_i: np.ndarray, strain_j: np.ndarray, fs: float, M: int, T: int, k_lo: int, F: int,
              nb: int, shifts) -> list[tuple[np.ndarray, np.ndarray]]:
    """All steps: the (Y, sigma) map of each time slide in ``shifts``."""
    si = column_spectra(strain_i, fs, M, T, k_lo, F)
    sj = column_spectra(strain_j, fs, M, T, k_lo, F)
    pi, pj = psd(si, fs, M, nb), psd(sj, fs, M, nb)
    return [form_map(si, pi, sj, pj, fs, M, int(s)) for s in shifts]
