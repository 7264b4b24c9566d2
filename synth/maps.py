"""Synthetic ft-maps: Gaussian noise with optional log-uniform sigma, and injections.

Noise model (the reading used throughout): Y = sigma * (n_re + i n_im) with
n_re, n_im iid N(0, 1), so that the complex SNR map p = Y / sigma (the paper's
complex signal-to-noise ratio, with rho = Y / sigma as in its appendix) has
iid standard-normal real and imaginary parts whatever sigma is.
"""
from __future__ import annotations

import hashlib

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to the uint64 states ``x`` (already advanced)."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _stream_words(seed: int, stream: int, n: int) -> np.ndarray:
    """n uint64 words of the SplitMix64 sequence keyed by (seed, stream)."""
    base = splitmix64(np.array([(seed * 0x100000001B3 + stream) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
    idx = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = base + idx * _GOLDEN
    return splitmix64(states)


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles in (0, 1): the top 53 bits of each word, offset by half an ulp."""
    w = _stream_words(seed, stream, n)
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normal_pairs(seed: int, stream: int, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Two arrays of n iid N(0,1) doubles by Box-Muller."""
    u = uniform01(seed, stream, 2 * n)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang), r * np.sin(ang)


def noise_map(T: int, F: int, seed: int, sigma: str | tuple = "unit", stream: int = 0):
    """Gaussian noise map.

    Returns (Y, sigma): Y complex64 [T][F], sigma float32 [T][F], time-major.
    ``sigma`` is "unit" (sigma = 1) or ("loguniform", lo, hi): log sigma uniform
    on [log lo, log hi]. Stream ``stream`` selects an independent map for the
    same seed (e.g. one per background map).
    """
    if T < 0 or F < 0:
        raise ValueError("T and F must be non-negative")
    n = T * F
    re, im = normal_pairs(seed, 2 * stream, n)
    if sigma == "unit":
        sig = np.ones(n, dtype=np.float64)
    else:
        kind, lo, hi = sigma
        if kind != "loguniform" or not (0 < lo <= hi):
            raise ValueError(f"bad sigma spec {sigma!r}")
        u = uniform01(seed, 2 * stream + 1, n)
        sig = np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * u)
    sig32 = sig.astype(np.float32)
    s = sig32.astype(np.float64)
    Y = (s * re + 1j * (s * im)).astype(np.complex64)
    return Y.reshape(T, F), sig32.reshape(T, F)


def add_pixels(Y: np.ndarray, sigma: np.ndarray, cols, rows, amp: float, phase_turns) -> None:
    """In place: Y[c, r] += sigma[c, r] * amp * exp(2 pi i phase) at the given pixels.

    The amplitude is in units of the complex SNR p = Y / sigma, so each listed
    pixel's p gains amp * exp(2 pi i phase). ``phase_turns`` is a scalar or one
    value per pixel (in turns). Pixels are added in the order given; listing a
    pixel twice adds twice.
    """
    cols = np.asarray(cols, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    ph = np.broadcast_to(np.asarray(phase_turns, dtype=np.float64), cols.shape)
    T, F = Y.shape
    if cols.shape != rows.shape:
        raise ValueError("cols and rows must have the same shape")
    if cols.size and (cols.min() < 0 or cols.max() >= T or rows.min() < 0 or rows.max() >= F):
        raise ValueError("pixel outside the map")
    for c, r, p in zip(cols.tolist(), rows.tolist(), ph.tolist()):
        s = float(sigma[c, r])
        Y[c, r] = np.complex64(complex(Y[c, r]) + s * amp * np.exp(2j * np.pi * p))


def bezier_rows_float(t0: int, t2: int, f0: float, f1: float, f2: float) -> tuple[np.ndarray, np.ndarray]:
    """Pixels of a drawn signal: one row per column t0..t2 along a quadratic curve, in float.

    Used only to draw synthetic signals into maps (a drawing helper, not the
    search's template rasteriser): column t0+k takes row floor(f(k/(t2-t0)))
    with f the quadratic Bezier through f0, f1, f2 (row units).
    """
    if t2 <= t0:
        raise ValueError("need t2 > t0")
    k = np.arange(t2 - t0 + 1, dtype=np.float64)
    x = k / (t2 - t0)
    f = (1 - x) ** 2 * f0 + 2 * (1 - x) * x * f1 + x**2 * f2
    return (t0 + k).astype(np.int64), np.floor(f).astype(np.int64)


def map_sha256(Y: np.ndarray, sigma: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(Y).tobytes())
    h.update(np.ascontiguousarray(sigma).tobytes())
    return h.hexdigest()
