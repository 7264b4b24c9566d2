"""Synthetic detector strain: white Gaussian noise and a delayed sinusoidal injection.

These stand in for the two detectors' strain time series from which the cross-power
ft-map is formed (the paper's recoloured LIGO and Monte Carlo data are not available).
Samples are FP32; noise is unit-variance (strain in arbitrary units: the complex SNR
map formed from it does not depend on an overall scale of either stream).
"""
from __future__ import annotations

import numpy as np

from .maps import normal_pairs


def white_strain(n: int, seed: int, stream: int = 0, std: float = 1.0) -> np.ndarray:
    """n samples of white Gaussian noise with standard deviation ``std``, FP32.

    Streams 2*stream and 2*stream+1 of the (seed, stream) generator are the two
    Box-Muller outputs, interleaved, so different ``stream`` values are independent.
    """
    if n < 0:
        raise ValueError("n must be non-negative")
    a, b = normal_pairs(seed, 1000 + stream, (n + 1) // 2)
    x = np.empty(2 * a.size, dtype=np.float64)
    x[0::2], x[1::2] = a, b
    return (std * x[:n]).astype(np.float32)


def add_tone(s: np.ndarray, fs: float, freq_hz: float, amp: float, phase_turns: float = 0.0,
             delay_s: float = 0.0, t_start_s: float = 0.0, t_stop_s: float | None = None,
             chirp_hz_per_s: float = 0.0) -> None:
    """In place: s[n] += amp cos(2 pi phi(n/fs - delay_s)), for t_start_s <= n/fs - delay_s < t_stop_s.

    phi(u) = phase_turns + freq_hz u + chirp_hz_per_s u^2 / 2 (a linear chirp; a tone when
    the chirp rate is 0). The same call with ``delay_s`` = tau on a second stream gives a
    signal that reaches that detector tau seconds later.
    """
    n = np.arange(s.size, dtype=np.float64)
    u = n / fs - delay_s
    on = u >= t_start_s
    if t_stop_s is not None:
        on &= u < t_stop_s
    phi = phase_turns + freq_hz * u + 0.5 * chirp_hz_per_s * u * u
    add = np.where(on, amp * np.cos(2.0 * np.pi * phi), 0.0)
    s[:] = (s.astype(np.float64) + add).astype(np.float32)
