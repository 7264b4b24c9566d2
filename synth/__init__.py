"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle scripts.

This module draws the ft-maps that stand in for the paper's LIGO / Monte Carlo
spectrograms (the data behind its Tables I-III are not available): complex
cross-power pixels Y and their standard deviations sigma, laid out time-major
([T][F], frequency contiguous), plus a helper that adds a complex amplitude at
a caller-given list of pixels (an injection).

It holds none of the search method's arithmetic: no template generator, no
rasteriser, no phase factor, no statistic. Callers that need the pixels of a
template (for an injection matched to it) obtain them elsewhere and pass them
in. ``strain`` draws the two detectors' strain streams (white noise, delayed
tones and chirps) from which cross-power maps are formed.

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) keyed by (seed, stream) and
turned into normals by the Box-Muller transform, all in numpy uint64/float64,
so the bytes do not depend on numpy's own generator streams.
"""
from .maps import (  # noqa: F401
    splitmix64,
    uniform01,
    normal_pairs,
    noise_map,
    add_pixels,
    bezier_rows_float,
    map_sha256,
)
from .strain import white_strain, add_tone  # noqa: F401
