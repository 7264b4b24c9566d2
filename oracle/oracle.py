"""ctypes wrapper of the C oracle (test infrastructure only).

Every function takes numpy arrays and returns numpy arrays / Python ints. Maps
are passed to C as FP64 copies: Y complex [T][F] -> interleaved (re, im)
doubles, sigma -> doubles (exact widening of FP32 inputs).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import build, lib_path

NORM_SQRT_N = 0
NORM_N = 1
FBITS = 8  # control frequencies are in units of 1/256 row
DTAU_UNIT_S = 2.0 ** -28  # time delays are integers in units of 2^-28 s

TRACK_DTYPE = np.dtype([("t0", "<i4"), ("t2", "<i4"), ("f0", "<u4"), ("f1", "<u4"),
                        ("f2", "<u4"), ("dtau", "<i4")])
# a template with a free t_mid (integer t1 in [t0, t2])
TRACK_TM_DTYPE = np.dtype([("t0", "<i4"), ("t1", "<i4"), ("t2", "<i4"), ("f0", "<u4"), ("f1", "<u4"),
                           ("f2", "<u4"), ("dtau", "<i4")])


class _Track(C.Structure):
    _fields_ = [("t0", C.c_int32), ("t2", C.c_int32), ("f0", C.c_uint32), ("f1", C.c_uint32),
                ("f2", C.c_uint32), ("dtau", C.c_int32)]


class _Map(C.Structure):
    _fields_ = [("Y", C.c_void_p), ("sigma", C.c_void_p), ("T", C.c_int32), ("F", C.c_int32),
                ("ld", C.c_int64), ("fq4_lo", C.c_int32), ("dfq4", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_npairs.argtypes = [C.c_int32, C.c_int32]
        L.orc_npairs.restype = C.c_int64
        L.orc_unrank.argtypes = [C.c_uint64, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_unrank.restype = None
        L.orc_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                               C.c_int32, C.POINTER(_Track)]
        L.orc_draw.restype = C.c_int
        L.orc_rows.argtypes = [C.POINTER(_Track), C.c_int32, C.c_void_p]
        L.orc_rows.restype = C.c_int
        L.orc_phase_turns.argtypes = [C.c_int64, C.c_int32]
        L.orc_phase_turns.restype = C.c_double
        L.orc_score.argtypes = [C.POINTER(_Map), C.POINTER(_Track), C.c_int32]
        L.orc_score.restype = C.c_double
        L.orc_score_gen.argtypes = [C.POINTER(_Map), C.c_uint64, C.c_uint32, C.c_int32, C.c_int32,
                                    C.c_uint64, C.c_int64, C.c_int32, C.c_void_p]
        L.orc_score_gen.restype = C.c_int
        L.orc_score_gen_idx.argtypes = [C.POINTER(_Map), C.c_uint64, C.c_uint32, C.c_int32, C.c_int32,
                                        C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
        L.orc_score_gen_idx.restype = C.c_int
        L.orc_score_list.argtypes = [C.POINTER(_Map), C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
        L.orc_draw_tm.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_void_p]
        L.orc_draw_tm.restype = C.c_int
        L.orc_rows_tm.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
        L.orc_rows_tm.restype = C.c_int
        L.orc_score_tm_gen_idx.argtypes = [C.POINTER(_Map), C.c_uint64, C.c_uint32, C.c_int32, C.c_int32, C.c_void_p,
                                           C.c_int64, C.c_int32, C.c_void_p]
        L.orc_score_tm_gen_idx.restype = C.c_int
        L.orc_score_tm_list.argtypes = [C.POINTER(_Map), C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
        L.orc_score_tm_list.restype = C.c_int
        L.orc_score_maxdelay_gen_idx.argtypes = [C.POINTER(_Map), C.c_uint64, C.c_uint32, C.c_int32, C.c_int32,
                                                 C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                                 C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_score_maxdelay_gen_idx.restype = C.c_int
        L.orc_score_maxdelay_list.argtypes = [C.POINTER(_Map), C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                              C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_score_maxdelay_list.restype = C.c_int
        L.orc_score_list.restype = C.c_int
        L.orc_argmax.argtypes = [C.c_void_p, C.c_int64]
        L.orc_argmax.restype = C.c_int64
        _bind_ext(L)
        _lib = L
    return _lib


def _bind_ext(L):
    """Bind the extension entry points (top-K, bilinear smooth SNR, refinement)."""
    L.orc_topk.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    L.orc_topk.restype = C.c_int
    L.orc_smooth.argtypes = [C.POINTER(_Map), C.c_void_p, C.c_int32, C.c_void_p]
    L.orc_smooth.restype = C.c_double
    L.orc_refine.argtypes = [C.POINTER(_Map), C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_void_p]
    L.orc_refine.restype = C.c_double
    L.orc_refine_trace.argtypes = [C.POINTER(_Map), C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                   C.c_void_p, C.c_void_p]
    L.orc_refine_trace.restype = C.c_double
    L.orc_theta_to_track.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_Track)]
    L.orc_theta_to_track.restype = None


# --------------------------------------------------------------------------- primitives

def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c, k, out)
    return out


def npairs(T: int, L: int) -> int:
    return int(lib().orc_npairs(T, L))


def unrank(k: int, L: int) -> tuple[int, int]:
    a, b = C.c_int32(), C.c_int32()
    lib().orc_unrank(k, L, C.byref(a), C.byref(b))
    return a.value, b.value


def dtau_units(dtau_max_s: float) -> int:
    """Delay bound in 2^-28 s units, rounded to nearest (10 ms -> 2684355)."""
    return int(round(dtau_max_s / DTAU_UNIT_S))


def draw(seed: int, stream: int, j: int, T: int, F: int, L: int, D: int) -> np.ndarray:
    t = _Track()
    if lib().orc_draw(seed, stream, j, T, F, L, D, C.byref(t)) != 0:
        raise ValueError("invalid draw parameters")
    out = np.zeros((), dtype=TRACK_DTYPE)
    for name in TRACK_DTYPE.names:
        out[name] = getattr(t, name)
    return out


def draw_many(seed: int, stream: int, first: int, n: int, T: int, F: int, L: int, D: int) -> np.ndarray:
    out = np.zeros(n, dtype=TRACK_DTYPE)
    t = _Track()
    fn = lib().orc_draw
    for i in range(n):
        if fn(seed, stream, first + i, T, F, L, D, C.byref(t)) != 0:
            raise ValueError("invalid draw parameters")
        out[i] = (t.t0, t.t2, t.f0, t.f1, t.f2, t.dtau)
    return out


def draw_patch_many(seed: int, stream: int, first: int, n: int, T: int, F: int, L: int, D: int,
                    center: int) -> np.ndarray:
    """Templates whose delay prior is a sky patch instead of the whole sky (Sec. VI): the delay is
    uniform on the integers [center - D, center + D] -- the isotropic draw on [-D, D] moved by
    ``center``, with every other field as draw_many. Under isotropy within a band of directions
    whose angle to the baseline spans [theta_1, theta_2], the delay is exactly uniform on the
    matching interval; a patch is taken as such a band."""
    if abs(center) + D >= 1 << 30:
        raise ValueError("the patch leaves the delay range")
    out = draw_many(seed, stream, first, n, T, F, L, D)
    out["dtau"] = out["dtau"].astype(np.int64) + center
    return out


def _as_track(tr) -> _Track:
    tr = np.asarray(tr, dtype=TRACK_DTYPE)
    return _Track(int(tr["t0"]), int(tr["t2"]), int(tr["f0"]), int(tr["f1"]), int(tr["f2"]),
                  int(tr["dtau"]))


def rows(tr, F: int) -> np.ndarray:
    t = _as_track(tr)
    N = t.t2 - t.t0 + 1
    out = np.zeros(max(N, 1), dtype=np.int32)
    if lib().orc_rows(C.byref(t), F, out.ctypes.data) != N:
        raise ValueError("invalid track")
    return out[:N]


def phase_turns(fq4: int, dtau: int) -> float:
    return float(lib().orc_phase_turns(fq4, dtau))


# --------------------------------------------------------------------------- maps and scores

class Map:
    """FP64 copy of a (Y, sigma) map for the oracle; keeps the buffers alive."""

    def __init__(self, Y: np.ndarray, sigma: np.ndarray, fq4_lo: int = 1600, dfq4: int = 16):
        Y = np.asarray(Y)
        sigma = np.asarray(sigma)
        if Y.ndim != 2 or Y.shape != sigma.shape:
            raise ValueError("Y and sigma must be [T][F] arrays of the same shape")
        self.T, self.F = Y.shape
        self.Yd = np.ascontiguousarray(Y.astype(np.complex128)).view(np.float64)
        self.sd = np.ascontiguousarray(sigma.astype(np.float64))
        self.fq4_lo, self.dfq4 = int(fq4_lo), int(dfq4)
        self.c = _Map(self.Yd.ctypes.data, self.sd.ctypes.data, self.T, self.F, self.F,
                      self.fq4_lo, self.dfq4)


def score(m: Map, tr, norm: int = NORM_SQRT_N) -> float:
    t = _as_track(tr)
    return float(lib().orc_score(C.byref(m.c), C.byref(t), norm))


def score_gen(m: Map, seed: int, stream: int, L: int, D: int, first: int, n: int,
              norm: int = NORM_SQRT_N) -> np.ndarray:
    z = np.zeros(n, dtype=np.float64)
    if lib().orc_score_gen(C.byref(m.c), seed, stream, L, D, first, n, norm, z.ctypes.data) != 0:
        raise ValueError("invalid parameters")
    return z


def score_gen_idx(m: Map, seed: int, stream: int, L: int, D: int, idx, norm: int = NORM_SQRT_N) -> np.ndarray:
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    z = np.zeros(idx.size, dtype=np.float64)
    if lib().orc_score_gen_idx(C.byref(m.c), seed, stream, L, D, idx.ctypes.data, idx.size, norm,
                               z.ctypes.data) != 0:
        raise ValueError("invalid parameters")
    return z


def score_list(m: Map, tracks: np.ndarray, norm: int = NORM_SQRT_N) -> np.ndarray:
    tracks = np.ascontiguousarray(np.asarray(tracks, dtype=TRACK_DTYPE))
    z = np.zeros(tracks.size, dtype=np.float64)
    lib().orc_score_list(C.byref(m.c), tracks.ctypes.data, tracks.size, norm, z.ctypes.data)
    return z


def draw_tm_many(seed: int, stream: int, first: int, n: int, T: int, F: int, L: int, D: int) -> np.ndarray:
    """Free-t_mid templates j = first .. first+n-1 (TRACK_TM_DTYPE)."""
    out = np.zeros(n, dtype=TRACK_TM_DTYPE)
    for i in range(n):
        if lib().orc_draw_tm(seed, stream, first + i, T, F, L, D, out[i:i + 1].ctypes.data) != 0:
            raise ValueError("invalid draw parameters")
    return out


def rows_tm(track, F: int) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(track, dtype=TRACK_TM_DTYPE).reshape(1))
    rows = np.zeros(int(t["t2"][0]) - int(t["t0"][0]) + 1, dtype=np.int32)
    if lib().orc_rows_tm(t.ctypes.data, F, rows.ctypes.data) < 0:
        raise ValueError("invalid track")
    return rows


def score_tm_gen_idx(m: Map, seed: int, stream: int, L: int, D: int, idx, norm: int = NORM_SQRT_N) -> np.ndarray:
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    z = np.zeros(idx.size, dtype=np.float64)
    if lib().orc_score_tm_gen_idx(C.byref(m.c), seed, stream, L, D, idx.ctypes.data, idx.size, norm,
                                  z.ctypes.data) != 0:
        raise ValueError("invalid parameters")
    return z


def score_tm_list(m: Map, tracks: np.ndarray, norm: int = NORM_SQRT_N) -> np.ndarray:
    tracks = np.ascontiguousarray(np.asarray(tracks, dtype=TRACK_TM_DTYPE))
    z = np.zeros(tracks.size, dtype=np.float64)
    lib().orc_score_tm_list(C.byref(m.c), tracks.ctypes.data, tracks.size, norm, z.ctypes.data)
    return z


def score_maxdelay_gen_idx(m: Map, seed: int, stream: int, L: int, D: int, idx, d0: int, step: int, n_tau: int,
                           norm: int = NORM_SQRT_N):
    """Delay-maximised scores of templates j = idx (geometry drawn as usual, delay replaced by
    the grid d0 + m*step, m < n_tau): (z_max, maximising m)."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    z = np.zeros(idx.size, dtype=np.float64)
    mm = np.zeros(idx.size, dtype=np.int32)
    if lib().orc_score_maxdelay_gen_idx(C.byref(m.c), seed, stream, L, D, idx.ctypes.data, idx.size, d0, step,
                                        n_tau, norm, z.ctypes.data, mm.ctypes.data) != 0:
        raise ValueError("invalid parameters")
    return z, mm


def score_maxdelay_list(m: Map, tracks: np.ndarray, d0: int, step: int, n_tau: int, norm: int = NORM_SQRT_N):
    tracks = np.ascontiguousarray(np.asarray(tracks, dtype=TRACK_DTYPE))
    z = np.zeros(tracks.size, dtype=np.float64)
    mm = np.zeros(tracks.size, dtype=np.int32)
    if lib().orc_score_maxdelay_list(C.byref(m.c), tracks.ctypes.data, tracks.size, d0, step, n_tau, norm,
                                     z.ctypes.data, mm.ctypes.data) != 0:
        raise ValueError("invalid parameters")
    return z, mm


def argmax(z: np.ndarray) -> int:
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    return int(lib().orc_argmax(z.ctypes.data, z.size))


# --------------------------------------------------------------------------- extensions

def topk(z: np.ndarray, K: int) -> np.ndarray:
    """Indices of the K best scores (score descending, index ascending; NaN lowest)."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    idx = np.zeros(max(K, 1), dtype=np.int64)
    if lib().orc_topk(z.ctypes.data, z.size, K, idx.ctypes.data) != 0:
        raise ValueError("bad K")
    return idx[:K]


def smooth(m: Map, theta, K: int, grad: bool = True):
    """Bilinear smooth SNR of theta = (tau0, tau2, phi0, phi1, phi2, dtau_ms); returns (z, grad[6])."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(6))
    g = np.zeros(6, dtype=np.float64)
    z = lib().orc_smooth(C.byref(m.c), th.ctypes.data, K, g.ctypes.data if grad else None)
    return float(z), g


def refine(m: Map, theta, K: int, steps: int, L: int, dtau_max_ms: float, sched=(1.0, 0.02, 0.5, 0.01)):
    """Projected ascent on the smooth SNR; returns (best theta, its smooth SNR)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(6)).copy()
    sc = np.ascontiguousarray(np.asarray(sched, dtype=np.float64))
    z = lib().orc_refine(C.byref(m.c), th.ctypes.data, K, steps, L, dtau_max_ms, sc.ctypes.data)
    return th, float(z)


def refine_trace(m: Map, theta, K: int, steps: int, L: int, dtau_max_ms: float, sched=(1.0, 0.02, 0.5, 0.01)):
    """As refine, plus every iterate: returns (best theta, its z~, trace[steps + 1][7]) where
    trace[s] = (theta_s, z~(theta_s)), theta_0 the projected start."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(6)).copy()
    sc = np.ascontiguousarray(np.asarray(sched, dtype=np.float64))
    tr = np.zeros((steps + 1, 7), dtype=np.float64)
    z = lib().orc_refine_trace(C.byref(m.c), th.ctypes.data, K, steps, L, dtau_max_ms, sc.ctypes.data,
                               tr.ctypes.data)
    return th, float(z), tr


def theta_to_track(theta, T: int, F: int, L: int, dtau_max: int) -> np.ndarray:
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(6))
    t = _Track()
    lib().orc_theta_to_track(th.ctypes.data, T, F, L, dtau_max, C.byref(t))
    out = np.zeros((), dtype=TRACK_DTYPE)
    for name in TRACK_DTYPE.names:
        out[name] = getattr(t, name)
    return out


def quantize_p16(Y: np.ndarray, sigma: np.ndarray):
    """FP16 storage of the complex SNR p = Y/sigma: 32 bits per pixel in polar form, with a per-map
    power-of-two scale.

    p is formed in FP32 (correctly rounded division). Its magnitude |p| (FP64, from the exact squares
    of the FP32 components: one rounding of the sum, one of the square root) is multiplied by 2^-e,
    e = ceil(log2(max |p|)) - 15 so that every scaled magnitude is at most 2^15, and rounded to
    binary16 (round to nearest even, straight from FP64: numpy's conversion). Its argument
    atan2(Im p, Re p) / (2 pi), a fraction of a turn, is rounded to the nearest multiple of 2^-16
    (ties to even) modulo one turn. Returns (the stored halves as a [T][F][2] uint16 array: [..., 0]
    the argument in units of 2^-16 turn, [..., 1] the binary16 bits of the scaled magnitude; e;
    the dequantised p = magnitude * 2^e * exp(2 pi i argument) as complex128).
    """
    pr = (Y.real.astype(np.float32) / sigma.astype(np.float32)).astype(np.float32)
    pi = (Y.imag.astype(np.float32) / sigma.astype(np.float32)).astype(np.float32)
    x, y = pr.astype(np.float64), pi.astype(np.float64)
    mag = np.sqrt(x * x + y * y)
    amax = float(mag.max(initial=0.0))
    e = 0
    if amax > 0:
        fr, k = math.frexp(amax)  # amax = fr * 2^k, fr in [1/2, 1): ceil(log2 amax) is k, or k - 1 at fr = 1/2
        e = (k if fr > 0.5 else k - 1) - 15
    mag16 = (mag * 2.0 ** -e).astype(np.float16)
    turns = np.arctan2(y, x) * 0.15915494309189535  # 1 / (2 pi), rounded
    arg16 = (np.rint(turns * 65536.0).astype(np.int64) & 0xFFFF).astype(np.uint16)
    q = np.stack([arg16, mag16.view(np.uint16)], axis=-1)
    deq = mag16.astype(np.float64) * 2.0 ** e * np.exp(2j * np.pi * (arg16.astype(np.float64) / 65536.0))
    return q, e, deq
