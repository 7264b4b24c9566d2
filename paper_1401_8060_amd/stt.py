"""Python binding of libstt (the C ABI in include/stt.h).

Argument marshalling only: every step of the search runs in the HIP kernels
of libstt.so. torch provides device memory and streams; tensors are passed by
data pointer. There is no fallback: if libstt.so is missing or fails to load
this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstt.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
NORM_SQRT_N, NORM_N = 0, 1
C64F32, C16 = 0, 1  # map element formats: (complex64 Y, float32 sigma) / FP16 p
FBITS = 8
MAX_T, MAX_F = 2896, 32767
DTAU_UNIT_S = 2.0 ** -28
PATH_AUTO, PATH_DIRECT, PATH_SLAB, PATH_WAVE = 0, 1, 2, 3
STAGE_SCORE, STAGE_BIN, STAGE_CALL = 0, 1, 2


class SttError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"stt error {status}: {msg}")
        self.status = status


class Track(C.Structure):
    _fields_ = [("t0", C.c_int32), ("t2", C.c_int32), ("f0", C.c_uint32), ("f1", C.c_uint32),
                ("f2", C.c_uint32), ("dtau", C.c_int32)]


class _Gen(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("stream", C.c_uint32), ("min_len", C.c_int32),
                ("dtau_max", C.c_int32), ("dtau_center", C.c_int32)]


class _Map(C.Structure):
    _fields_ = [("T", C.c_int32), ("F", C.c_int32), ("ld", C.c_int64), ("dtype", C.c_int32),
                ("scale_exp", C.c_int32), ("Y", C.c_void_p), ("sigma", C.c_void_p),
                ("fq4_lo", C.c_int32), ("dfq4", C.c_int32)]


class _Spectro(C.Structure):
    _fields_ = [("fs", C.c_double), ("M", C.c_int32), ("k_lo", C.c_int32), ("F", C.c_int32), ("nb", C.c_int32)]


@dataclass
class Spectro:
    """Map-formation parameters (stt_spectro): sample rate, samples per column (a power of two;
    columns overlap by half), the kept bins k_lo .. k_lo+F-1, neighbour columns per side in P'."""
    fs: float
    M: int
    k_lo: int
    F: int
    nb: int = 4

    def c(self) -> _Spectro:
        return _Spectro(float(self.fs), self.M, self.k_lo, self.F, self.nb)

    def fq4(self) -> tuple[int, int]:
        """(fq4_lo, dfq4) of the formed maps: row r at (k_lo + r) fs / M Hz, in 1/16 Hz."""
        d = 16.0 * self.fs / self.M
        if d != int(d):
            raise ValueError(f"fs/M = {self.fs / self.M} Hz is not a multiple of 1/16 Hz")
        return int(d) * self.k_lo, int(d)

    def n_columns(self, n_samples: int) -> int:
        """Largest T with every column inside n_samples samples."""
        return max(0, 2 * n_samples // self.M - 1)


_lib = None


def lib():
    """Load libstt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_1401_8060_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        sigs = {
            "stt_create": ([C.c_int, vp, C.POINTER(vp)], i32),
            "stt_destroy": ([vp], i32),
            "stt_set_stream": ([vp, vp], i32),
            "stt_sync": ([vp], i32),
            "stt_strerror": ([i32], C.c_char_p),
            "stt_last_error": ([vp], C.c_char_p),
            "stt_reserve": ([vp, i64], i32),
            "stt_set_timing": ([vp, i32], i32),
            "stt_kernel_ms": ([vp, i32, C.POINTER(C.c_float)], i32),
            "stt_kernel_ms_total": ([vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int32)], i32),
            "stt_set_path": ([vp, i32, i32], i32),
            "stt_set_slab_shape": ([vp, i32, i32], i32),
            "stt_set_trig": ([vp, i32], i32),
            "stt_set_staging": ([vp, i32], i32),
            "stt_make_tracks": ([vp, C.POINTER(_Gen), i32, i32, i64, i64, vp], i32),
            "stt_score": ([vp, C.POINTER(_Map), C.POINTER(_Gen), vp, i64, i64, i32, vp, vp], i32),
            "stt_argmax": ([vp, vp, i64, i64, vp], i32),
            "stt_key_encode": ([C.c_float, C.c_uint32], u64),
            "stt_key_decode": ([u64, C.POINTER(C.c_float), C.POINTER(C.c_uint32)], None),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _bind_ext(L)
        _lib = L
    return _lib


def _bind_ext(L):
    """Entry points of the extensions (precision, batching, differentiation), bound when exported."""
    from . import stt_ext
    stt_ext.bind(L)


EXPORTED = [
    "stt_create", "stt_destroy", "stt_set_stream", "stt_sync", "stt_strerror", "stt_last_error",
    "stt_reserve", "stt_set_timing", "stt_kernel_ms", "stt_kernel_ms_total", "stt_set_path", "stt_set_slab_shape", "stt_set_trig", "stt_set_staging", "stt_make_tracks", "stt_score",
    "stt_argmax", "stt_key_encode", "stt_key_decode",
]


# ----------------------------------------------------------------------------- plain data

@dataclass
class Gen:
    """Template law: Philox seed/stream, minimum length L (pixels), delay half-width and centre
    (2^-28 s units; centre 0 is the all-sky prior, another centre a sky patch's delay band)."""
    seed: int = 1
    stream: int = 0
    min_len: int = 10
    dtau_max: int = 2684355  # 10 ms
    dtau_center: int = 0

    def c(self) -> _Gen:
        return _Gen(self.seed, self.stream, self.min_len, self.dtau_max, self.dtau_center)


def dtau_units(seconds: float) -> int:
    return int(round(seconds / DTAU_UNIT_S))


class Map:
    """A (Y, sigma) ft-map on the GPU: Y complex64 [T][F] (or [T][ld]), sigma float32 same shape."""

    def __init__(self, Y: torch.Tensor, sigma: torch.Tensor, fq4_lo: int = 1600, dfq4: int = 16):
        if Y.dtype != torch.complex64 or sigma.dtype != torch.float32:
            raise TypeError("Y must be complex64 and sigma float32")
        if Y.dim() != 2 or Y.shape != sigma.shape:
            raise ValueError("Y and sigma must be [T][F] tensors of the same shape")
        if not (Y.is_cuda and sigma.is_cuda):
            raise ValueError("Y and sigma must be on the GPU")
        if Y.stride(1) != 1 or sigma.stride(1) != 1 or Y.stride(0) != sigma.stride(0):
            raise ValueError("frequency must be contiguous and both arrays share the column stride")
        self.Y, self.sigma = Y, sigma
        self.T, self.F = Y.shape
        self.ld = Y.stride(0)
        self.fq4_lo, self.dfq4 = fq4_lo, dfq4

    def c(self) -> _Map:
        return _Map(self.T, self.F, self.ld, C64F32, 0, self.Y.data_ptr(), self.sigma.data_ptr(),
                    self.fq4_lo, self.dfq4)


class P16Map:
    """An FP16 map of the complex SNR p = Y/sigma in polar form: data [T][ld][2] int16 halves of one
    32-bit word per pixel, [..., 0] arg p in units of 2^-16 turn, [..., 1] the binary16 bits of
    |p| * 2^-scale_exp."""

    def __init__(self, data: torch.Tensor, scale_exp: int, fq4_lo: int = 1600, dfq4: int = 16):
        if data.dtype != torch.int16 or data.dim() != 3 or data.shape[2] != 2 or not data.is_cuda:
            raise ValueError("data must be a [T][F][2] int16 tensor on the GPU")
        if data.stride(2) != 1 or data.stride(1) != 2:
            raise ValueError("pairs must be contiguous and frequency-contiguous")
        self.data = data
        self.T, self.F = data.shape[0], data.shape[1]
        self.ld = data.stride(0) // 2
        self.scale_exp = int(scale_exp)
        self.fq4_lo, self.dfq4 = fq4_lo, dfq4
        self.Y = data  # device placement for allocations

    def c(self) -> _Map:
        return _Map(self.T, self.F, self.ld, C16, self.scale_exp, self.data.data_ptr(), None,
                    self.fq4_lo, self.dfq4)


def key_decode(key: int) -> tuple[float, int]:
    z, j = C.c_float(), C.c_uint32()
    lib().stt_key_decode(C.c_uint64(int(key) & 0xFFFFFFFFFFFFFFFF), C.byref(z), C.byref(j))
    return z.value, j.value


def key_encode(z: float, j: int) -> int:
    return int(lib().stt_key_encode(z, j))


def tracks_tensor(n: int, device="cuda") -> torch.Tensor:
    """An uninitialised [n][6] int32 tensor laid out as stt_track records."""
    return torch.empty((n, 6), dtype=torch.int32, device=device)


# ----------------------------------------------------------------------------- context

class Context:
    """An stt_ctx bound to a device and (by default) torch's current stream on it."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self._L = lib()
        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = s
        h = C.c_void_p()
        st = self._L.stt_create(device, C.c_void_p(s.cuda_stream), C.byref(h))
        if st != OK:
            raise SttError(st, "stt_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self._L.stt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st: int):
        if st != OK:
            raise SttError(st, self._L.stt_last_error(self.h).decode())

    # -- configuration
    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        self._chk(self._L.stt_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def sync(self):
        self._chk(self._L.stt_sync(self.h))

    def reserve(self, max_tracks: int):
        self._chk(self._L.stt_reserve(self.h, max_tracks))

    def set_timing(self, on: bool):
        self._chk(self._L.stt_set_timing(self.h, 1 if on else 0))

    def kernel_ms(self, which: int = STAGE_SCORE) -> float:
        ms = C.c_float()
        self._chk(self._L.stt_kernel_ms(self.h, which, C.byref(ms)))
        return ms.value

    def kernel_ms_total(self, which: int = STAGE_SCORE) -> tuple[float, int]:
        """(summed milliseconds, number of calls) of a stage since the last total."""
        tot, cnt = C.c_double(), C.c_int32()
        self._chk(self._L.stt_kernel_ms_total(self.h, which, C.byref(tot), C.byref(cnt)))
        return tot.value, cnt.value

    def set_path(self, path: int, lds_bytes: int = 0):
        self._chk(self._L.stt_set_path(self.h, path, lds_bytes))

    def set_slab_shape(self, wg: int, tpt: int):
        self._chk(self._L.stt_set_slab_shape(self.h, wg, tpt))

    def set_staging(self, dma: bool):
        self._chk(self._L.stt_set_staging(self.h, 1 if dma else 0))

    def set_trig(self, hw: bool):
        self._chk(self._L.stt_set_trig(self.h, 1 if hw else 0))

    # -- entry points
    def make_tracks(self, gen: Gen, T: int, F: int, first: int, n: int, out: torch.Tensor | None = None):
        if out is None:
            out = tracks_tensor(n)
        if out.dtype != torch.int32 or out.shape != (n, 6) or not out.is_contiguous():
            raise ValueError("out must be a contiguous [n][6] int32 tensor")
        g = gen.c()
        self._chk(self._L.stt_make_tracks(self.h, C.byref(g), T, F, first, n, C.c_void_p(out.data_ptr())))
        return out

    def score(self, m: Map, gen: Gen | None = None, tracks: torch.Tensor | None = None, first: int = 0,
              n: int | None = None, norm: int = NORM_SQRT_N, snr: torch.Tensor | bool | None = True,
              best_key: torch.Tensor | None = None):
        """Score n tracks (generated from gen, or the given [n][6] int32 tracks).

        Returns (snr tensor or None, best_key tensor). ``snr=True`` allocates the
        output; pass a float32 tensor of n elements to reuse one, or None to skip
        it. ``best_key`` is a 1-element int64 tensor that is max-merged into
        (created as 0 when not given).
        """
        if tracks is not None:
            if tracks.dtype != torch.int32 or tracks.dim() != 2 or tracks.shape[1] != 6 or not tracks.is_contiguous():
                raise ValueError("tracks must be a contiguous [n][6] int32 tensor")
            if n is None:
                n = tracks.shape[0]
            if n > tracks.shape[0]:
                raise ValueError("n exceeds the number of given tracks")
        if n is None:
            raise ValueError("n is required with generated tracks")
        if snr is True:
            snr = torch.empty(n, dtype=torch.float32, device=m.Y.device)
        if snr is not None and snr is not False:
            if snr.dtype != torch.float32 or snr.numel() < n or not snr.is_contiguous():
                raise ValueError("snr must be a contiguous float32 tensor of at least n elements")
        else:
            snr = None
        if best_key is None:
            best_key = torch.zeros(1, dtype=torch.int64, device=m.Y.device)
        mc = m.c()
        g = gen.c() if gen is not None else None
        self._chk(self._L.stt_score(self.h, C.byref(mc), C.byref(g) if g is not None else None,
                                    C.c_void_p(tracks.data_ptr()) if tracks is not None else None,
                                    first, n, norm,
                                    C.c_void_p(snr.data_ptr()) if snr is not None else None,
                                    C.c_void_p(best_key.data_ptr())))
        return snr, best_key

    def score_noalloc(self, m: Map, snr: torch.Tensor | None, best_key: torch.Tensor, gen: Gen | None = None,
                      tracks: torch.Tensor | None = None, first: int = 0, n: int | None = None,
                      norm: int = NORM_SQRT_N):
        """stt_score_noalloc: as score(), with caller-given outputs (snr may be None) and the library's
        fixed scratch instead of allocated memory (at most 4194304 templates per call)."""
        if tracks is not None:
            if tracks.dtype != torch.int32 or tracks.dim() != 2 or tracks.shape[1] != 6 or not tracks.is_contiguous():
                raise ValueError("tracks must be a contiguous [n][6] int32 tensor")
            n = tracks.shape[0] if n is None else n
        if n is None:
            raise ValueError("n is required with generated tracks")
        if snr is not None and (snr.dtype != torch.float32 or snr.numel() < n or not snr.is_contiguous()):
            raise ValueError("snr must be a contiguous float32 tensor of at least n elements")
        if best_key.dtype != torch.int64 or best_key.numel() < 1:
            raise ValueError("best_key must be an int64 tensor")
        mc = m.c()
        g = gen.c() if gen is not None else None
        self._chk(self._L.stt_score_noalloc(self.h, C.byref(mc), C.byref(g) if g is not None else None,
                                            C.c_void_p(tracks.data_ptr()) if tracks is not None else None,
                                            first, n, norm, C.c_void_p(snr.data_ptr()) if snr is not None else None,
                                            C.c_void_p(best_key.data_ptr())))
        return snr, best_key

    def make_tracks_tm(self, gen: Gen, T: int, F: int, first: int, n: int) -> torch.Tensor:
        """Free-t_mid templates j = first .. first+n-1 as an [n][7] int32 tensor (t0, t1, t2, f0, f1, f2, dtau)."""
        out = torch.empty((max(n, 1), 7), dtype=torch.int32, device="cuda")
        g = gen.c()
        self._chk(self._L.stt_make_tracks_tm(self.h, C.byref(g), T, F, first, n, C.c_void_p(out.data_ptr())))
        return out[:n]

    def score_tm(self, m: Map, gen: Gen | None = None, tracks: torch.Tensor | None = None, first: int = 0,
                 n: int | None = None, norm: int = NORM_SQRT_N, snr: torch.Tensor | bool | None = True,
                 best_key: torch.Tensor | None = None):
        """Score free-t_mid templates (generated from gen, or the given [n][7] int32 tracks): (snr, best_key)."""
        if tracks is not None:
            if tracks.dtype != torch.int32 or tracks.dim() != 2 or tracks.shape[1] != 7 or not tracks.is_contiguous():
                raise ValueError("tracks must be a contiguous [n][7] int32 tensor")
            if n is None:
                n = tracks.shape[0]
            if n > tracks.shape[0]:
                raise ValueError("n exceeds the number of given tracks")
        if n is None:
            raise ValueError("n is required with generated tracks")
        if snr is True:
            snr = torch.empty(n, dtype=torch.float32, device=m.Y.device)
        if snr is False:
            snr = None
        if snr is not None and (snr.dtype != torch.float32 or snr.numel() < n or not snr.is_contiguous()):
            raise ValueError("snr must be a contiguous float32 tensor of at least n elements")
        if best_key is None:
            best_key = torch.zeros(1, dtype=torch.int64, device=m.Y.device)
        mc = m.c()
        g = gen.c() if gen is not None else None
        self._chk(self._L.stt_score_tm(self.h, C.byref(mc), C.byref(g) if g is not None else None,
                                       C.c_void_p(tracks.data_ptr()) if tracks is not None else None, first, n,
                                       norm, C.c_void_p(snr.data_ptr()) if snr is not None else None,
                                       C.c_void_p(best_key.data_ptr())))
        return snr, best_key

    def score_maxdelay(self, m: Map, dtau0: int, dtau_step: int, n_tau: int, gen: Gen | None = None,
                       tracks: torch.Tensor | None = None, first: int = 0, n: int | None = None,
                       norm: int = NORM_SQRT_N, snr: torch.Tensor | bool | None = True,
                       tau_idx: torch.Tensor | bool | None = True, best_key: torch.Tensor | None = None):
        """Delay-maximised scores over the grid dtau0 + m*dtau_step (m < n_tau): returns
        (snr or None, maximising delay index or None, best_key), as score() does for one delay."""
        if tracks is not None:
            if tracks.dtype != torch.int32 or tracks.dim() != 2 or tracks.shape[1] != 6 or not tracks.is_contiguous():
                raise ValueError("tracks must be a contiguous [n][6] int32 tensor")
            if n is None:
                n = tracks.shape[0]
            if n > tracks.shape[0]:
                raise ValueError("n exceeds the number of given tracks")
        if n is None:
            raise ValueError("n is required with generated tracks")
        dev = m.Y.device
        if snr is True:
            snr = torch.empty(n, dtype=torch.float32, device=dev)
        if snr is False:
            snr = None
        if snr is not None and (snr.dtype != torch.float32 or snr.numel() < n or not snr.is_contiguous()):
            raise ValueError("snr must be a contiguous float32 tensor of at least n elements")
        if tau_idx is True:
            tau_idx = torch.empty(n, dtype=torch.int32, device=dev)
        if tau_idx is False:
            tau_idx = None
        if tau_idx is not None and (tau_idx.dtype != torch.int32 or tau_idx.numel() < n or not tau_idx.is_contiguous()):
            raise ValueError("tau_idx must be a contiguous int32 tensor of at least n elements")
        if best_key is None:
            best_key = torch.zeros(1, dtype=torch.int64, device=dev)
        mc = m.c()
        g = gen.c() if gen is not None else None
        self._chk(self._L.stt_score_maxdelay(self.h, C.byref(mc), C.byref(g) if g is not None else None,
                                             C.c_void_p(tracks.data_ptr()) if tracks is not None else None,
                                             first, n, dtau0, dtau_step, n_tau, norm,
                                             C.c_void_p(snr.data_ptr()) if snr is not None else None,
                                             C.c_void_p(tau_idx.data_ptr()) if tau_idx is not None else None,
                                             C.c_void_p(best_key.data_ptr())))
        return snr, tau_idx, best_key

    def pack_p16(self, m: Map) -> P16Map:
        """FP16 copy of the map's complex SNR p = Y/sigma in polar form with a per-map 2^e scale
        (synchronises)."""
        out = torch.empty((m.T, m.F, 2), dtype=torch.int16, device=m.Y.device)
        e = C.c_int32()
        mc = m.c()
        self._chk(self._L.stt_map_pack_p16(self.h, C.byref(mc), C.c_void_p(out.data_ptr()), m.F, C.byref(e)))
        return P16Map(out, e.value, m.fq4_lo, m.dfq4)

    def topk(self, snr: torch.Tensor, K: int, first: int = 0, n: int | None = None):
        """(int64 indices, float32 scores) of the K best of snr[0..n), best first."""
        if snr.dtype != torch.float32 or not snr.is_contiguous():
            raise ValueError("snr must be a contiguous float32 tensor")
        n = snr.numel() if n is None else n
        idx = torch.empty(K, dtype=torch.int64, device=snr.device)
        val = torch.empty(K, dtype=torch.float32, device=snr.device)
        self._chk(self._L.stt_topk(self.h, C.c_void_p(snr.data_ptr()), n, first, K, C.c_void_p(idx.data_ptr()),
                                   C.c_void_p(val.data_ptr())))
        return idx, val

    def rescore_f64(self, m: Map, idx: torch.Tensor, gen: Gen | None = None, tracks: torch.Tensor | None = None,
                    first: int = 0, norm: int = NORM_SQRT_N) -> torch.Tensor:
        """FP64 scores of tracks idx (drawn from gen, or tracks[idx - first]) on the FP32 map."""
        if idx.dtype != torch.int64 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 tensor")
        out = torch.empty(idx.numel(), dtype=torch.float64, device=idx.device)
        mc = m.c()
        g = gen.c() if gen is not None else None
        self._chk(self._L.stt_rescore_f64(self.h, C.byref(mc), C.byref(g) if g is not None else None,
                                          C.c_void_p(tracks.data_ptr()) if tracks is not None else None,
                                          tracks.shape[0] if tracks is not None else 0, first,
                                          C.c_void_p(idx.data_ptr()), idx.numel(), norm, C.c_void_p(out.data_ptr())))
        return out

    def autotune(self, m, gen: Gen, n: int, cache_path: str | None = None) -> tuple[int, int, int]:
        """Pick (and apply) the fastest slab shape and LDS budget for this map and call size."""
        out = (C.c_int32 * 3)()
        mc = m.c()
        g = gen.c()
        self._chk(self._L.stt_autotune(self.h, C.byref(mc), C.byref(g), n,
                                       cache_path.encode() if cache_path else None, out))
        return out[0], out[1], out[2]

    def autotune_batch(self, maps, gen: Gen, n_trk, cache_path: str | None = None) -> tuple[int, int, int]:
        """Pick (and apply) the fastest slab shape and LDS budget for this batch of maps (as score_batch)."""
        nm = len(maps)
        if nm < 1 or len(n_trk) != nm:
            raise ValueError("one template count per map, at least one map")
        out = (C.c_int32 * 3)()
        arr = (_Map * nm)(*[m.c() for m in maps])
        ns = (C.c_int64 * nm)(*[int(x) for x in n_trk])
        g = gen.c()
        self._chk(self._L.stt_autotune_batch(self.h, arr, nm, C.byref(g), ns,
                                             cache_path.encode() if cache_path else None, out))
        return out[0], out[1], out[2]

    # -- differentiation
    def tracks_at(self, gen: Gen, T: int, F: int, idx: torch.Tensor) -> torch.Tensor:
        """Templates at the given indices (int64 tensor), as an [n][6] int32 tensor."""
        if idx.dtype != torch.int64 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 tensor")
        out = tracks_tensor(idx.numel(), device=idx.device)
        g = gen.c()
        self._chk(self._L.stt_tracks_at(self.h, C.byref(g), T, F, C.c_void_p(idx.data_ptr()), idx.numel(),
                                        C.c_void_p(out.data_ptr())))
        return out

    def tracks_to_theta(self, tracks: torch.Tensor):
        """(theta [n][6] float32, K [n] int32) of plain templates."""
        n = tracks.shape[0]
        theta = torch.empty((n, 6), dtype=torch.float32, device=tracks.device)
        K = torch.empty(n, dtype=torch.int32, device=tracks.device)
        self._chk(self._L.stt_tracks_to_theta(self.h, C.c_void_p(tracks.data_ptr()), n, C.c_void_p(theta.data_ptr()),
                                              C.c_void_p(K.data_ptr())))
        return theta, K

    @staticmethod
    def _theta_ok(theta, K):
        if theta.dtype != torch.float32 or theta.dim() != 2 or theta.shape[1] != 6 or not theta.is_contiguous():
            raise ValueError("theta must be a contiguous [n][6] float32 tensor")
        if K.dtype != torch.int32 or K.numel() != theta.shape[0] or not K.is_contiguous():
            raise ValueError("K must be a contiguous int32 tensor with one entry per template")

    def smooth(self, m, theta: torch.Tensor, K: torch.Tensor) -> torch.Tensor:
        self._theta_ok(theta, K)
        z = torch.empty(theta.shape[0], dtype=torch.float32, device=theta.device)
        mc = m.c()
        self._chk(self._L.stt_smooth(self.h, C.byref(mc), C.c_void_p(theta.data_ptr()), C.c_void_p(K.data_ptr()),
                                     theta.shape[0], C.c_void_p(z.data_ptr())))
        return z

    def grad(self, m, theta: torch.Tensor, K: torch.Tensor):
        """(z~ [n], dz~/dtheta [n][6]) from the hand-written backward kernel."""
        self._theta_ok(theta, K)
        n = theta.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=theta.device)
        g = torch.empty((n, 6), dtype=torch.float32, device=theta.device)
        mc = m.c()
        self._chk(self._L.stt_grad(self.h, C.byref(mc), C.c_void_p(theta.data_ptr()), C.c_void_p(K.data_ptr()), n,
                                   C.c_void_p(z.data_ptr()), C.c_void_p(g.data_ptr())))
        return z, g

    def refine(self, m, theta: torch.Tensor, K: torch.Tensor, min_len: int, dtau_max: int, steps: int = 50,
               sched=(1.0, 0.02, 0.5, 0.01), norm: int = NORM_SQRT_N, plain: bool = True):
        """Projected ascent of z~ from theta (copied). Returns (best theta, its z~, plain templates, their z)."""
        self._theta_ok(theta, K)
        n = theta.shape[0]
        th = theta.clone()
        zs = torch.empty(n, dtype=torch.float32, device=theta.device)
        tr = tracks_tensor(n, device=theta.device) if plain else None
        zp = torch.empty(n, dtype=torch.float32, device=theta.device) if plain else None
        sc = (C.c_float * 4)(*sched)
        mc = m.c()
        self._chk(self._L.stt_refine(self.h, C.byref(mc), min_len, dtau_max, C.c_void_p(th.data_ptr()),
                                     C.c_void_p(K.data_ptr()), n, steps, sc, C.c_void_p(zs.data_ptr()),
                                     C.c_void_p(tr.data_ptr()) if plain else None,
                                     C.c_void_p(zp.data_ptr()) if plain else None, norm))
        return th, zs, tr, zp

    def set_graph(self, on: bool):
        self._chk(self._L.stt_set_graph(self.h, 1 if on else 0))

    def score_batch(self, maps, gen: Gen, n_trk, norm: int = NORM_SQRT_N, best_keys: torch.Tensor | None = None,
                    snr=None) -> torch.Tensor:
        """Score n_trk[m] templates on each map m (Philox stream gen.stream + m) in one launch.

        Returns the [n_maps] int64 best-key tensor (max-merged into ``best_keys`` when given).
        ``snr`` is None or a list of per-map float32 tensors (entries may be None).
        """
        nm = len(maps)
        if len(n_trk) != nm:
            raise ValueError("one template count per map")
        dev = maps[0].Y.device if nm else torch.device("cuda")
        if best_keys is None:
            best_keys = torch.zeros(nm, dtype=torch.int64, device=dev)
        if best_keys.dtype != torch.int64 or best_keys.numel() < nm or not best_keys.is_contiguous():
            raise ValueError("best_keys must be a contiguous int64 tensor with one entry per map")
        arr = (_Map * max(nm, 1))(*[m.c() for m in maps])
        ns = (C.c_int64 * max(nm, 1))(*[int(x) for x in n_trk])
        ptrs = None
        if snr is not None:
            if len(snr) != nm:
                raise ValueError("one snr entry per map")
            for t, n in zip(snr, n_trk):
                if t is not None and (t.dtype != torch.float32 or t.numel() < n or not t.is_contiguous()):
                    raise ValueError("snr tensors must be contiguous float32 with n_trk elements")
            ptrs = (C.c_void_p * max(nm, 1))(*[t.data_ptr() if t is not None else None for t in snr])
        g = gen.c()
        self._chk(self._L.stt_score_batch(self.h, arr, nm, C.byref(g), ns, norm, C.c_void_p(best_keys.data_ptr()),
                                          ptrs))
        return best_keys

    # -- significance
    def significance(self, bg_keys: torch.Tensor, fg_keys: torch.Tensor | None = None, alpha: float = 1e-3):
        """(n_louder int64 [n_fg], fap float32 [n_fg], z_alpha float32 [1]) of foreground best keys
        against background best keys (one per map); z_alpha is None when alpha is None."""
        for t in (bg_keys, fg_keys):
            if t is not None and (t.dtype != torch.int64 or not t.is_contiguous() or not t.is_cuda):
                raise ValueError("keys must be contiguous int64 CUDA tensors")
        n_fg = 0 if fg_keys is None else fg_keys.numel()
        dev = bg_keys.device
        cnt = torch.empty(n_fg, dtype=torch.int64, device=dev)
        fap = torch.empty(n_fg, dtype=torch.float32, device=dev)
        za = torch.empty(1, dtype=torch.float32, device=dev) if alpha is not None else None
        self._chk(self._L.stt_significance(
            self.h, C.c_void_p(bg_keys.data_ptr()), bg_keys.numel(),
            C.c_void_p(fg_keys.data_ptr()) if n_fg else None, n_fg, float(alpha or 0.0),
            C.c_void_p(cnt.data_ptr()) if n_fg else None, C.c_void_p(fap.data_ptr()) if n_fg else None,
            C.c_void_p(za.data_ptr()) if za is not None else None))
        return cnt, fap, za

    def follow_up(self, maps, keys: torch.Tensor, gen: Gen, n_deep: int, k: int = 10,
                  norm: int = NORM_SQRT_N) -> list[int]:
        """stt_follow_up: search the maps of rank <= k again with n_deep templates drawn with
        ``gen`` (Philox stream gen.stream + m) and max-merge into ``keys`` in place (Sec. V).
        Returns the indices of the maps searched."""
        if keys.dtype != torch.int64 or keys.numel() != len(maps) or not keys.is_contiguous() or not keys.is_cuda:
            raise ValueError("one int64 CUDA key per map")
        nm = len(maps)
        arr = (_Map * max(nm, 1))(*[m.c() for m in maps])
        chosen = (C.c_int32 * max(nm, 1))()
        n_chosen = C.c_int32(0)
        g = gen.c()
        self._chk(self._L.stt_follow_up(self.h, arr, nm, C.c_void_p(keys.data_ptr()), C.byref(g), int(n_deep), int(k),
                                        norm, chosen, C.byref(n_chosen)))
        return [int(chosen[i]) for i in range(n_chosen.value)]

    # -- map formation
    def spectra(self, strain: torch.Tensor, p: Spectro, T: int | None = None, spec: torch.Tensor | None = None,
                psd: torch.Tensor | None = None) -> tuple[torch.Tensor, torch.Tensor]:
        """Column spectra s~ (complex64 [T][F]) and P' (float32 [T][F]) of one detector's strain."""
        if strain.dtype != torch.float32 or not strain.is_cuda or not strain.is_contiguous():
            raise ValueError("strain must be a contiguous float32 CUDA tensor")
        n = strain.numel()
        if T is None:
            T = p.n_columns(n)
        dev = strain.device
        if spec is None:
            spec = torch.empty((T, p.F), dtype=torch.complex64, device=dev)
        if psd is None:
            psd = torch.empty((T, p.F), dtype=torch.float32, device=dev)
        for t, dt in ((spec, torch.complex64), (psd, torch.float32)):
            if t.dtype != dt or tuple(t.shape) != (T, p.F) or not t.is_contiguous():
                raise ValueError("spec / psd must be contiguous [T][F] complex64 / float32")
        pc = p.c()
        self._chk(self._L.stt_spectra(self.h, C.byref(pc), C.c_void_p(strain.data_ptr()), n, T,
                                      C.c_void_p(spec.data_ptr()), C.c_void_p(psd.data_ptr())))
        return spec, psd

    def form_maps(self, p: Spectro, spec_i: torch.Tensor, psd_i: torch.Tensor, spec_j: torch.Tensor,
                  psd_j: torch.Tensor, shifts, ld: int | None = None, out: list | None = None) -> list:
        """One Map per time slide: column t of I against column (t + shift) mod T of J.

        ``out`` may give the Maps to write (same T, F; reused across calls); otherwise new
        [T][ld] buffers are allocated (ld defaults to F)."""
        T = spec_i.shape[0]
        for t, dt in ((spec_i, torch.complex64), (spec_j, torch.complex64), (psd_i, torch.float32),
                      (psd_j, torch.float32)):
            if t.dtype != dt or tuple(t.shape) != (T, p.F) or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("spectra and P' must be contiguous [T][F] CUDA tensors of one shape")
        shifts = [int(x) for x in shifts]
        fq4_lo, dfq4 = p.fq4()
        if out is None:
            ld = p.F if ld is None else ld
            out = []
            for _ in shifts:
                Y = torch.empty((T, ld), dtype=torch.complex64, device=spec_i.device)[:, :p.F]
                sg = torch.empty((T, ld), dtype=torch.float32, device=spec_i.device)[:, :p.F]
                out.append(Map(Y, sg, fq4_lo, dfq4))
        if len(out) != len(shifts):
            raise ValueError("one output map per shift")
        for m in out:
            if (m.T, m.F) != (T, p.F) or m.ld != out[0].ld:
                raise ValueError("output maps must be [T][F] with one column stride")
        ns = len(shifts)
        sh = (C.c_int32 * max(ns, 1))(*shifts)
        yp = (C.c_void_p * max(ns, 1))(*[m.Y.data_ptr() for m in out])
        sp = (C.c_void_p * max(ns, 1))(*[m.sigma.data_ptr() for m in out])
        pc = p.c()
        self._chk(self._L.stt_form_maps(self.h, C.byref(pc), T, C.c_void_p(spec_i.data_ptr()),
                                        C.c_void_p(psd_i.data_ptr()), C.c_void_p(spec_j.data_ptr()),
                                        C.c_void_p(psd_j.data_ptr()), ns, sh, out[0].ld if out else p.F, yp, sp))
        return out

    def argmax(self, snr: torch.Tensor, first: int = 0, best_key: torch.Tensor | None = None) -> torch.Tensor:
        if snr.dtype != torch.float32 or not snr.is_contiguous():
            raise ValueError("snr must be a contiguous float32 tensor")
        if best_key is None:
            best_key = torch.zeros(1, dtype=torch.int64, device=snr.device)
        self._chk(self._L.stt_argmax(self.h, C.c_void_p(snr.data_ptr()), snr.numel(), first,
                                     C.c_void_p(best_key.data_ptr())))
        return best_key


def decode_best(best_key: torch.Tensor) -> tuple[float, int]:
    """(score, track index) of a best-key tensor (synchronises)."""
    return key_decode(int(best_key.item()) & 0xFFFFFFFFFFFFFFFF)
