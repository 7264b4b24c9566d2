"""The probe library behind the roofline's measured ceilings (issue rates, streaming reads, LDS
reads): it loads and exports its entry points on the CPU; on a GPU each probe returns plausible
rates."""
from __future__ import annotations

import ctypes as C
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = os.path.join(ROOT, "paper_1401_8060_amd", "libstt_probe.so")
SYMBOLS = ("stt_probe_count", "stt_probe_name", "stt_probe_issue", "stt_probe_stream", "stt_probe_lds")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(PROBE):
        pytest.skip("libstt_probe.so not built")
    L = C.CDLL(PROBE)
    L.stt_probe_name.restype = C.c_char_p
    L.stt_probe_issue.argtypes = [C.c_int, C.c_int, C.c_int] + [C.POINTER(C.c_double)] * 3
    L.stt_probe_stream.argtypes = [C.c_int, C.c_int64, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.stt_probe_lds.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    return L


def test_probe_library_exports(lib):
    for s in SYMBOLS:
        assert hasattr(lib, s), s
    n = lib.stt_probe_count()
    assert n >= 10
    names = [lib.stt_probe_name(i).decode() for i in range(n)]
    assert "v_cos_f32" in names and "v_fma_f64" in names and lib.stt_probe_name(n).decode() == "?"


def test_probe_arguments_rejected_before_any_gpu_call(lib):
    d1, d2, d3 = C.c_double(), C.c_double(), C.c_double()
    assert lib.stt_probe_issue(0, -1, 16, C.byref(d1), C.byref(d2), C.byref(d3)) == -1
    assert lib.stt_probe_stream(0, 15, 1, C.byref(d1), C.byref(d2)) == -1
    assert lib.stt_probe_stream(0, 1 << 20, 0, C.byref(d1), C.byref(d2)) == -1
    assert lib.stt_probe_lds(0, 1, 0, C.byref(d1), C.byref(d2)) == -1


@pytest.mark.gpu
def test_probes_measure_plausible_rates(lib):
    r, f, ms = C.c_double(), C.c_double(), C.c_double()
    assert lib.stt_probe_issue(0, 0, 256, C.byref(r), C.byref(f), C.byref(ms)) == 0
    assert 8.0 < r.value < 512.0 and 500.0 < f.value < 4000.0  # lanes per clock per CU; MHz
    g = C.c_double()
    assert lib.stt_probe_stream(0, 8 << 20, 4, C.byref(g), C.byref(ms)) == 0
    assert 100.0 < g.value < 200_000.0  # GB/s
    lds = {}
    for rnd in (0, 1):
        assert lib.stt_probe_lds(0, rnd, 64, C.byref(g), C.byref(ms)) == 0
        lds[rnd] = g.value
    assert 100.0 < lds[1] <= 1.2 * lds[0]  # random rows never beat conflict-free ones by much
