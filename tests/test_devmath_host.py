"""The kernels' integer arithmetic, compiled for the host, against the CPU oracle.

dev_common.hpp (generator, unranking, exact DDA rasteriser, phase rotation,
key encoding) is __host__ __device__; this suite builds it into a host program
and checks it without a GPU: generated templates and rasterised rows must be
bit-exact with the oracle, the phase rotation within its polynomial bound.
"""
from __future__ import annotations

import math
import os
import shutil
import struct
import subprocess

from fractions import Fraction

import numpy as np
import pytest

D10MS = 2684355  # 10 ms in 2^-28 s units

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_devmath(tmp_path_factory, defines=()):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("devmath") / "devmath"
    src = os.path.join(ROOT, "tests", "helpers", "devmath_host.cpp")
    subprocess.run([hipcc, "-O2", "-x", "hip", "--offload-arch=gfx950", "-w", *[f"-D{d}" for d in defines],
                    "-I", os.path.join(ROOT, "paper_1401_8060_amd", "csrc"), src, "-o", str(out)],
                   check=True, capture_output=True)

    def run(lines):
        r = subprocess.run([str(out)], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        return r.stdout.strip().split("\n")
    return run


@pytest.fixture(scope="module")
def devmath(tmp_path_factory):
    return _build_devmath(tmp_path_factory)


@pytest.fixture(scope="module")
def devmath_ulp(tmp_path_factory):
    """The same harness with every FP32 square root and reciprocal of the free-t_mid rows moved by
    one ulp (a harsher error than the hardware's)."""
    return _build_devmath(tmp_path_factory, ["STT_HOST_ULP_PERTURB"])


def test_generated_templates_bit_exact(orc, devmath):
    cases = []
    sel = np.random.default_rng(99)
    for (T, F, L, D) in [(100, 128, 10, 2684355), (1000, 1000, 10, 2684355), (2896, 32767, 2, (1 << 30) - 1),
                         (12, 4, 10, 0), (10, 1, 10, 5), (500, 151, 70, 2684355), (2000, 2000, 10, 1)]:
        for j in list(range(40)) + sel.integers(0, 2 ** 32 - 1, 40).tolist():
            seed = int(sel.integers(0, 2 ** 64 - 1, dtype=np.uint64))
            stream = int(sel.integers(0, 2 ** 32 - 1))
            cases.append((seed, stream, int(j), T, F, L, D))
    out = devmath([f"draw {s} {st} {j} {T} {F} {L} {D}" for (s, st, j, T, F, L, D) in cases])
    for c, line in zip(cases, out):
        want = orc.draw(*c).tolist()
        assert tuple(int(x) for x in line.split()) == tuple(int(x) for x in want), c


def test_dda_rows_bit_exact(orc, devmath):
    sel = np.random.default_rng(7)
    cases = []
    for _ in range(3000):
        F = int(sel.choice([1, 2, 3, 128, 1000, 2000, 32767]))
        Dt = int(sel.choice([1, 2, 3, 9, 99, 999, 1999, 2895]))
        f = sel.integers(0, F * 256, size=3)
        cases.append((0, Dt, int(f[0]), int(f[1]), int(f[2]), F))
    # extremes: corners of the frequency range, longest tracks
    for F in (1, 1000, 32767):
        hi = F * 256 - 1
        for Dt in (1, 2895):
            for f in [(0, 0, 0), (hi, hi, hi), (0, hi, 0), (hi, 0, hi), (0, hi, hi), (hi, 0, 0), (0, 0, hi)]:
                cases.append((5, 5 + Dt, *f, F))
    out = devmath([f"rows {a} {b} {c} {d} {e}" for (a, b, c, d, e, F) in cases])
    for c, line in zip(cases, out):
        got = [int(x) for x in line.split()]
        want = orc.rows(np.array(c[:5] + (0,), dtype=orc.TRACK_DTYPE), c[5]).tolist()
        assert got == want, c


def test_rewound_dda_reaches_exact_rows(orc, devmath):
    """Starting the DDA up to a whole map before the template (as the slab scorer
    does for the first column of a wave) still gives the exact rows."""
    sel = np.random.default_rng(8)
    cases = []
    for _ in range(2000):
        F = int(sel.choice([1, 7, 1000, 32767]))
        Dt = int(sel.choice([1, 2, 5, 64, 999, 2895]))
        k0 = -int(sel.choice([0, 1, 15, 63, 500, 2895]))
        f = sel.integers(0, F * 256, size=3)
        cases.append((0, Dt, int(f[0]), int(f[1]), int(f[2]), k0, F))
    out = devmath([f"rowsat {a} {b} {c} {d} {e} {k}" for (a, b, c, d, e, k, F) in cases])
    for c, line in zip(cases, out):
        got = [int(x) for x in line.split()]
        want = orc.rows(np.array(c[:5] + (0,), dtype=orc.TRACK_DTYPE), c[6]).tolist()
        assert got == want, c


@pytest.mark.parametrize("cmd", ["rowsat", "rowsf"])
def test_rewound_walks_exhaustive_short_tracks(orc, devmath, cmd):
    """Every control-frequency triple on a 1/32-row grid of a 3-row band, every
    length up to 6 and rewinds of 0..3 columns: both walks equal the oracle's rows."""
    F = 3
    grid = list(range(0, F * 256, 8)) + [F * 256 - 1]
    cases = []
    for Dt in range(1, 7):
        for f0 in grid[::3]:
            for f1 in grid[::5]:
                for f2 in grid[::7]:
                    cases.append((0, Dt, f0, f1, f2, -(Dt % 4)))
    out = devmath([f"{cmd} {a} {b} {c} {d} {e} {k}" for (a, b, c, d, e, k) in cases])
    for c, line in zip(cases, out):
        want = orc.rows(np.array(c[:5] + (0,), dtype=orc.TRACK_DTYPE), F).tolist()
        assert [int(x) for x in line.split()] == want, c


def test_fp64_walk_bit_exact_random(orc, devmath):
    sel = np.random.default_rng(11)
    cases = []
    for _ in range(3000):
        F = int(sel.choice([1, 2, 7, 1000, 2000, 32767]))
        Dt = int(sel.choice([1, 2, 5, 64, 999, 1999, 2895]))
        k0 = -int(sel.choice([0, 1, 15, 63, 500, 2895]))
        f = sel.integers(0, F * 256, size=3)
        cases.append((0, Dt, int(f[0]), int(f[1]), int(f[2]), k0, F))
    for F in (1, 1000, 32767):
        hi = F * 256 - 1
        for Dt in (1, 2, 2895):
            for f in [(0, 0, 0), (hi, hi, hi), (0, hi, 0), (hi, 0, hi), (0, hi, hi), (hi, 0, 0), (0, 0, hi)]:
                for k0 in (0, -2895):
                    cases.append((0, Dt, *f, k0, F))
    out = devmath([f"rowsf {a} {b} {c} {d} {e} {k}" for (a, b, c, d, e, k, F) in cases])
    for c, line in zip(cases, out):
        got = [int(x) for x in line.split()]
        want = orc.rows(np.array(c[:5] + (0,), dtype=orc.TRACK_DTYPE), c[6]).tolist()
        assert got == want, c


def test_phase_rotation_accuracy(devmath):
    sel = np.random.default_rng(3)
    ph = sel.integers(0, 2 ** 32, 20000).tolist() + [0, 2 ** 30, 2 ** 31, 3 * 2 ** 30, 2 ** 32 - 1,
                                                     2 ** 30 - 1, 2 ** 30 + 1, 2 ** 31 - 1]
    pr = sel.standard_normal(len(ph)).astype(np.float32)
    pi = sel.standard_normal(len(ph)).astype(np.float32)
    out = devmath([f"rot {a} {float(b):.9e} {float(c):.9e}" for a, b, c in zip(ph, pr, pi)])
    got = np.array([float(x) for x in out])
    turns = np.array([((a + 2 ** 31) % 2 ** 32 - 2 ** 31) / 2 ** 32 for a in ph])
    want = np.cos(2 * np.pi * turns) * pr.astype(np.float64) - np.sin(2 * np.pi * turns) * pi.astype(np.float64)
    err = np.abs(got - want) / np.maximum(1.0, np.abs(pr) + np.abs(pi))
    assert err.max() < 5e-7


def test_phase_argument(devmath):
    """The scorers' sine/cosine argument is the Eq. 8 phase f*dtau in turns, f = (fq4_lo + row*dfq4)/16 Hz
    and dtau in 2^-28 s, as an FP32 number in [1, 2) equal to the phase mod 1 rounded to 23 fractional
    bits: within 2^-24 turn of the exact value (mod 1), checked against rational arithmetic."""
    sel = np.random.default_rng(21)
    cases = []
    for _ in range(20000):
        cases.append((int(sel.integers(0, 2 ** 20)), int(sel.integers(1, 2 ** 8)),
                      int(sel.integers(-(2 ** 30) + 1, 2 ** 30)), int(sel.integers(0, 2 ** 15))))
    cases += [(1600, 16, 2684355, 32766), (1048575, 255, -1073741823, 32767), (0, 1, 0, 0), (1600, 16, 1 << 27, 1)]
    got = devmath([f"phx {a} {b} {c} {d}" for a, b, c, d in cases])
    for (fq4, dfq, dtau, row), g in zip(cases, got):
        exact = Fraction((fq4 + row * dfq) * dtau, 2 ** 32)  # (fq4/16 Hz)(dtau 2^-28 s) turns
        err = (Fraction(float(np.float32(g))) - exact) % 1  # the printed FP32 value, read back exactly
        err = min(err, 1 - err)
        assert err <= Fraction(1, 2 ** 24), (fq4, dfq, dtau, row, g)
        assert 1.0 <= float(g) < 2.0


def test_key_order_and_special_values(devmath):
    zs = [-math.inf, -3.5, -1e-30, -0.0, 0.0, 1e-30, 2.0, 2.0, math.inf, math.nan]
    js = [5, 4, 3, 2, 1, 9, 7, 6, 0, 8]
    keys = [int(x, 16) for x in devmath([f"key {z!r} {j}" for z, j in zip(zs, js)])]
    assert all(k > 0 for k in keys)
    assert keys[3] >> 32 == keys[4] >> 32  # -0 and +0 share the score bits
    # score order, then lower index first
    assert keys[0] < keys[1] < keys[2] < keys[3] < keys[4]
    assert keys[4] < keys[5] < keys[6] < keys[7] < keys[8]
    assert keys[9] >> 32 == keys[0] >> 32  # NaN counts as -inf


def test_free_tmid_draw_bit_exact(orc, devmath):
    """draw_track_tm (the kernels' generator of free-t_mid templates) against the oracle's."""
    T, F, L = 700, 300, 10
    want = orc.draw_tm_many(21, 4, 1000, 3000, T, F, L, D10MS)
    got = devmath([f"drawtm 21 4 {1000 + i} {T} {F} {L} {D10MS}" for i in range(3000)])
    assert [tuple(int(x) for x in g.split()) for g in got] == [tuple(int(v) for v in w) for w in want.tolist()]


@pytest.mark.parametrize("mode", ["rounded", "one_ulp_off"])
def test_free_tmid_rows_bit_exact(orc, devmath, devmath_ulp, mode):
    """row_tm (an FP32 pass within a certified window, else FP64 with the exact fallback) against
    the oracle's exact integer rows: random templates over the full size range, every t1 of small
    templates, and control frequencies on row boundaries (where the fallbacks decide); once with
    correctly rounded FP32 square roots and reciprocals and once with each moved by one ulp."""
    run = devmath if mode == "rounded" else devmath_ulp
    rng = np.random.default_rng(41)
    cases = []
    F = 32767
    for _ in range(400):
        T = int(rng.integers(2, 2897))
        t0 = int(rng.integers(0, T - 1))
        t2 = int(rng.integers(t0 + 1, T))
        cases.append((t0, int(rng.integers(t0, t2 + 1)), t2, *[int(x) for x in rng.integers(0, F * 256, 3)]))
    for t0, t2 in [(0, 1), (3, 9), (0, 40), (100, 131)]:
        for t1 in range(t0, t2 + 1):
            cases.append((t0, t1, t2, 256 * int(rng.integers(0, 50)), 256 * int(rng.integers(0, 50)),
                          256 * int(rng.integers(0, 50))))
            cases.append((t0, t1, t2, *[int(x) for x in rng.integers(0, 50 * 256, 3)]))
    cases += [(0, 0, 2895, 0, F * 256 - 1, 0), (0, 2895, 2895, F * 256 - 1, 0, F * 256 - 1),
              (7, 7, 2000, 12345, 12345, 12345)]
    for _ in range(400):  # the search maps' band, F = 1000
        t0 = int(rng.integers(0, 999))
        t2 = int(rng.integers(t0 + 1, 1000))
        cases.append((t0, int(rng.integers(t0, t2 + 1)), t2, *[int(x) for x in rng.integers(0, 1000 * 256, 3)]))
    got = run([f"rowstm {' '.join(str(v) for v in c)}" for c in cases])
    for c, g in zip(cases, got):
        tr = np.array([c + (0,)], dtype=orc.TRACK_TM_DTYPE)
        assert [int(x) for x in g.split()] == orc.rows_tm(tr, F).tolist(), c


def test_free_tmid_fp32_pass_mostly_stands(devmath):
    """On the search maps' band (F = 1000) the FP32 pass decides almost every column: the exact
    path runs for under 1 % of them."""
    rng = np.random.default_rng(42)
    cases = []
    for _ in range(300):
        t0 = int(rng.integers(0, 900))
        t2 = int(rng.integers(t0 + 50, 1000))
        cases.append((t0, int(rng.integers(t0, t2 + 1)), t2, *[int(x) for x in rng.integers(0, 1000 * 256, 3)]))
    got = devmath([f"tmstat {' '.join(str(v) for v in c)}" for c in cases])
    fb = sum(int(g.split()[0]) for g in got)
    cols = sum(c[2] - c[0] for c in cases)
    assert fb / cols < 0.01, (fb, cols)


@pytest.mark.parametrize("mode", ["rounded", "one_ulp_off"])
def test_free_tmid_fp32_error_inside_window(devmath, devmath_ulp, mode):
    """The FP32 pass's actual error against an FP64 evaluation stays well inside its certified
    window on every column of random templates (both bands, all shapes of t1), also when each
    square root and reciprocal is one ulp off."""
    run = devmath if mode == "rounded" else devmath_ulp
    rng = np.random.default_rng(43)
    cases = []
    for F, T in ((1000, 1000), (32767, 2896), (151, 500)):
        for _ in range(250):
            t0 = int(rng.integers(0, T - 1))
            t2 = int(rng.integers(t0 + 1, T))
            t1 = int(rng.choice([t0, t2, int(rng.integers(t0, t2 + 1))]))
            cases.append((t0, t1, t2, *[int(x) for x in rng.integers(0, F * 256, 3)]))
    worst = max(float(w) for w in run([f"tmerr {' '.join(str(v) for v in c)}" for c in cases]))
    assert worst < 0.8, worst
