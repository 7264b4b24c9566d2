"""bench.py's output line on the GPU: a small workload through the real command line, and the
one-JSON-line contract (metric, value, step timing, roofline with its derivation, the
non-binding lines and the argmax-only leg) checked field by field."""
from __future__ import annotations

import json
import math
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout  # exactly one JSON line on stdout
    return json.loads(lines[0])


def test_search_record_contract(tmp_path):
    d = _run("--workload", "plain_100x128_1e4", "--steps", "3", "--warmup", "1", "--no-cpu-baseline",
             "--tune-cache", str(tmp_path / "tune.json"))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["unit"] == "tracks/s" and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert d["config"]["workload"] == "plain_100x128_1e4" and d["config"]["n_tracks"] == 10_000
    assert math.isclose(d["value"], 10_000 / (d["ms_per_step"] * 1e-3), rel_tol=1e-9)
    r = d["roofline"]
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["kernel_ms"] > 0
    # achieved = algorithmic flops / kernel time; frac = achieved / peak; peak from the issue mix
    assert math.isclose(r["achieved"], d["track_px"] * r["flops_per_track_px"] / (r["kernel_ms"] * 1e-3) / 1e12,
                        rel_tol=1e-9)
    assert math.isclose(r["frac"], r["achieved"] / r["peak"], rel_tol=1e-9)
    pd = r["peak_derivation"]
    assert math.isclose(r["peak"], pd["ceiling_px_s"] * r["flops_per_track_px"] / 1e12, rel_tol=1e-9)
    assert {"fp32_flops", "lds_read", "gather_line"} <= set(r["not_binding"])
    assert r["not_binding"]["gather_line"]["peak"] == 8000.0


def test_full_search_record_has_its_traffic_and_argmax_leg():
    """The headline workload in its launch configuration: the committed counter summary matches
    the kernel sources and slab shape, so the record carries measured traffic and the memory-side
    line; the argmax-only leg is timed beside the per-template one."""
    d = _run("--steps", "2", "--warmup", "1", "--no-cpu-baseline")
    assert d["config"]["workload"] == "search_1000x1000_1e7" and d["config"]["per_track_snr"] is True
    r = d["roofline"]
    assert r["traffic"] is not None and r["memory_side"] is not None
    assert 0.0 < r["memory_side"]["frac"] < 2.0 and 0.0 < r["frac"] < 1.0
    a = d["argmax_only"]
    assert a["traffic"] is not None and a["best"] == d["best"]  # the same search, same winner
    assert a["kernel_ms"] > 0 and a["ms_per_step"] > 0
