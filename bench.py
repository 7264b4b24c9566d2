#!/usr/bin/env python3
"""Throughput of the template search on one MI355X.

Default workload (the one the headline metric is quoted on): a step is one
pass of the whole hot path on the search-scale map -- generate 10^7 random
quadratic-Bezier templates (Philox), bin them by time extent, score every one
on a T=1000 x F=1000 complex64 map (log-uniform sigma, one injected track at
SNR 8) with the random-phase-factor statistic, write the per-track SNRs and
reduce to the max/argmax key. The map is resident in HBM before the timed
region. Other workloads (--workload) measure the batched, FP16 and small
configurations; each prints one JSON line of the same form.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Bézier tracks scored/sec per MI355X (track-pixels/s, % gather roofline)"
HBM_PEAK_GBS = 8000.0
TUNE_CACHE = os.path.join(ROOT, "paper_1401_8060_amd", "tuning", "gfx950.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1401_8060_amd", "csrc", f) for f in ("kernels.hpp", "dev_common.hpp")]
MAPFORM_SOURCES = [os.path.join(ROOT, "paper_1401_8060_amd", "csrc", "mapform.hpp")]
BYTES_F32 = 12  # complex64 Y + float32 sigma: the caller's pixel record of one template pixel
BYTES_P16 = 4   # one 32-bit polar word of an FP16 map

# ---- the roofline: vector-ALU issue, from gfx950's unit counts and clock -----------------------
# 256 CUs, each 4 SIMDs of 16 lanes; per clock a CU completes 64 lanes of a full-rate instruction
# (FP64 add and FMA, 32-bit integer multiply and three-operand add, shift-add, funnel shift, FP32
# with a 16-bit operand), 128 lanes of an FP32 FMA or add or a 32-bit integer add, 32 lanes of a
# transcendental (sine, cosine, square root, reciprocal). The probe library measures these rates
# at the live shader clock (bench.py --issue-rates; profiles/issue_rates_gfx950.md): 60-61, 103-114
# and 31 lanes per clock per CU.
N_CU, CLOCK_HZ = 256, 2.4e9
LANES_PER_CLK = {"full": 64, "double": 128, "trans": 32}
FP32_PEAK_TFLOPS = 157.3              # 256 x 128 lanes x 2 flops x 2.4 GHz
# Memory-side ceilings measured by the probe library (bench.py --mem-rates;
# profiles/memory_rates_gfx950.md): 8-byte LDS reads at random rows, as the scorers' gathers (the
# conflict-free rate, about twice that, is a lower bound of the LDS peak), and streaming reads of
# buffers beyond the 32 MB of L2 -- 6.5-7.2 TB/s up to 192 MB (the MALL), 6.1-6.5 TB/s from HBM.
LDS_RANDOM_GBS = 51000.0
FAR_READ_GBS = 6800.0
# Instructions of the inner loop per template pixel (one template, one column), by issue class:
#   plain scorer, FP32 map (polar fold): the row of Eq. 6 by the exact FP64 recurrence (1 FMA,
#   2 adds), its LDS address (shift-add), the phase of Eq. 8 plus arg p (integer multiply, add3),
#   the phase as FP32 turns (funnel shift): 7 full-rate; the cosine: 1 transcendental; the term's
#   FMA: 1 double-rate. FP16 map: the term takes its binary16 magnitude in a mixed FMA (full rate).
CORE_MIX = {"full": 7, "double": 1, "trans": 1}
CORE_MIX_P16 = {"full": 8, "double": 0, "trans": 1}
#   free t_mid: the row is an independent root per column -- D = b^2 + 4 a dt and 2 dt carried by
#   one add each (2 double), D as FP32 (full), square root and reciprocal of the reduced root
#   2 dt / (b + sqrt(D)) (2 transcendental; its add, multiply and the two FMAs of the Bezier value:
#   4 double), the fraction, truncation and certified-window test (fraction, convert, compare: 3
#   full; subtract: 1 double); then the plain term (address, phase, turns: 4 full; cosine; FMA).
CORE_MIX_TM = {"full": 8, "double": 8, "trans": 3}
#   delay grid, per template pixel of one launch of 8 delays: row and address (4 full); first
#   delay's phase (3 full), sine and cosine; the grid step's phase (3 full), sine and cosine; 7
#   rotations of (cos, sin) (4 double each) and 8 term FMAs (double).
CORE_MIX_MD = {"full": 10, "double": 36, "trans": 4}
# Algorithmic flops per template pixel (the statistic of Eq. 8 as counted for this path: about 6
# FP32 flops and one sine-cosine pair, each of sine and cosine counted as one).
FLOPS_PER_TRACK_PX = 8


def issue_ceiling_px_s(mix):
    """Template pixels per second at which `mix` keeps every SIMD issuing (unit counts x clock)."""
    return N_CU * CLOCK_HZ / sum(n / LANES_PER_CLK[k] for k, n in mix.items() if n)


WORKLOADS = {
    # search-scale plain map: T=1000 x F=1000, 1 s x 1 Hz pixels from 100 Hz, 10^7 tracks, FP32
    "search_1000x1000_1e7": dict(kind="single", T=1000, F=1000, n=10_000_000, seed=2, L=10, dtau_s=0.01,
                                 sigma=("loguniform", 0.5, 2.0), inject=(200, 799, 250.5, 600.25, 450.75)),
    # the paper's Table III shape (151 Hz x 250 s at 1 s x 1 Hz with 50% overlap -> 500 columns),
    # t_min 35 s of ADI 1 at the 0.5 s column stride -> 70 columns, 2 x 10^7 templates
    "paper_table3_151x500_2e7": dict(kind="single", T=500, F=151, n=20_000_000, seed=3, L=70, dtau_s=0.01,
                                     sigma=("loguniform", 0.5, 2.0), inject=None),
    # small plain map: T=100 x F=128, sigma = 1, 10^4 tracks, Philox seed 1 (latency-bound)
    "plain_100x128_1e4": dict(kind="single", T=100, F=128, n=10_000, seed=1, L=10, dtau_s=0.01, sigma="unit",
                              inject=None),
    # batched background: 256 maps, T uniform on [500, 2000], F=1000, 10^6 tracks per map, one graph launch
    "batch_256maps_1e6": dict(kind="batch", n_maps=256, T_lo=500, T_hi=2000, F=1000, n=1_000_000, seed=3, L=10,
                              dtau_s=0.01, sigma=("loguniform", 0.5, 2.0)),
    # differentiation: T=1000 x F=1000 with 8 injected tracks at SNR 5..10; top-1024 of 10^6 refined 50 steps
    "refine_1000x1000_1e6": dict(kind="refine", T=1000, F=1000, n=1_000_000, seed=5, L=10, dtau_s=0.01,
                                 sigma=("loguniform", 0.5, 2.0), K=1024, steps=50, n_inj=8, inject=None),
    # free t_mid: the search map, 10^7 templates with all six random numbers (t1 anywhere in [t0, t2])
    "tmid_1000x1000_1e7": dict(kind="tmid", T=1000, F=1000, n=10_000_000, seed=2, L=10, dtau_s=0.01,
                               sigma=("loguniform", 0.5, 2.0), inject=(200, 799, 250.5, 600.25, 450.75)),
    # delay-maximised: the search map, 10^6 templates each maximised over 16 delays spanning +-10 ms
    "maxdelay_1000x1000_1e6x16": dict(kind="maxdelay", T=1000, F=1000, n=1_000_000, seed=2, L=10, dtau_s=0.01,
                                      sigma=("loguniform", 0.5, 2.0), n_tau=16,
                                      inject=(200, 799, 250.5, 600.25, 450.75)),
    # map formation: two detectors' strain, 500.5 s at 4096 Hz (white noise plus a chirp reaching J 3 ms
    # after I), columns of 1 s overlapping by half -> T=1000, 100-1099 Hz -> F=1000, P' from 4 columns a
    # side; 256 time slides of J by 2k columns, i.e. 256 background maps of 1000 x 1000
    "mapform_1000x1000_256slides": dict(kind="mapform", fs=4096.0, M=4096, T=1000, k_lo=100, F=1000, nb=4,
                                        n_slides=256, slide_cols=2, seed=6,
                                        chirp=dict(f0=250.0, rate=1.0, amp=0.02, t0=100.0, t1=400.0, delay=0.003)),
    # the background pipeline around the search: strain as for map formation (the chirp at 0.05) -> 256 slide maps
    # (zero lag + 255 background) -> 10^6 templates per map in one batch -> FAP of the zero-lag maximum
    # against the 255 background maxima -> follow-up of the 10 loudest maps with 10^7 templates each
    "background_256slides_1e6": dict(kind="background", fs=4096.0, M=4096, T=1000, k_lo=100, F=1000, nb=4,
                                      n_slides=256, slide_cols=2, seed=6, n=1_000_000, L=10, dtau_s=0.01,
                                      alpha=1e-3, n_deep=10_000_000, k_follow=10,
                                      chirp=dict(f0=250.0, rate=1.0, amp=0.05, t0=100.0, t1=400.0, delay=0.003)),
    # precision: T=2000 x F=2000 stored in FP16, 10^8 tracks, top-1024 re-scored in FP64
    "precision_2000x2000_1e8": dict(kind="precision", T=2000, F=2000, n=100_000_000, seed=4, L=10, dtau_s=0.01,
                                    sigma=("loguniform", 0.5, 2.0), K=1024,
                                    inject=(150, 1799, 500.5, 1500.25, 900.75)),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_map(w, stream=0, T=None):
    import synth
    T = T or w["T"]
    Y, s = synth.noise_map(T, w["F"], seed=1000 + w["seed"], sigma=w["sigma"], stream=stream)
    if w.get("inject"):
        cols, rows = synth.bezier_rows_float(*w["inject"])
        dt0 = int(round(0.003 / 2.0 ** -28))
        synth.add_pixels(Y, s, cols, rows, 8.0 / math.sqrt(cols.size), -((100.0 + rows) * dt0 * 2.0 ** -28))
    return Y, s, synth.map_sha256(Y, s)


def count_px(ctx, g, T, F, n):
    """Exact track-pixel count of templates 0..n-1 (outside any timed region)."""
    px, chunk = 0, 1 << 24
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        tr = ctx.make_tracks(g, T, F, a, b - a)
        px += int((tr[:, 1] - tr[:, 0] + 1).sum().item())
        del tr
    return px


def cpu_baseline(w, Y, s, dtau_max, budget_s=12.0):
    """The oracle (single-threaded FP64 C, unchanged) on the first tracks of the same workload, run
    over disjoint template ranges on every host core this process may use: a calibration pass on
    one thread sizes a sample of about budget_s seconds on all of them."""
    import oracle
    from oracle import shard
    om = oracle.Map(Y, s)
    threads = shard.host_threads()
    n0 = 2000
    t = time.perf_counter()
    oracle.score_gen(om, w["seed"], 0, w["L"], dtau_max, 0, n0)
    dt1 = time.perf_counter() - t
    per_core = n0 / max(dt1, 1e-9)
    n = int(min(w["n"], max(n0, per_core * threads * budget_s)))
    t = time.perf_counter()
    shard.score_gen(om, w["seed"], 0, w["L"], dtau_max, 0, n, threads=threads)
    dt = time.perf_counter() - t
    return dict(value=n / dt, unit="tracks/s", cores=threads, kind="oracle", smt=shard.smt_active(),
                per_core_value=per_core,
                sample=f"first {n} of the {w['n']} tracks of the same map and seed on {threads} threads "
                       f"(one template range each, oracle unchanged), {dt:.1f} s; one thread alone on the "
                       f"first {n0}: {per_core:.3g} tracks/s")


def base_record(args, workload, w, n_tracks, ms_step, px, dtype):
    return {
        "metric": METRIC,
        "value": n_tracks / (ms_step * 1e-3),
        "unit": "tracks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": workload},
        "track_px_per_s": px / (ms_step * 1e-3),
        "track_px": px,
    }


def kernel_source_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, shape, sources=None):
    """HBM-side bytes per launch from the committed counter summary of this workload, if it was
    taken on the current kernel sources (``sources``, the scorers' by default) and the same slab
    shape; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash(sources):
        return None
    if shape is not None and kv.get("slab_shape") != "x".join(str(x) for x in shape):
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline(kernel, kernel_ms, px, bpp, traffic=None, mix=None, lds_bpp=8, units=1, mix_units=1):
    """Roofline record of a scoring kernel (kernel_ms: its mean launch time; px: template pixels per
    launch, times `units` evaluations of the statistic per pixel for the delay grid; `mix` counts
    the instructions of `mix_units` such evaluations).

    The scorers keep map columns in LDS and re-read them there, so HBM carries a small part of the
    pixel records they consume (measured: `traffic`); what binds them is vector-ALU issue. The
    peak is the flop rate at which the inner loop's instruction mix (`mix`) keeps every SIMD of the
    chip issuing (unit counts x 2.4 GHz), with FLOPS_PER_TRACK_PX algorithmic flops per pixel, so
    frac = achieved pixel rate / issue ceiling. Beside it, not binding: the same flops against the
    FP32 vector peak; the LDS bytes the kernel reads against the measured random-row LDS read rate;
    the caller's pixel record against HBM bandwidth (the metric's "% gather roofline", above 1
    because pixels come from LDS). With a measured `traffic`, `memory_side` rates the bytes that
    left the L2s (slab staging, served by the MALL or HBM) against the measured streaming-read
    rate beyond the L2s: near 1, the kernel is bound by staging rather than by issue."""
    mix = mix or CORE_MIX
    sec = kernel_ms * 1e-3
    rate = px * units / sec
    ceiling = issue_ceiling_px_s(mix) * mix_units
    achieved = rate * FLOPS_PER_TRACK_PX / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": ceiling * FLOPS_PER_TRACK_PX / 1e12, "unit": "TFLOP/s",
            "frac": rate / ceiling, "traffic": traffic, "kernel": kernel, "kernel_ms": kernel_ms,
            "flops_per_track_px": FLOPS_PER_TRACK_PX,
            "peak_derivation": {"issue_mix_per_px": mix, "lanes_per_clk_per_cu": LANES_PER_CLK, "cus": N_CU,
                                "clock_hz": CLOCK_HZ, "ceiling_px_s": ceiling},
            "not_binding": {
                "fp32_flops": {"achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": achieved / FP32_PEAK_TFLOPS},
                "lds_read": {"bytes_per_track_px": lds_bpp, "achieved": rate * lds_bpp / 1e9,
                             "peak": LDS_RANDOM_GBS, "unit": "GB/s", "frac": rate * lds_bpp / 1e9 / LDS_RANDOM_GBS,
                             "peak_is": "measured 8-byte LDS reads at random rows"},
                "gather_line": {"bytes_per_track_px": bpp, "achieved": rate * bpp / 1e9, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": rate * bpp / 1e9 / HBM_PEAK_GBS}},
            "memory_side": None if traffic is None else {
                "achieved": traffic / sec / 1e9, "peak": FAR_READ_GBS, "unit": "GB/s",
                "frac": traffic / sec / 1e9 / FAR_READ_GBS,
                "peak_is": "measured streaming reads beyond the L2s (MALL-resident buffers)"}}


def timed(args, fn, torch):
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / args.steps


def run_single(args, name, w):
    import torch
    import paper_1401_8060_amd.stt as stt
    dtau_max = stt.dtau_units(w["dtau_s"])
    log(f"bench: building map {w['T']}x{w['F']}")
    Y, s, sha = make_map(w)
    dev = torch.device("cuda:0")
    m = stt.Map(torch.from_numpy(Y).to(dev), torch.from_numpy(s).to(dev))
    ctx = stt.Context(0)
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    n = w["n"]
    px = count_px(ctx, g, w["T"], w["F"], n)
    ctx.reserve(n)
    # slab shape and LDS budget from the tuning cache (searched and stored when missing; untimed setup)
    choice = ctx.autotune(m, g, n, args.tune_cache) if n >= 4096 else None
    if choice:
        log(f"bench: autotuned slab shape {choice[0]}x{choice[1]}, LDS {choice[2]} B")
    snr = None if args.no_snr else torch.empty(n, dtype=torch.float32, device=dev)
    key = torch.zeros(1, dtype=torch.int64, device=dev)

    def step():
        key.zero_()
        ctx.score(m, gen=g, n=n, snr=snr, best_key=key)

    log(f"bench: {n} tracks, {px} track-pixels; warmup {args.warmup}, timing {args.steps} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ms_step = timed(argparse.Namespace(warmup=0, steps=args.steps), step, torch)
    score_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    kern_ms = score_ms / max(cnt, 1)
    zk, jk = stt.decode_best(key)
    log(f"bench: {ms_step:.3f} ms/step, scoring kernel {kern_ms:.3f} ms avg over {cnt}; best z={zk:.4f} j={jk}")
    out = base_record(args, name, w, n, ms_step, px, "f32")
    out["config"].update({"T": w["T"], "F": w["F"], "n_tracks": n, "min_len": w["L"], "dtau_max_s": w["dtau_s"],
                          "sigma": list(w["sigma"]) if w["sigma"] != "unit" else "unit",
                          "injection": w["inject"] is not None, "per_track_snr": snr is not None, "map_sha256": sha[:16],
                          "slab_shape": list(choice) if choice else None})
    out["best"] = {"z": zk, "j": jk}
    out["roofline"] = roofline("k_score_slab" if n >= 4096 else "k_score_direct", kern_ms, px, BYTES_F32,
                               measured_traffic(name + ("_argmax" if snr is None else ""), choice))
    if snr is not None and not args.no_argmax_leg:
        # the search proper keeps only the loudest template (Sec. III, V): the same steps with no
        # per-template output, whose scattered 4-byte stores dominate the kernel's HBM writes
        def step_argmax():
            key.zero_()
            ctx.score(m, gen=g, n=n, snr=None, best_key=key)

        for _ in range(args.warmup):
            step_argmax()
        torch.cuda.synchronize()
        ctx.set_timing(True)
        ms_a = timed(argparse.Namespace(warmup=0, steps=args.steps), step_argmax, torch)
        sa, ca = ctx.kernel_ms_total(stt.STAGE_SCORE)
        ctx.set_timing(False)
        za, ja = stt.decode_best(key)
        log(f"bench: argmax only {ms_a:.3f} ms/step, scoring kernel {sa / max(ca, 1):.3f} ms; best z={za:.4f} j={ja}")
        out["argmax_only"] = {"value": n / (ms_a * 1e-3), "ms_per_step": ms_a, "kernel_ms": sa / max(ca, 1),
                              "track_px_per_s": px / (ms_a * 1e-3), "best": {"z": za, "j": ja},
                              "traffic": measured_traffic(name + "_argmax", choice)}
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, Y, s, dtau_max)
    ctx.close()
    return out


def run_batch(args, name, w):
    import numpy as np
    import torch
    import synth
    import paper_1401_8060_amd.stt as stt
    dtau_max = stt.dtau_units(w["dtau_s"])
    u = synth.uniform01(w["seed"], 99, w["n_maps"])
    Ts = (w["T_lo"] + np.floor(u * (w["T_hi"] - w["T_lo"] + 1))).astype(int).tolist()
    dev = torch.device("cuda:0")
    ctx = stt.Context(0)
    log(f"bench: building {w['n_maps']} maps, T in [{min(Ts)}, {max(Ts)}], F={w['F']}")
    maps = []
    for k, T in enumerate(Ts):
        Y, s, _ = make_map(w, stream=k, T=T)
        maps.append(stt.Map(torch.from_numpy(Y).to(dev), torch.from_numpy(s).to(dev)))
        del Y, s
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    ns = [w["n"]] * len(maps)
    px = sum(count_px(ctx, stt.Gen(seed=g.seed, stream=k, min_len=g.min_len, dtau_max=g.dtau_max), T, w["F"], w["n"])
             for k, T in enumerate(Ts))
    fp16 = args.map_dtype == "p16"
    smaps = [ctx.pack_p16(m) for m in maps] if fp16 else maps
    choice = ctx.autotune_batch(smaps, g, ns, args.tune_cache)
    log(f"bench: autotuned slab shape {choice[0]}x{choice[1]}, LDS {choice[2]} B")
    keys = torch.zeros(len(maps), dtype=torch.int64, device=dev)

    def step():
        keys.zero_()
        ctx.score_batch(smaps, g, ns, best_keys=keys)

    log(f"bench: {len(maps)} maps x {w['n']} tracks, {px} track-pixels")
    ms_step = timed(args, step, torch)
    # kernel breakdown from direct (uncaptured) launches of the same batch
    ctx.set_graph(False)
    ctx.set_timing(True)
    for _ in range(3):
        step()
    score_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    ctx.set_graph(True)
    kern_ms = score_ms / max(cnt, 1)
    log(f"bench: {ms_step:.3f} ms/step (graph replay), batch scoring kernel {kern_ms:.3f} ms")
    out = base_record(args, name, w, len(maps) * w["n"], ms_step, px, "f16" if fp16 else "f32")
    out["config"].update({"n_maps": len(maps), "T_range": [w["T_lo"], w["T_hi"]], "F": w["F"],
                          "tracks_per_map": w["n"], "map_dtype": args.map_dtype, "graph": True,
                          "slab_shape": list(choice)})
    out["roofline"] = roofline("k_score_batch", kern_ms, px, BYTES_P16 if fp16 else BYTES_F32,
                               measured_traffic(name + ("_p16" if fp16 else ""), choice),
                               mix=CORE_MIX_P16 if fp16 else CORE_MIX, lds_bpp=4 if fp16 else 8)
    if fp16:
        # error of FP16 storage against plain FP32 scoring of the same maps, on two maps in full
        errs = []
        for k in (0, len(maps) // 2):
            gk = stt.Gen(seed=g.seed, stream=k, min_len=g.min_len, dtau_max=g.dtau_max)
            z32 = ctx.score(maps[k], gen=gk, n=w["n"])[0].double()
            z16 = ctx.score(smaps[k], gen=gk, n=w["n"])[0].double()
            errs.append((z16 - z32).abs())
        e = torch.cat(errs)
        out["fp16_vs_fp32"] = {"max_abs_dz": e.max().item(), "mean_abs_dz": e.mean().item(),
                               "sample": "all tracks of maps 0 and n_maps/2"}
    ctx.close()
    return out


def run_precision(args, name, w):
    import torch
    import paper_1401_8060_amd.stt as stt
    dtau_max = stt.dtau_units(w["dtau_s"])
    log(f"bench: building map {w['T']}x{w['F']}")
    Y, s, sha = make_map(w)
    dev = torch.device("cuda:0")
    m = stt.Map(torch.from_numpy(Y).to(dev), torch.from_numpy(s).to(dev))
    ctx = stt.Context(0)
    pm = ctx.pack_p16(m)
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    n, K = w["n"], w["K"]
    px = count_px(ctx, g, w["T"], w["F"], n)
    ctx.reserve(n)
    choice = ctx.autotune(pm, g, n, args.tune_cache)
    log(f"bench: autotuned slab shape {choice[0]}x{choice[1]}, LDS {choice[2]} B")
    snr = torch.empty(n, dtype=torch.float32, device=dev)
    res = {}

    def step():
        ctx.score(pm, gen=g, n=n, snr=snr)
        idx, val = ctx.topk(snr, K)
        res["idx"], res["val"] = idx, val
        res["z64"] = ctx.rescore_f64(m, idx, gen=g)

    ctx.set_timing(True)
    ms_step = timed(args, step, torch)
    score_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    kern_ms = score_ms / max(cnt, 1)
    err = (res["val"].double() - res["z64"]).abs()
    best = int(torch.argmax(res["z64"]).item())
    log(f"bench: {ms_step:.3f} ms/step, FP16 scoring kernel {kern_ms:.3f} ms; top-{K} |dz| max {err.max().item():.2e}")

    out = base_record(args, name, w, n, ms_step, px, "f16")
    out["config"].update({"T": w["T"], "F": w["F"], "n_tracks": n, "map_dtype": "p16", "scale_exp": pm.scale_exp,
                          "top_k": K, "rescore": "f64", "map_sha256": sha[:16], "slab_shape": list(choice)})
    out["roofline"] = roofline("k_score_slab", kern_ms, px, BYTES_P16, measured_traffic(name, choice),
                               mix=CORE_MIX_P16, lds_bpp=4)
    out["topk_fp16_vs_fp64"] = {"max_abs_dz": err.max().item(), "mean_abs_dz": err.mean().item(),
                                "reference": "the library's FP64 re-score (k_rescore_f64) of the same templates"}
    if not args.no_cpu_baseline:
        # the CPU leg: the oracle (FP64, on the FP32 map) scores the top-K templates; its time is the CPU
        # baseline and its scores the reference of the FP16 error record (relative to max(1, |z|))
        import numpy as np
        import oracle
        log(f"bench: the CPU oracle on the top {K}")
        idx = res["idx"].cpu().numpy().astype(np.uint64)
        t = time.perf_counter()
        z_orc = oracle.score_gen_idx(oracle.Map(Y, s), w["seed"], 0, w["L"], dtau_max, idx)
        dt = time.perf_counter() - t
        z16 = res["val"].cpu().numpy().astype(np.float64)
        rel = np.abs(z16 - z_orc) / np.maximum(1.0, np.abs(z_orc))
        out["topk_fp16_vs_oracle"] = {"max_rel_dz": float(rel.max()), "mean_rel_dz": float(rel.mean()),
                                      "relative_to": "max(1, |z_oracle|)",
                                      "reference": f"the FP64 CPU oracle on the FP32 map, the top {K} templates"}
        out["cpu_baseline"] = dict(value=K / dt, unit="tracks/s", cores=1, kind="oracle",
                                   sample=f"the top {K} templates of the step (FP64 on the FP32 map), one thread, "
                                          f"{dt:.2f} s")
    out["best"] = {"z64": res["z64"][best].item(), "j": int(res["idx"][best].item())}
    ctx.close()
    return out


def run_tmid(args, name, w):
    import torch
    import paper_1401_8060_amd.stt as stt
    dtau_max = stt.dtau_units(w["dtau_s"])
    log(f"bench: building map {w['T']}x{w['F']}")
    Y, s, sha = make_map(w)
    dev = torch.device("cuda:0")
    m = stt.Map(torch.from_numpy(Y).to(dev), torch.from_numpy(s).to(dev))
    ctx = stt.Context(0)
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    n = w["n"]
    px = count_px(ctx, g, w["T"], w["F"], n)  # a free t_mid keeps the time extent, so the pixel count
    snr = torch.empty(n, dtype=torch.float32, device=dev)
    key = torch.zeros(1, dtype=torch.int64, device=dev)

    def step_fn():
        key.zero_()
        ctx.score_tm(m, gen=g, n=n, snr=snr, best_key=key)

    for _ in range(args.warmup):
        step_fn()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ms_step = timed(argparse.Namespace(warmup=0, steps=args.steps), step_fn, torch)
    score_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    kern_ms = score_ms / max(cnt, 1)
    zk, jk = stt.decode_best(key)
    log(f"bench: {ms_step:.3f} ms/step, free-t_mid scoring kernel {kern_ms:.3f} ms; best z={zk:.4f} j={jk}")
    out = base_record(args, name, w, n, ms_step, px, "f32")
    out["config"].update({"T": w["T"], "F": w["F"], "n_tracks": n, "templates": "free t_mid",
                          "map_sha256": sha[:16]})
    out["roofline"] = roofline("k_score_tm_slab", kern_ms, px, BYTES_F32, measured_traffic(name, None),
                               mix=CORE_MIX_TM)
    out["best"] = {"z": zk, "j": jk}
    ctx.close()
    return out


def run_maxdelay(args, name, w):
    import torch
    import paper_1401_8060_amd.stt as stt
    dtau_max = stt.dtau_units(w["dtau_s"])
    log(f"bench: building map {w['T']}x{w['F']}")
    Y, s, sha = make_map(w)
    dev = torch.device("cuda:0")
    m = stt.Map(torch.from_numpy(Y).to(dev), torch.from_numpy(s).to(dev))
    ctx = stt.Context(0)
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    n, nt = w["n"], w["n_tau"]
    d0, step = -dtau_max, (2 * dtau_max) // (nt - 1)
    px = count_px(ctx, g, w["T"], w["F"], n)
    ctx.reserve(n)
    snr = torch.empty(n, dtype=torch.float32, device=dev)
    tidx = torch.empty(n, dtype=torch.int32, device=dev)
    key = torch.zeros(1, dtype=torch.int64, device=dev)

    def step_fn():
        key.zero_()
        ctx.score_maxdelay(m, d0, step, nt, gen=g, n=n, snr=snr, tau_idx=tidx, best_key=key)

    for _ in range(args.warmup):
        step_fn()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ms_step = timed(argparse.Namespace(warmup=0, steps=args.steps), step_fn, torch)
    score_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    kern_ms = score_ms / max(cnt, 1)
    zk, jk = stt.decode_best(key)
    mk = int(tidx[jk].item())
    log(f"bench: {ms_step:.3f} ms/step, delay-grid scoring ({(nt + 7) // 8} launches) {kern_ms:.3f} ms; "
        f"best z={zk:.4f} j={jk} delay index {mk} ({(d0 + mk * step) * 2.0 ** -28 * 1e3:.3f} ms)")
    out = base_record(args, name, w, n, ms_step, px, "f32")
    out["config"].update({"T": w["T"], "F": w["F"], "n_tracks": n, "n_tau": nt, "dtau0": d0, "dtau_step": step,
                          "map_sha256": sha[:16]})
    out["template_delays_per_s"] = n * nt / (ms_step * 1e-3)
    # the grid runs in launches of up to 8 delays; the stage time covers all of them, so one launch
    # averages kern_ms / launches over (on average) nt / launches delays of every template pixel
    launches = (nt + 7) // 8
    out["roofline"] = roofline("k_score_md_slab", kern_ms / launches, px, BYTES_F32, measured_traffic(name, None),
                               mix=CORE_MIX_MD,
                               units=nt / launches, mix_units=8)
    out["roofline"]["launches_per_step"] = launches
    out["best"] = {"z": zk, "j": jk, "delay_index": mk}
    ctx.close()
    return out


def run_mapform(args, name, w):
    import numpy as np
    import torch
    import synth
    import paper_1401_8060_amd.stt as stt
    p = stt.Spectro(w["fs"], w["M"], w["k_lo"], w["F"], w["nb"])
    T, F, ns = w["T"], w["F"], w["n_slides"]
    n = (T + 1) * w["M"] // 2
    log(f"bench: building {n} samples of strain per detector")
    strains = []
    for k in range(2):
        x = synth.white_strain(n, seed=w["seed"], stream=k)
        ch = w["chirp"]
        synth.add_tone(x, w["fs"], ch["f0"], ch["amp"], delay_s=ch["delay"] * k, t_start_s=ch["t0"],
                       t_stop_s=ch["t1"], chirp_hz_per_s=ch["rate"])
        strains.append(x)
    dev = torch.device("cuda:0")
    xi, xj = (torch.from_numpy(x).to(dev) for x in strains)
    ctx = stt.Context(0)
    shifts = [w["slide_cols"] * k for k in range(ns)]
    si = torch.empty((T, F), dtype=torch.complex64, device=dev)
    sj = torch.empty_like(si)
    pi = torch.empty((T, F), dtype=torch.float32, device=dev)
    pj = torch.empty_like(pi)
    maps = ctx.form_maps(p, *ctx.spectra(xi, p, T, si, pi), *ctx.spectra(xj, p, T, sj, pj), shifts)

    def step_fn():
        ctx.spectra(xi, p, T, si, pi)
        ctx.spectra(xj, p, T, sj, pj)
        ctx.form_maps(p, si, pi, sj, pj, shifts, out=maps)

    for _ in range(args.warmup):
        step_fn()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ms_step = timed(argparse.Namespace(warmup=0, steps=args.steps), step_fn, torch)
    form_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    form_ms /= max(cnt, 1)
    # a second pass for the whole-call brackets (a total query forgets the calls it summed)
    timed(argparse.Namespace(warmup=0, steps=args.steps), step_fn, torch)
    call_ms, ncall = ctx.kernel_ms_total(stt.STAGE_CALL)
    ctx.set_timing(False)
    launches = (ns + 15) // 16
    spectra_ms = call_ms / args.steps - form_ms  # the two stt_spectra calls of a step
    launch_ms = form_ms / launches
    px = ns * T * F
    log(f"bench: {ms_step:.3f} ms/step; spectra+P' {spectra_ms:.3f} ms, {ns} slide maps {form_ms:.3f} ms "
        f"({launches} launches of k_form_maps, {launch_ms * 1e3:.1f} us each)")
    # algorithmic bytes of one k_form_maps launch: its slides' maps written (8 B Y + 4 B sigma per
    # pixel) and both detectors' spectra and P' read once (2 x 12 B per pixel)
    per_launch = [min(16, ns - k) for k in range(0, ns, 16)]
    bytes_launch = sum(12 * T * F * m + 24 * T * F for m in per_launch) / launches
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    fq4_lo, dfq4 = p.fq4()
    out = {
        "metric": "cross-power map pixels formed/sec per MI355X (time-slide background maps)",
        "value": px / (ms_step * 1e-3), "unit": "map pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "fs": w["fs"], "M": w["M"], "T": T, "F": F, "k_lo": w["k_lo"], "nb": w["nb"],
                   "n_slides": ns, "slide_cols": w["slide_cols"], "fq4_lo": fq4_lo, "dfq4": dfq4},
        "maps_per_s": ns / (ms_step * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "traffic": measured_traffic(name, None, MAPFORM_SOURCES), "kernel": "k_form_maps",
                     "kernel_ms": launch_ms,
                     "launches_per_step": launches, "bytes_per_launch": bytes_launch},
        "spectra_ms": spectra_ms,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the map-formation oracle")
        from oracle import mapform
        k = ns  # the whole step takes the oracle a few seconds
        t = time.perf_counter()
        mapform.form_maps(strains[0], strains[1], w["fs"], w["M"], T, w["k_lo"], F, w["nb"], shifts[:k])
        dt = time.perf_counter() - t
        out["cpu_baseline"] = dict(value=k * T * F / dt, unit="map pixels/s", cores=1, kind="oracle",
                                   sample=f"the whole step (both detectors' spectra and P', all {k} slide maps), "
                                          f"numpy FP64, one thread, {dt:.1f} s")
    ctx.close()
    return out


def run_background(args, name, w):
    import torch
    import synth
    import paper_1401_8060_amd.stt as stt
    p = stt.Spectro(w["fs"], w["M"], w["k_lo"], w["F"], w["nb"])
    T, F, ns = w["T"], w["F"], w["n_slides"]
    n_smp = (T + 1) * w["M"] // 2
    log(f"bench: building {n_smp} samples of strain per detector")
    strains = []
    for k in range(2):
        x = synth.white_strain(n_smp, seed=w["seed"], stream=k)
        ch = w["chirp"]
        synth.add_tone(x, w["fs"], ch["f0"], ch["amp"], delay_s=ch["delay"] * k, t_start_s=ch["t0"],
                       t_stop_s=ch["t1"], chirp_hz_per_s=ch["rate"])
        strains.append(x)
    dev = torch.device("cuda:0")
    xi, xj = (torch.from_numpy(x).to(dev) for x in strains)
    ctx = stt.Context(0)
    shifts = [w["slide_cols"] * k for k in range(ns)]
    si = torch.empty((T, F), dtype=torch.complex64, device=dev)
    sj = torch.empty_like(si)
    pi = torch.empty((T, F), dtype=torch.float32, device=dev)
    pj = torch.empty_like(pi)
    maps = ctx.form_maps(p, *ctx.spectra(xi, p, T, si, pi), *ctx.spectra(xj, p, T, sj, pj), shifts)
    dtau_max = stt.dtau_units(w["dtau_s"])
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    g_deep = stt.Gen(seed=w["seed"] + 1, stream=0, min_len=w["L"], dtau_max=dtau_max)  # a new seed per run
    nt = [w["n"]] * ns
    choice = ctx.autotune_batch(maps, g, nt, args.tune_cache)
    log(f"bench: autotuned batch slab shape {choice[0]}x{choice[1]}, LDS {choice[2]} B")
    keys = torch.zeros(ns, dtype=torch.int64, device=dev)
    state = {}

    def step():
        ctx.spectra(xi, p, T, si, pi)
        ctx.spectra(xj, p, T, sj, pj)
        ctx.form_maps(p, si, pi, sj, pj, shifts, out=maps)
        keys.zero_()
        ctx.score_batch(maps, g, nt, best_keys=keys)
        cnt, fap, za = ctx.significance(keys[1:], keys[:1], alpha=w["alpha"])
        state["fap0"], state["za"], state["keys0"] = fap, za, keys.clone()
        state["chosen"] = ctx.follow_up(maps, keys, g_deep, w["n_deep"], k=w["k_follow"])

    ms_step = timed(args, step, torch)
    # the batch kernel's share, from direct (uncaptured) launches of the same batch
    ctx.set_graph(False)
    ctx.set_timing(True)
    for _ in range(2):
        keys.zero_()
        ctx.score_batch(maps, g, nt, best_keys=keys)
    score_ms, cnt_b = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    ctx.set_graph(True)
    kern_ms = score_ms / max(cnt_b, 1)
    k0 = state["keys0"].cpu().numpy().view("uint64")  # the batch's keys, before the follow-up
    z_all = [stt.key_decode(int(k))[0] for k in k0]
    z0 = z_all[0]
    loud = max(range(1, ns), key=lambda m: z_all[m])
    fap0, za = float(state["fap0"].item()), float(state["za"].item())
    log(f"bench: {ms_step:.3f} ms/step; batch kernel {kern_ms:.3f} ms; zero-lag z={z0:.3f}, FAP {fap0:.4f} "
        f"against {ns - 1} slides, z_alpha {za:.3f} (slide {loud}, shift {shifts[loud]} columns); "
        f"followed up {len(state['chosen'])} maps")
    px_batch = sum(count_px(ctx, stt.Gen(seed=g.seed, stream=k, min_len=g.min_len, dtau_max=g.dtau_max), T, F,
                            w["n"]) for k in range(ns))
    out = {
        "metric": "background maps searched/sec per MI355X (strain -> slide maps -> 10^6 templates each -> FAP)",
        "value": ns / (ms_step * 1e-3), "unit": "maps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "fs": w["fs"], "M": w["M"], "T": T, "F": F, "n_slides": ns,
                   "tracks_per_map": w["n"], "alpha": w["alpha"], "n_deep": w["n_deep"], "k_follow": w["k_follow"],
                   "slab_shape": list(choice)},
        "roofline": roofline("k_score_batch", kern_ms, px_batch, BYTES_F32, None),
        "zero_lag": {"z": z0, "fap": fap0, "z_alpha": za, "loudest_slide": loud, "followed_up": len(state["chosen"])},
    }
    ctx.close()
    return out


def run_refine(args, name, w):
    import numpy as np
    import torch
    import synth
    import paper_1401_8060_amd.stt as stt
    dtau_max = stt.dtau_units(w["dtau_s"])
    T, F = w["T"], w["F"]
    log(f"bench: building map {T}x{F} with {w['n_inj']} injections")
    Y, s, _ = make_map(w)
    u = synth.uniform01(w["seed"], 77, 6 * w["n_inj"]).reshape(w["n_inj"], 6)
    inj = []
    for i in range(w["n_inj"]):
        t0 = int(u[i, 0] * (T - 300))
        t2 = t0 + 100 + int(u[i, 1] * 190)
        f = 20 + u[i, 2:5] * (F - 40)
        dt = int(round((u[i, 5] * 2 - 1) * 0.008 / 2.0 ** -28))
        snr = 5.0 + 5.0 * i / (w["n_inj"] - 1)
        cols, rows = synth.bezier_rows_float(t0, t2, *f)
        synth.add_pixels(Y, s, cols, rows, snr / math.sqrt(cols.size), -((100.0 + rows) * dt * 2.0 ** -28))
        inj.append(dict(t0=t0, t2=t2, snr=snr))
    dev = torch.device("cuda:0")
    m = stt.Map(torch.from_numpy(Y).to(dev), torch.from_numpy(s).to(dev))
    ctx = stt.Context(0)
    g = stt.Gen(seed=w["seed"], stream=0, min_len=w["L"], dtau_max=dtau_max)
    n, K = w["n"], w["K"]
    px = count_px(ctx, g, T, F, n)
    choice = ctx.autotune(m, g, n, args.tune_cache)
    log(f"bench: autotuned slab shape {choice[0]}x{choice[1]}, LDS {choice[2]} B")
    snr = torch.empty(n, dtype=torch.float32, device=dev)
    res = {}

    def step():
        ctx.score(m, gen=g, n=n, snr=snr)
        idx, val = ctx.topk(snr, K)
        tr = ctx.tracks_at(g, T, F, idx)
        th, Ks = ctx.tracks_to_theta(tr)
        res.update(val=val, th0=th, K=Ks)
        res["out"] = ctx.refine(m, th, Ks, w["L"], dtau_max, steps=w["steps"])

    ms_step = timed(args, step, torch)
    z_plain0 = res["val"].double()
    z_s0 = ctx.smooth(m, res["th0"], res["K"]).double()
    th, zs, trr, zp = res["out"]
    log(f"bench: {ms_step:.3f} ms/step; best plain z {z_plain0.max().item():.3f} -> refined {zp.max().item():.3f}")
    out = base_record(args, name, w, n, ms_step, px, "f32")
    out["config"].update({"T": T, "F": F, "n_tracks": n, "top_k": K, "steps": w["steps"], "injections": inj})
    out["refine"] = {"best_plain_z_random_search": z_plain0.max().item(),
                     "best_plain_z_after_refine": zp.max().item(),
                     "mean_smooth_gain": (zs.double() - z_s0).mean().item(),
                     "improved_fraction": (zp.double() > z_plain0).double().mean().item()}
    # the refinement kernel alone, from calls without the plain re-score: each of its steps + 1
    # evaluations gathers the 4 bilinear neighbours of every sample of every template, 8 B each (p of
    # the folded complex map)
    ctx.set_timing(True)
    for _ in range(3):
        ctx.refine(m, res["th0"], res["K"], w["L"], dtau_max, steps=w["steps"], plain=False)
    ref_ms, cnt = ctx.kernel_ms_total(stt.STAGE_SCORE)
    ctx.set_timing(False)
    ref_ms /= max(cnt, 1)
    gbytes = (w["steps"] + 1) * int(res["K"].sum().item()) * 4 * 8
    achieved = gbytes / (ref_ms * 1e-3) / 1e9
    log(f"bench: k_refine {ref_ms:.3f} ms per launch, {gbytes / 1e6:.0f} MB gathered ({achieved:.0f} GB/s)")
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_refine", "kernel_ms": ref_ms,
                       "bytes_per_launch": gbytes,
                       "note": "bilinear gathers served from L2/MALL: the kernel waits on their latency, "
                               "not on HBM bandwidth"}
    ctx.close()
    return out


def issue_rates(iters: int = 4096) -> dict:
    """Vector-ALU issue rates (lane-instructions per shader clock per CU) of the instructions in the
    scorers' inner loops, from the probe library (eight independent register chains per lane, eight
    waves per SIMD; the shader clock measured inside each launch)."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_1401_8060_amd", "libstt_probe.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(path)
    L.stt_probe_name.restype = C.c_char_p
    L.stt_probe_issue.argtypes = [C.c_int, C.c_int, C.c_int] + [C.POINTER(C.c_double)] * 3
    rates, mhz = {}, []
    for op in range(L.stt_probe_count()):
        r, f, ms = C.c_double(), C.c_double(), C.c_double()
        rc = L.stt_probe_issue(0, op, iters, C.byref(r), C.byref(f), C.byref(ms))
        name = L.stt_probe_name(op).decode()
        if rc != 0:
            raise RuntimeError(f"issue probe {name} failed ({rc})")
        rates[name] = round(r.value, 2)
        mhz.append(f.value)
        log(f"bench: {name:16s} {r.value:7.2f} lanes/clk/CU  ({ms.value:.2f} ms at {f.value:.0f} MHz)")
    return {"lanes_per_clk_per_cu": rates, "shader_mhz": [round(min(mhz)), round(max(mhz))],
            "method": "8 independent register chains per lane, unrolled x4, 8 waves per SIMD, "
                      f"{iters} iterations; clock from the cycle and wall counters of the first wave"}


def mem_rates() -> dict:
    """Memory-side ceilings from the probe library: streaming reads of buffers from 8 MB (inside
    the 8 x 4 MB of L2) through 32-256 MB (beyond the L2s, inside the 256 MB MALL) to 4 GB (HBM);
    8-byte LDS reads at random rows and at conflict-free rows."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_1401_8060_amd", "libstt_probe.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(path)
    L.stt_probe_stream.argtypes = [C.c_int, C.c_int64, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.stt_probe_lds.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    out = {}
    sizes_mb = (8, 16, 32, 48, 64, 96, 128, 192, 256, 384, 1024, 4096)
    for name, nbytes, reps in ((f"{mb}MB", mb << 20, max(2, 3000 // mb)) for mb in sizes_mb):
        g, ms = C.c_double(), C.c_double()
        rc = L.stt_probe_stream(0, nbytes, reps, C.byref(g), C.byref(ms))
        if rc != 0:
            raise RuntimeError(f"stream probe {name} failed ({rc})")
        out[f"stream_read_{name}_GBs"] = round(g.value, 1)
        log(f"bench: stream read {name:11s} {g.value:9.1f} GB/s ({ms.value:.3f} ms, {reps} passes)")
    for name, rnd in (("random_rows", 1), ("conflict_free", 0)):
        g, ms = C.c_double(), C.c_double()
        rc = L.stt_probe_lds(0, rnd, 4096, C.byref(g), C.byref(ms))
        if rc != 0:
            raise RuntimeError(f"LDS probe {name} failed ({rc})")
        out[f"lds_read_8B_{name}_GBs"] = round(g.value, 1)
        log(f"bench: LDS 8-byte reads, {name:13s} {g.value:9.1f} GB/s ({ms.value:.3f} ms)")
    out["method"] = ("streaming: float4 grid-stride reads, 8 workgroups of 256 lanes per CU, timed after one "
                     "untimed launch; LDS: ds_read_b64 from a 16 KB table per workgroup, 8 waves per SIMD, "
                     "8 independent rows per lane per iteration")
    return out


def summarize_pmc(paths: list[str], kernel: str) -> dict:
    """Mean per dispatch of every counter that rocprofv3 --pmc wrote (counter_collection.csv files)
    for the kernels whose name contains ``kernel``, with the dispatch count and register counts."""
    import csv
    vals, disp, regs = {}, set(), set()
    for path in paths:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if kernel not in row["Kernel_Name"]:
                    continue
                d = (path, row["Dispatch_Id"])
                disp.add(d)
                regs.add((row.get("VGPR_Count"), row.get("SGPR_Count"), row.get("LDS_Block_Size"),
                          row.get("Workgroup_Size"), row.get("Grid_Size")))
                vals.setdefault(row["Counter_Name"], {})
                vals[row["Counter_Name"]][d] = vals[row["Counter_Name"]].get(d, 0.0) + float(row["Counter_Value"])
    out = {"kernel": kernel, "dispatches": len(disp),
           "launch": [dict(zip(("vgpr", "sgpr", "lds", "wg", "grid"), r)) for r in sorted(regs, key=str)]}
    out["mean_per_dispatch"] = {k: sum(v.values()) / len(v) for k, v in sorted(vals.items())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="search_1000x1000_1e7", choices=sorted(WORKLOADS))
    ap.add_argument("--map-dtype", default="f32", choices=["f32", "p16"], help="batch workload map storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-snr", action="store_true", help="reduce to the argmax only (no per-track output)")
    ap.add_argument("--no-argmax-leg", action="store_true",
                    help="search workloads: skip the second, argmax-only timing (counter runs of one mode)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache (JSON); a missing entry is searched on the GPU and stored")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device (a known-size kernel for counter scaling)")
    ap.add_argument("--issue-rates", action="store_true",
                    help="measure the vector-ALU issue rates of the scorers' instructions and exit")
    ap.add_argument("--mem-rates", action="store_true",
                    help="measure the streaming-read (L2, MALL, HBM) and LDS-read ceilings and exit")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="CSV",
                    help="print the mean per dispatch of the counters in rocprofv3 counter_collection.csv files "
                         "for the kernel named by --kernel, and exit (no GPU needed)")
    ap.add_argument("--kernel", default="k_score_slab", help="kernel name filter of --summarize-pmc")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc, args.kernel), indent=1), flush=True)
        return
    if args.issue_rates:
        print(json.dumps({"issue_rates": issue_rates()}), flush=True)
        return
    if args.mem_rates:
        print(json.dumps({"mem_rates": mem_rates()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the search shards by template range "
              "or by map with no communication but a max, which is not implemented here.", file=sys.stderr)
        sys.exit(2)
    w = WORKLOADS[args.workload]
    runner = {"single": run_single, "batch": run_batch, "precision": run_precision, "refine": run_refine,
              "maxdelay": run_maxdelay, "tmid": run_tmid, "mapform": run_mapform,
              "background": run_background}[w["kind"]]
    out = runner(args, args.workload, w)
    if args.copy_probe_mb:
        import torch
        nb = args.copy_probe_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
