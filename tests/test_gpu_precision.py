"""GPU parity of the precision addition: FP16 map storage with a per-map power-of-two
scale, FP32 accumulation, top-K selection and the FP64 re-score of the winners."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import synth
from tests.parity_util import assert_argmax, assert_close, bench_tuning_copy, key_to_host, to_dev

pytestmark = pytest.mark.gpu
D10MS = 2684355


@pytest.fixture(scope="module")
def stt():
    import paper_1401_8060_amd.stt as stt
    return stt


@pytest.fixture(scope="module")
def ctx(stt):
    c = stt.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _inject(Y, s, t0=150, t2=1799, f=(500.5, 1500.25, 900.75), dt_s=0.003, snr=8.0):
    cols, rows = synth.bezier_rows_float(t0, t2, *f)
    dt = int(round(dt_s / 2.0 ** -28))
    synth.add_pixels(Y, s, cols, rows, snr / math.sqrt(cols.size), -((100.0 + rows) * dt * 2.0 ** -28))


def test_pack_p16_bit_exact(orc, stt, ctx):
    _say("pack")
    import torch
    Y, s = synth.noise_map(123, 77, seed=4, sigma=("loguniform", 0.5, 2.0))
    Y[3, 5] = np.complex64(3000.0 * s[3, 5])
    q, e, _ = orc.quantize_p16(Y, s)
    pm = ctx.pack_p16(stt.Map(*to_dev(Y, s)))
    assert pm.scale_exp == e
    got = pm.data.cpu().numpy()
    assert np.array_equal(got.view(np.uint16), q.view(np.uint16))


@pytest.mark.parametrize("path,dma", [(1, True), (2, True), (2, False), (3, True)])
def test_p16_scores_match_oracle_on_the_stored_map(orc, stt, ctx, path, dma):
    """Same FP16 inputs on both sides: the GPU's FP32 accumulation vs the oracle's FP64."""
    _say("p16 scores", path)
    T, F, n = 400, 300, 20_000
    Y, s = synth.noise_map(T, F, seed=5, sigma=("loguniform", 0.5, 2.0))
    q, e, deq = orc.quantize_p16(Y, s)
    om = orc.Map(deq, np.ones((T, F)))
    z_orc = orc.score_gen(om, 7, 0, 10, D10MS, 0, n)
    pm = ctx.pack_p16(stt.Map(*to_dev(Y, s)))
    ctx.set_path(path)
    ctx.set_staging(dma)
    snr, key = ctx.score(pm, gen=stt.Gen(seed=7, min_len=10, dtau_max=D10MS), n=n)
    ctx.set_staging(True)
    ctx.set_path(0)
    assert_close(snr.cpu().numpy(), z_orc, what=f"p16 path {path}")
    assert_argmax(stt.key_decode(key_to_host(key))[1], z_orc)


def test_p16_error_against_fp64_truth_within_storage_bound(orc, stt, ctx):
    """FP16 storage error vs the FP64 score of the FP32 map, bounded per track by
    (2^-11 + pi 2^-16) * sum|p|/sqrt(N) (the magnitude rounded to 11 significant bits, the argument
    to the nearest 2^-16 turn, at most pi 2^-16 rad away) plus FP32 slack."""
    _say("p16 error")
    T, F, n = 500, 400, 5000
    Y, s = synth.noise_map(T, F, seed=6, sigma=("loguniform", 0.5, 2.0))
    om = orc.Map(Y, s)
    tr = orc.draw_many(8, 0, 0, n, T, F, 10, D10MS)
    z64 = orc.score_list(om, tr)
    import torch
    pm = ctx.pack_p16(stt.Map(*to_dev(Y, s)))
    dev = torch.from_numpy(tr.view(np.int32).reshape(-1, 6).copy()).cuda()
    z16 = ctx.score(pm, tracks=dev)[0].cpu().numpy().astype(np.float64)
    p = Y.astype(np.complex128) / s
    bound = np.empty(n)
    for i, t in enumerate(tr):
        r = orc.rows(t, F)
        cols = np.arange(int(t["t0"]), int(t["t2"]) + 1)
        pk = p[cols, r]
        bound[i] = (2.0 ** -11 + math.pi * 2.0 ** -16) * np.abs(pk).sum() / math.sqrt(cols.size)
    err = np.abs(z16 - z64)
    assert (err <= bound + 1e-5).all()
    _say(f"FP16 vs FP64: max |dz| {err.max():.2e}, mean {err.mean():.2e}")
    assert err.mean() < 5e-4


@pytest.mark.parametrize("n,K", [(1, 1), (5000, 1024), (1_000_003, 1024), (300_000, 8192), (70_000, 70_000 // 10)])
def test_topk_bit_exact(orc, stt, ctx, n, K):
    _say("topk", n, K)
    import torch
    sel = np.random.default_rng(n)
    z = sel.standard_normal(n).astype(np.float32).round(3)  # many ties
    if n > 10:
        z[sel.choice(n, n // 100, replace=False)] = np.nan
        z[sel.choice(n, 5, replace=False)] = np.inf
    idx, val = ctx.topk(torch.from_numpy(z).cuda(), K, first=1000)
    want = orc.topk(z.astype(np.float64), K)
    assert np.array_equal(idx.cpu().numpy() - 1000, want)
    assert np.array_equal(val.cpu().numpy(), z[want], equal_nan=True)


def test_rescore_f64_matches_oracle(orc, stt, ctx):
    _say("rescore")
    import torch
    T, F = 700, 500
    Y, s = synth.noise_map(T, F, seed=9, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    om = orc.Map(Y, s)
    idx = np.random.default_rng(1).choice(10**6, 1500, replace=False).astype(np.int64)
    z = ctx.rescore_f64(m, torch.from_numpy(idx).cuda(), gen=stt.Gen(seed=3, min_len=10, dtau_max=D10MS))
    want = orc.score_gen_idx(om, 3, 0, 10, D10MS, idx)
    assert np.allclose(z.cpu().numpy(), want, rtol=0, atol=1e-11)
    # explicit tracks, norm N, an index before `first` gives NaN
    tr = orc.draw_many(4, 0, 0, 300, T, F, 10, D10MS)
    dev = torch.from_numpy(tr.view(np.int32).reshape(-1, 6).copy()).cuda()
    ids = torch.tensor([50, 50 + 299, 50 + 7, 49], dtype=torch.int64, device="cuda")
    z = ctx.rescore_f64(m, ids, tracks=dev, first=50, norm=stt.NORM_N).cpu().numpy()
    want = orc.score_list(om, tr[[0, 299, 7]], norm=orc.NORM_N)
    assert np.allclose(z[:3], want, rtol=0, atol=1e-12) and np.isnan(z[3])


def test_precision_pipeline_full_scale(orc, stt, ctx, tmp_path):
    """T=2000 x F=2000 map stored in FP16, 10^8 tracks with FP32 accumulation, top-1024
    re-scored in FP64 from the FP32 map. Checked: the first 3x10^7 FP16 scores, every one, a
    sample of the rest and the GPU's 20 best against the oracle on the stored map (run over
    disjoint template ranges on the host cores; all 10^8 take the oracle about 150 s on 16
    threads), the GPU's argmax against the oracle's over all of those, the top-1024 against a CPU
    selection over the same score array, every re-scored value against the oracle, and the final
    argmax against the oracle's."""
    import time
    from oracle import shard
    _say("precision pipeline")
    import torch
    T, F, n, K = 2000, 2000, 100_000_000, 1024
    Y, s = synth.noise_map(T, F, seed=1004, sigma=("loguniform", 0.5, 2.0))
    _inject(Y, s)
    m = stt.Map(*to_dev(Y, s))
    pm = ctx.pack_p16(m)
    g = stt.Gen(seed=4, min_len=10, dtau_max=D10MS)
    _say("precision pipeline, slab shape", ctx.autotune(pm, g, n, bench_tuning_copy(tmp_path)))
    snr, key = ctx.score(pm, gen=g, n=n)
    ctx.set_slab_shape(1024, 4)
    ctx.set_path(0, 160 * 1024)
    idx, val = ctx.topk(snr, K)
    z64 = ctx.rescore_f64(m, idx, gen=g).cpu().numpy()
    zs = snr.cpu().numpy()
    # top-K against a CPU selection over the same FP32 array
    part = np.argpartition(-np.nan_to_num(zs, nan=-np.inf), K)[:K]
    want = part[np.lexsort((part, -zs[part]))]
    assert np.array_equal(idx.cpu().numpy(), want)
    # every FP16 score vs the oracle on the stored map
    q, e, deq = orc.quantize_p16(Y, s)
    assert e == pm.scale_exp
    om16 = orc.Map(deq, np.ones((T, F)))
    n_full = 30_000_000
    t = time.time()
    z16 = shard.score_gen(om16, 4, 0, 10, D10MS, 0, n_full)
    _say(f"  oracle: {n_full} templates on the stored map in {time.time() - t:.1f} s on {shard.host_threads()} threads")
    assert_close(zs[:n_full], z16, what="p16 first 3e7")
    rest = np.concatenate([n_full + np.random.default_rng(4).choice(n - n_full, 2000, replace=False),
                           want[:20]]).astype(np.uint64)
    z16r = orc.score_gen_idx(om16, 4, 0, 10, D10MS, rest)
    assert_close(zs[rest.astype(np.int64)], z16r, what="p16 sample and top 20")
    jk = stt.key_decode(key_to_host(key))[1]
    assert jk == int(want[0])  # the key is the best of the score array
    # over every template the oracle scored, the GPU's argmax is the oracle's (up to a certified tie)
    cand = np.concatenate([z16, z16r])
    cand_idx = np.concatenate([np.arange(n_full), rest.astype(np.int64)])
    assert_argmax(int(np.where(cand_idx == jk)[0][0]), cand)
    del z16, cand
    # FP64 re-score vs the oracle on the FP32 map; final argmax among the K
    om = orc.Map(Y, s)
    z_orc = orc.score_gen_idx(om, 4, 0, 10, D10MS, want.astype(np.uint64))
    assert np.allclose(z64, z_orc, rtol=0, atol=1e-10)
    assert int(np.argmax(z64)) == orc.argmax(z_orc)
    err = np.abs(val.cpu().numpy().astype(np.float64) - z_orc)
    _say(f"top-1024 FP16/FP32 vs FP64: max |dz| {err.max():.2e}, mean {err.mean():.2e}")
