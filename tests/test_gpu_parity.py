"""GPU parity: libstt (HIP, gfx950) against the CPU oracle, element by element.

Every call goes through the C ABI (ctypes binding). Inputs are seeded
synthetic maps; expected values come from the oracle only. Templates and
argmax indices must match exactly (argmax up to a certified FP64 near-tie);
FP32 scores within 1e-5 * max(1, |z|).
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import synth
from tests.parity_util import TOL, assert_argmax, assert_close, bench_tuning_copy, key_to_host, to_dev

pytestmark = pytest.mark.gpu

D10MS = 2684355  # 10 ms in 2^-28 s units


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


def _gen(stt, seed=1, stream=0, L=10, D=D10MS):
    return stt.Gen(seed=seed, stream=stream, min_len=L, dtau_max=D)


def _score_both(ctx, stt, m, **kw):
    out = {}
    for path in (stt.PATH_DIRECT, stt.PATH_SLAB, stt.PATH_WAVE):
        ctx.set_path(path)
        snr, key = ctx.score(m, **kw)
        out[path] = (snr.cpu().numpy().astype(np.float64), key_to_host(key))
    ctx.set_path(stt.PATH_AUTO)
    return out


# ----------------------------------------------------------------------------- generator

@pytest.mark.parametrize("T,F,L,D,seed,stream,first,n", [
    (100, 128, 10, D10MS, 1, 0, 0, 10000),
    (1000, 1000, 10, D10MS, 2, 7, 123456, 5003),
    (2896, 32767, 2, (1 << 30) - 1, 2 ** 63 + 5, 2 ** 32 - 1, 2 ** 32 - 777, 777),
    (12, 4, 12, 0, 9, 1, 0, 1),
])
def test_make_tracks_bit_exact(orc, stt, ctx, T, F, L, D, seed, stream, first, n):
    _say("make_tracks", T, F, L, D, first, n)
    g = _gen(stt, seed, stream, L, D)
    got = ctx.make_tracks(g, T, F, first, n).cpu().numpy()
    want = orc.draw_many(seed, stream, first, n, T, F, L, D)
    for k, name in enumerate(orc.TRACK_DTYPE.names):
        assert np.array_equal(got[:, k].astype(np.int64), want[name].astype(np.int64)), name


# ----------------------------------------------------------------------------- plain map (configuration 1)

def test_config1_plain_map_full(orc, stt, ctx):
    """T=100 x F=128, sigma = 1, 10^4 tracks, Philox seed 1: every score and the argmax."""
    _say("config1")
    T, F, n = 100, 128, 10_000
    Y, s = synth.noise_map(T, F, seed=1001, sigma="unit")
    m = stt.Map(*to_dev(Y, s))
    z_orc = orc.score_gen(orc.Map(Y, s), 1, 0, 10, D10MS, 0, n)
    for path, (z, key) in _score_both(ctx, stt, m, gen=_gen(stt), n=n).items():
        assert_close(z, z_orc, what=f"path {path}")
        zk, jk = stt.key_decode(key)
        assert_argmax(jk, z_orc)
        assert zk == np.float32(z[jk])
    res = list(_score_both(ctx, stt, m, gen=_gen(stt), n=n).values())
    # every scorer walks each template in the same order with the same partial-sum grid
    for other in res[1:]:
        assert np.array_equal(res[0][0], other[0]) and res[0][1] == other[1]


def test_norm_n_is_mean(orc, stt, ctx):
    _say("norm N")
    T, F, n = 64, 40, 6000
    Y, s = synth.noise_map(T, F, seed=5, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    z_orc = orc.score_gen(orc.Map(Y, s), 3, 0, 10, D10MS, 0, n, norm=orc.NORM_N)
    for path, (z, key) in _score_both(ctx, stt, m, gen=_gen(stt, 3), n=n, norm=stt.NORM_N).items():
        assert_close(z, z_orc, what=f"path {path}")
        assert_argmax(stt.key_decode(key)[1], z_orc)


@pytest.mark.parametrize("lds", [1024, 2048, 160 * 1024])
def test_slab_boundaries_and_ragged_tail(orc, stt, ctx, lds):
    """Slabs of 1, 3 and 64 columns (616 B per column of 77 rows); n spans several
    workgroups with a ragged tail; first > 0."""
    _say("slabs", lds)
    T, F, n, first = 301, 77, 3 * 1024 + 37, 12345
    Y, s = synth.noise_map(T, F, seed=77, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    z_orc = orc.score_gen(orc.Map(Y, s), 4, 2, 10, D10MS, first, n)
    ctx.set_path(stt.PATH_SLAB, lds)
    snr, key = ctx.score(m, gen=_gen(stt, 4, 2), first=first, n=n)
    ctx.set_path(stt.PATH_AUTO, 160 * 1024)
    assert_close(snr.cpu().numpy(), z_orc, what="slab")
    zk, jk = stt.key_decode(key_to_host(key))
    assert_argmax(jk - first, z_orc)


SHAPES = [(1024, 4), (512, 4), (256, 4), (1024, 2), (512, 2)]


@pytest.mark.parametrize("wg,tpt", SHAPES)
def test_every_slab_shape(orc, stt, ctx, wg, tpt):
    """Each compiled (workgroup, templates per lane) shape of the slab scorer, on a map whose
    width leaves a ragged staging walk (F=333) and a call that ends in a partial workgroup."""
    _say("shape", wg, tpt)
    T, F, n, first = 257, 333, 9000, 77
    Y, s = synth.noise_map(T, F, seed=90, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    z_orc = orc.score_gen(orc.Map(Y, s), 21, 4, 10, D10MS, first, n)
    ctx.set_path(stt.PATH_SLAB)
    ctx.set_slab_shape(wg, tpt)
    try:
        snr, key = ctx.score(m, gen=_gen(stt, 21, 4), first=first, n=n)
    finally:
        ctx.set_slab_shape(1024, 4)
        ctx.set_path(stt.PATH_AUTO)
    assert_close(snr.cpu().numpy(), z_orc, what=f"shape {wg}x{tpt}")
    assert_argmax(stt.key_decode(key_to_host(key))[1] - first, z_orc)


def test_explicit_tracks_and_invalid_ones(orc, stt, ctx):
    import torch
    _say("explicit")
    T, F = 90, 33
    Y, s = synth.noise_map(T, F, seed=8, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    tr = orc.draw_many(6, 0, 0, 5000, T, F, 10, D10MS)
    hi = F * 256 - 1
    edge = np.array([(0, T - 1, 0, 0, 0, 0), (0, T - 1, hi, hi, hi, D10MS), (T - 2, T - 1, 0, hi, hi, -D10MS),
                     (0, 1, hi, 0, hi, 1), (5, 60, 0, hi, 0, 12345), (40, 41, 100, 200, 300, -7)],
                    dtype=orc.TRACK_DTYPE)
    bad = np.array([(-1, 10, 0, 0, 0, 0), (5, 5, 0, 0, 0, 0), (3, T, 0, 0, 0, 0), (0, 20, F * 256, 0, 0, 0),
                    (9, 4, 0, 0, 0, 0)], dtype=orc.TRACK_DTYPE)
    allt = np.concatenate([tr, edge, bad])
    z_orc = orc.score_list(orc.Map(Y, s), allt)
    assert np.isnan(z_orc[-len(bad):]).all()
    dev = torch.from_numpy(allt.view(np.int32).reshape(-1, 6).copy()).cuda()
    for path in (stt.PATH_DIRECT, stt.PATH_SLAB, stt.PATH_WAVE):
        ctx.set_path(path)
        snr, key = ctx.score(m, tracks=dev, first=100)
        assert_close(snr.cpu().numpy(), z_orc, what=f"explicit path {path}")
        assert_argmax(stt.key_decode(key_to_host(key))[1] - 100, z_orc)
    ctx.set_path(stt.PATH_AUTO)


# ----------------------------------------------------------------------------- search-scale map (configuration 2)

def _config2_map(T=1000, F=1000):
    Y, s = synth.noise_map(T, F, seed=1002, sigma=("loguniform", 0.5, 2.0))
    cols, rows = synth.bezier_rows_float(200, 799, 250.5, 600.25, 450.75)
    dt0 = int(round(0.003 / 2.0 ** -28))
    f_hz = 100.0 + rows
    synth.add_pixels(Y, s, cols, rows, 8.0 / math.sqrt(cols.size), -(f_hz * dt0 * 2.0 ** -28))
    return Y, s


def test_config2_reduced_full_oracle(orc, stt, ctx):
    """T=F=1000, log-uniform sigma, one injection; 2e5 tracks scored by both sides in full."""
    _say("config2 reduced")
    n = 200_000
    Y, s = _config2_map()
    m = stt.Map(*to_dev(Y, s))
    z_orc = orc.score_gen(orc.Map(Y, s), 2, 0, 10, D10MS, 0, n)
    snr, key = ctx.score(m, gen=_gen(stt, 2), n=n)
    assert_close(snr.cpu().numpy(), z_orc, what="config2 reduced")
    assert_argmax(stt.key_decode(key_to_host(key))[1], z_orc)


def test_config2_full_scale_full_oracle(orc, stt, ctx, tmp_path):
    """10^7 tracks in the benchmark's launch configuration (its map, seed and tuned slab shape),
    every score against the oracle (run over disjoint template ranges on the host cores) and the
    GPU's argmax against the oracle's argmax over all 10^7 (Sec. III: the maximum over every
    template; Sec. V: one maximum per spectrogram)."""
    import time
    from oracle import shard
    n = 10_000_000
    Y, s = _config2_map()
    m = stt.Map(*to_dev(Y, s))
    choice = ctx.autotune(m, _gen(stt, 2), n, bench_tuning_copy(tmp_path))
    _say("config2 full, slab shape", choice)
    snr, key = ctx.score(m, gen=_gen(stt, 2), n=n)
    ctx.set_slab_shape(1024, 4)
    ctx.set_path(stt.PATH_AUTO, 160 * 1024)
    z = snr.cpu().numpy()
    zk, jk = stt.key_decode(key_to_host(key))
    # the key is the argmax of the score array (lowest index among equal scores)
    assert jk == int(np.argmax(z)) and zk == z[jk]
    t = time.time()
    z_orc = shard.score_gen(orc.Map(Y, s), 2, 0, 10, D10MS, 0, n)
    _say(f"  oracle: 10^7 templates in {time.time() - t:.1f} s on {shard.host_threads()} threads")
    assert_close(z, z_orc, what="config2 full scale")
    assert_argmax(jk, z_orc)


# ----------------------------------------------------------------------------- reductions and run combination

def test_split_runs_merge_to_one_run(stt, ctx):
    """Sec. V: maxima of runs over disjoint ranges (or seeds) combine into the single-run maximum."""
    _say("split runs")
    import torch
    T, F = 400, 300
    Y, s = synth.noise_map(T, F, seed=12, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    g = _gen(stt, 5)
    _, whole = ctx.score(m, gen=g, n=300_000, snr=None)
    merged = torch.zeros(1, dtype=torch.int64, device="cuda")
    for a, b in [(0, 12345), (12345, 200_000), (200_000, 300_000)]:
        ctx.score(m, gen=g, first=a, n=b - a, snr=None, best_key=merged)
    assert key_to_host(whole) == key_to_host(merged)
    # determinism: the same call twice gives identical scores
    z1, k1 = ctx.score(m, gen=g, n=50_000)
    z2, k2 = ctx.score(m, gen=g, n=50_000)
    assert torch.equal(z1, z2) and key_to_host(k1) == key_to_host(k2)


def test_argmax_entry_point(stt, ctx):
    import torch
    _say("argmax")
    z = np.random.default_rng(4).standard_normal(1_000_003).astype(np.float32)
    z[[1000, 2000]] = z.max() + 1
    z[[5, 77, 999_999]] = np.float32(np.nan)
    key = ctx.argmax(torch.from_numpy(z).cuda(), first=10)
    zk, jk = stt.key_decode(key_to_host(key))
    assert jk == 1010 and zk == z[1000]
    allnan = torch.full((1000,), float("nan"), device="cuda")
    zk, jk = stt.key_decode(key_to_host(ctx.argmax(allnan)))
    assert math.isinf(zk) and zk < 0 and jk == 0


# ----------------------------------------------------------------------------- degenerate and extreme shapes

def test_degenerate_cases(orc, stt, ctx):
    import torch
    _say("degenerate")
    # n = 0 is a no-op
    Y, s = synth.noise_map(30, 8, seed=3)
    m = stt.Map(*to_dev(Y, s))
    key = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.score(m, gen=_gen(stt), n=0, snr=None, best_key=key)
    assert key_to_host(key) == 0
    om = orc.Map(Y, s)
    # L = T: a single possible extent; dtau_max = 0 (targeted, Eq. 5); F = 1
    for (T, F, L, D) in [(30, 8, 30, D10MS), (30, 8, 2, 0)]:
        z_orc = orc.score_gen(om, 8, 0, L, D, 0, 5000)
        for path, (z, k) in _score_both(ctx, stt, m, gen=_gen(stt, 8, 0, L, D), n=5000).items():
            assert_close(z, z_orc, what=f"T={T} L={L} D={D} path {path}")
    Y1, s1 = synth.noise_map(50, 1, seed=4)
    m1 = stt.Map(*to_dev(Y1, s1))
    z_orc = orc.score_gen(orc.Map(Y1, s1), 1, 0, 10, D10MS, 0, 4096)
    for path, (z, k) in _score_both(ctx, stt, m1, gen=_gen(stt), n=4096).items():
        assert_close(z, z_orc, what=f"F=1 path {path}")


def test_largest_map_duration_and_index_range(orc, stt, ctx):
    _say("largest T")
    T, F = 2896, 64
    Y, s = synth.noise_map(T, F, seed=6, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    first = 2 ** 32 - 6000
    z_orc = orc.score_gen(orc.Map(Y, s), 11, 3, 2, D10MS, first, 6000)
    for path, (z, k) in _score_both(ctx, stt, m, gen=_gen(stt, 11, 3, 2), first=first, n=6000).items():
        assert_close(z, z_orc, what=f"T=2896 path {path}")
        assert_argmax(stt.key_decode(k)[1] - first, z_orc)


def test_brute_force_tiny_map(orc, stt, ctx):
    """Every template of a grid on a 12 x 4 map: all scores and the argmax."""
    import torch
    _say("brute force")
    T, F, L = 12, 4, 10
    Y, s = synth.noise_map(T, F, seed=41, sigma=("loguniform", 0.5, 2.0))
    fgrid = [0, 200, 300, 511, 700, 1023]
    rows = [(a, e + L - 1, f0, f1, f2, dt) for e in range(T - L + 1) for a in range(e + 1)
            for f0 in fgrid for f1 in fgrid for f2 in fgrid for dt in (-D10MS, -D10MS // 3, 0, D10MS // 2)]
    tr = np.array(rows, dtype=orc.TRACK_DTYPE)
    z_orc = orc.score_list(orc.Map(Y, s), tr)
    m = stt.Map(*to_dev(Y, s))
    dev = torch.from_numpy(tr.view(np.int32).reshape(-1, 6).copy()).cuda()
    for path in (stt.PATH_DIRECT, stt.PATH_SLAB, stt.PATH_WAVE):
        ctx.set_path(path)
        snr, key = ctx.score(m, tracks=dev)
        assert_close(snr.cpu().numpy(), z_orc, what=f"brute path {path}")
        assert_argmax(stt.key_decode(key_to_host(key))[1], z_orc)
    ctx.set_path(stt.PATH_AUTO)


def test_matched_injection_recovers_amplitude(orc, stt, ctx):
    """A noise-free map holding one injection matched to a template scores its amplitude (8)."""
    import torch
    _say("injection")
    T, F = 300, 200
    tr = orc.draw_many(17, 0, 0, 3, T, F, 10, D10MS)
    s = np.exp(np.random.default_rng(0).uniform(np.log(0.5), np.log(2.0), (T, F))).astype(np.float32)
    dev = torch.from_numpy(tr.view(np.int32).reshape(-1, 6).copy()).cuda()
    for i, t in enumerate(tr):
        Y = np.zeros((T, F), dtype=np.complex64)
        r = orc.rows(t, F)
        cols = np.arange(int(t["t0"]), int(t["t2"]) + 1)
        fq4 = 1600 + 16 * r.astype(np.int64)
        synth.add_pixels(Y, s, cols, r, 8.0 / math.sqrt(cols.size), -(fq4 * int(t["dtau"])) / 2.0 ** 32)
        m = stt.Map(*to_dev(Y, s))
        snr, _ = ctx.score(m, tracks=dev)
        z = snr.cpu().numpy()
        assert_close(z, orc.score_list(orc.Map(Y, s), tr))
        assert z[i] == pytest.approx(8.0, abs=1e-4)


# ----------------------------------------------------------------------------- errors

def test_argument_errors_write_nothing(stt, ctx):
    import torch
    _say("errors")
    Y, s = synth.noise_map(20, 8, seed=3)
    m = stt.Map(*to_dev(Y, s))
    key = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(stt.SttError) as e:
        ctx.score(m, gen=stt.Gen(min_len=1), n=10, snr=None, best_key=key)
    assert e.value.status == stt.ERANGE
    with pytest.raises(stt.SttError) as e:
        ctx.score(m, gen=stt.Gen(min_len=21), n=10, snr=None, best_key=key)
    assert e.value.status == stt.ERANGE
    with pytest.raises(stt.SttError) as e:
        ctx.score(m, gen=stt.Gen(), first=2 ** 32 - 5, n=10, snr=None, best_key=key)
    assert e.value.status == stt.ERANGE
    with pytest.raises(stt.SttError) as e:
        ctx.score(m, gen=stt.Gen(), n=10, norm=7, snr=None, best_key=key)
    assert e.value.status == stt.EINVAL
    with pytest.raises(stt.SttError) as e:
        ctx.make_tracks(stt.Gen(), 3000, 10, 0, 4)
    assert e.value.status == stt.ERANGE
    wide = stt.Map(*to_dev(*synth.noise_map(4, 21000, seed=1)))  # 168 KB per column
    ctx.set_path(stt.PATH_SLAB)
    with pytest.raises(stt.SttError) as e:
        ctx.score(wide, gen=stt.Gen(min_len=2), n=10, snr=None, best_key=key)
    assert e.value.status == stt.EUNSUPPORTED
    ctx.set_path(stt.PATH_AUTO)
    torch.cuda.synchronize()
    assert key_to_host(key) == 0


@pytest.mark.parametrize("F", [1000, 1024, 77, 4000])
def test_dma_and_register_staging_identical(orc, stt, ctx, F):
    """The folded-map LDS-DMA staging and the register staging give bit-identical scores
    (same p = Y/sigma bits, same walk); checked on one map against the oracle too."""
    import torch
    _say("staging", F)
    T, n = 260, 30_000
    Y, s = synth.noise_map(T, F, seed=F, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    g = _gen(stt, 12, 1)
    ctx.set_path(stt.PATH_SLAB)
    res = []
    for dma in (True, False):
        ctx.set_staging(dma)
        res.append(ctx.score(m, gen=g, n=n))
    ctx.set_staging(True)
    ctx.set_path(stt.PATH_AUTO)
    assert torch.equal(res[0][0], res[1][0]) and key_to_host(res[0][1]) == key_to_host(res[1][1])
    if F == 1000:
        z_orc = orc.score_gen(orc.Map(Y, s), 12, 1, 10, D10MS, 0, n)
        assert_close(res[0][0].cpu().numpy(), z_orc, what="dma staging")
    # batches: folded maps of several widths against register-staged ones
    maps = [m, stt.Map(*to_dev(*synth.noise_map(150, F, seed=F + 1)))]
    keys = []
    for dma in (True, False):
        ctx.set_staging(dma)
        keys.append(ctx.score_batch(maps, g, [20_000, 9_999]).clone())
    ctx.set_staging(True)
    assert torch.equal(keys[0], keys[1])


# The slab scorers take templates in the order of the two-pass bucket sort; the direct
# scorer takes them in index order. Their arithmetic is the same, so every template's score
# and the best key must agree bit for bit. The outputs start as a NaN payload that no scorer
# writes: a template the sort lost would keep it.
SENTINEL = np.uint32(0x7FBADBAD)


def _slab_and_direct(stt, ctx, m, count, **kw):
    import torch
    out = {}
    for path in (stt.PATH_DIRECT, stt.PATH_SLAB):
        ctx.set_path(path)
        snr = torch.from_numpy(np.full(count, SENTINEL, dtype=np.uint32).view(np.float32)).cuda()
        _, key = ctx.score(m, snr=snr, **kw)
        out[path] = (snr.cpu().numpy().view(np.uint32), key_to_host(key))
    ctx.set_path(stt.PATH_AUTO)
    d, sl = out[stt.PATH_DIRECT], out[stt.PATH_SLAB]
    assert not (d[0] == SENTINEL).any() and not (sl[0] == SENTINEL).any(), "templates left unscored"
    assert np.array_equal(sl[0], d[0])
    assert sl[1] == d[1]


@pytest.mark.parametrize("T,n,L", [
    (1000, 10_000_000, 10),   # the search map: 7875 buckets, 124 groups, 1221 sort chunks
    (1000, 3 * 8192, 10),     # whole sort chunks; 36 buckets of 128 columns
    (1024, 3_000_001, 10),    # 128 buckets per axis: the full 8256 buckets, 129 groups
    (130, 65537, 120),        # templates of at least 120 of 130 columns: most buckets empty
    (2000, 1_048_577, 500),   # a ragged tail of one template
])
def test_bucket_sort_slab_equals_direct(stt, ctx, T, n, L):
    _say("sort", T, n, L)
    F = 64
    Y, s = synth.noise_map(T, F, seed=T + L, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    _slab_and_direct(stt, ctx, m, n, gen=_gen(stt, seed=T + 3, stream=1, L=L), n=n)


def test_bucket_sort_explicit_tracks_slab_equals_direct(stt, ctx):
    """The sort of a given template list (buckets from the records, invalid records in bucket 0)."""
    import torch
    _say("sort explicit")
    T, F, n = 700, 90, 200_003
    Y, s = synth.noise_map(T, F, seed=5, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    tracks = ctx.make_tracks(_gen(stt, seed=8, stream=3), T, F, 0, n)
    tracks[torch.arange(0, n, 97, device=tracks.device), 1] = T + 5  # t2 past the map: invalid
    _slab_and_direct(stt, ctx, m, n, tracks=tracks)
