"""stt_score_noalloc: the scoring call that takes its work memory from the library's fixed
per-device array instead of allocating. Its results are compared with stt_score's, bit for
bit (the same kernels on the same inputs), over two calls in a row, the second smaller, so
that the second call also runs over what the first one left in the array."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synth
from tests.parity_util import to_dev

pytestmark = pytest.mark.gpu
D10MS = 2684355
NA_MAX_TRACKS = 1 << 22


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


def _both(stt, ctx, m, n, gen=None, tracks=None, first=0):
    import torch
    z_ref, k_ref = ctx.score(m, gen=gen, tracks=tracks, first=first, n=n)
    z = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    k = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.score_noalloc(m, z, k, gen=gen, tracks=tracks, first=first, n=n)
    ctx.sync()
    return z_ref.cpu().numpy(), k_ref.cpu().numpy(), z.cpu().numpy(), k.cpu().numpy()


@pytest.mark.parametrize("dma", [True, False])
def test_noalloc_equals_score_on_two_calls(stt, ctx, dma):
    ctx.set_staging(dma)
    try:
        # first call: a larger map and template count (slab path, binned, folded map)
        T, F, n = 700, 600, 400_000
        _say(f"noalloc first call T={T} F={F} n={n} dma={dma}")
        Y, s = synth.noise_map(T, F, seed=31, sigma=("loguniform", 0.5, 2.0))
        m = stt.Map(*to_dev(Y, s))
        g = stt.Gen(seed=11, min_len=10, dtau_max=D10MS)
        z_ref, k_ref, z, k = _both(stt, ctx, m, n, gen=g, first=123)
        assert np.array_equal(z.view(np.uint32), z_ref.view(np.uint32))
        assert np.array_equal(k, k_ref)
        # second call, smaller: another map and fewer templates over the leftovers of the first
        T, F, n = 150, 130, 6000
        _say(f"noalloc second call T={T} F={F} n={n} dma={dma}")
        Y, s = synth.noise_map(T, F, seed=32, sigma="unit")
        m2 = stt.Map(*to_dev(Y, s))
        g2 = stt.Gen(seed=12, min_len=10, dtau_max=D10MS)
        z_ref, k_ref, z, k = _both(stt, ctx, m2, n, gen=g2)
        assert np.array_equal(z.view(np.uint32), z_ref.view(np.uint32))
        assert np.array_equal(k, k_ref)
    finally:
        ctx.set_staging(True)


def test_noalloc_given_tracks_and_small_calls(stt, ctx):
    import torch
    T, F = 300, 257
    Y, s = synth.noise_map(T, F, seed=33, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    g = stt.Gen(seed=13, min_len=10, dtau_max=D10MS)
    for n in (20_000, 100):  # slab path, then the one-wave-per-template path
        _say(f"noalloc given tracks n={n}")
        tr = ctx.make_tracks(g, T, F, 0, n)
        tr[5, 1] = T + 3  # an invalid template scores NaN on both
        z_ref, k_ref, z, k = _both(stt, ctx, m, n, tracks=tr, first=7)
        assert np.isnan(z[5]) and np.isnan(z_ref[5])
        assert np.array_equal(z.view(np.uint32), z_ref.view(np.uint32))
        assert np.array_equal(k, k_ref)
    del torch


def test_noalloc_at_its_largest_call(stt, ctx):
    """n = 4194304 templates on a map whose fold takes 31.25 MiB of the 32: the sort's
    regions reach the end of the fixed array."""
    T, F, n = 2000, 2000, NA_MAX_TRACKS
    _say(f"noalloc largest call T={T} F={F} n={n}")
    Y, s = synth.noise_map(T, F, seed=35, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    g = stt.Gen(seed=14, min_len=10, dtau_max=D10MS)
    z_ref, k_ref, z, k = _both(stt, ctx, m, n, gen=g)
    assert not np.isnan(z).any()
    assert np.array_equal(z.view(np.uint32), z_ref.view(np.uint32))
    assert np.array_equal(k, k_ref)


def test_noalloc_rejects_sizes_beyond_its_scratch(stt, ctx):
    import torch
    Y, s = synth.noise_map(100, 128, seed=34, sigma="unit")
    m = stt.Map(*to_dev(Y, s))
    g = stt.Gen(seed=1, min_len=10, dtau_max=D10MS)
    k = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(stt.SttError) as e:
        ctx.score_noalloc(m, None, k, gen=g, n=NA_MAX_TRACKS + 1)
    assert e.value.status == stt.ERANGE
    # a map whose folded copy exceeds 32 MiB: 2000 x 2100 -> 2000 x 2176 x 8 B
    Yb = torch.zeros((2000, 2100), dtype=torch.complex64, device="cuda")
    sb = torch.ones((2000, 2100), dtype=torch.float32, device="cuda")
    with pytest.raises(stt.SttError) as e:
        ctx.score_noalloc(stt.Map(Yb, sb), None, k, gen=g, n=10_000)
    assert e.value.status == stt.ERANGE
    assert int(k.item()) == 0  # nothing was enqueued
