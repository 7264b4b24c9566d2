"""GPU parity of the sky-patch delay prior (Sec. VI): generated templates whose delays are uniform
on [c - D, c + D] -- bit-identical to the oracle's draw, scored within the tolerance on every path,
and the same in a batch as per map."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synth
from tests.parity_util import assert_argmax, assert_close, key_to_host, to_dev

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


@pytest.mark.parametrize("center,D", [(0, D10MS), (-1_000_000, 300_000), (2 ** 30 - 1 - D10MS, D10MS), (77, 0)])
def test_patch_draw_bit_identical(orc, stt, ctx, center, D):
    _say("patch draw", center, D)
    g = stt.Gen(seed=12, stream=3, min_len=10, dtau_max=D, dtau_center=center)
    tr = ctx.make_tracks(g, 400, 150, 1000, 5000).cpu().numpy()
    want = orc.draw_patch_many(12, 3, 1000, 5000, 400, 150, 10, D, center)
    got = tr.view(orc.TRACK_DTYPE).reshape(-1)
    for name in orc.TRACK_DTYPE.names:
        assert np.array_equal(got[name], want[name]), name


@pytest.mark.parametrize("path", [0, 1, 2, 3])
def test_patch_scores_match_oracle(orc, stt, ctx, path):
    _say("patch scores, path", path)
    T, F, n = 300, 200, 20_000
    Y, s = synth.noise_map(T, F, seed=81, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    c, D = 805_306, 134_218  # a band around 3 ms, +-0.5 ms
    g = stt.Gen(seed=5, stream=0, min_len=10, dtau_max=D, dtau_center=c)
    ctx.set_path(path)
    z, key = ctx.score(m, gen=g, n=n)
    ctx.set_path(0)
    tracks = orc.draw_patch_many(5, 0, 0, n, T, F, 10, D, c)
    z_orc = orc.score_list(orc.Map(Y, s), tracks)
    assert_close(z.cpu().numpy(), z_orc, what=f"patch path {path}")
    assert_argmax(stt.key_decode(key_to_host(key))[1], z_orc)


def test_patch_batch_equals_per_map(stt, ctx):
    _say("patch batch")
    import torch
    maps = []
    for k, T in enumerate((200, 450, 333)):
        Y, s = synth.noise_map(T, 120, seed=82, sigma=("loguniform", 0.5, 2.0), stream=k)
        maps.append(stt.Map(*to_dev(Y, s)))
    g = stt.Gen(seed=6, stream=10, min_len=10, dtau_max=50_000, dtau_center=-400_000)
    ns = [7000, 12000, 9000]
    keys = ctx.score_batch(maps, g, ns).cpu().numpy().view(np.uint64).tolist()
    for k, m in enumerate(maps):
        gk = stt.Gen(seed=6, stream=10 + k, min_len=10, dtau_max=50_000, dtau_center=-400_000)
        _, kk = ctx.score(m, gen=gk, n=ns[k])
        assert keys[k] == key_to_host(kk)
    assert torch.cuda.is_available()


def test_patch_outside_delay_range(stt, ctx):
    g = stt.Gen(seed=1, min_len=10, dtau_max=D10MS, dtau_center=2 ** 30 - D10MS)
    with pytest.raises(stt.SttError) as e:
        ctx.make_tracks(g, 100, 50, 0, 10)
    assert e.value.status == stt.ERANGE
