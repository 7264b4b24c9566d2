"""GPU parity of the differentiation addition: the smooth statistic, its hand-written
gradient, the autograd binding and the projected-ascent refinement."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import synth
from tests.parity_util import assert_smooth_close, smooth_fp32_bound, assert_close, to_dev

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


def _thetas(T, F, n, seed):
    sel = np.random.default_rng(seed)
    K = sel.integers(10, min(T, 300), n).astype(np.int32)
    a = sel.uniform(-5, T - 5, n)
    th = np.stack([a, a + K + sel.uniform(-3, 30, n), *sel.uniform(-2, F + 1, (3, n)),
                   sel.uniform(-12, 12, n)], axis=1).astype(np.float32)
    return th, K


def test_tracks_at_and_theta(orc, stt, ctx):
    import torch
    _say("tracks_at")
    idx = np.array([0, 5, 2 ** 32 - 1, 123456789, 77], dtype=np.int64)
    g = stt.Gen(seed=8, stream=3, min_len=10, dtau_max=D10MS)
    tr = ctx.tracks_at(g, 900, 700, torch.from_numpy(idx).cuda()).cpu().numpy()
    for i, j in enumerate(idx):
        assert tuple(tr[i]) == tuple(int(x) for x in orc.draw(8, 3, int(j), 900, 700, 10, D10MS).tolist())
    th, K = ctx.tracks_to_theta(torch.from_numpy(tr).cuda())
    th, K = th.cpu().numpy(), K.cpu().numpy()
    assert np.array_equal(K, tr[:, 1] - tr[:, 0] + 1)
    assert np.array_equal(th[:, 0], tr[:, 0].astype(np.float32))
    assert np.array_equal(th[:, 2], (tr[:, 2].astype(np.float64) / 256).astype(np.float32))
    assert np.allclose(th[:, 5], tr[:, 5] * 2.0 ** -28 * 1e3, rtol=1e-7)


@pytest.mark.parametrize("p16", [False, True])
def test_smooth_and_gradient_match_oracle(orc, stt, ctx, p16):
    import torch
    _say("smooth/grad", p16)
    T, F, n = 400, 250, 600
    Y, s = synth.noise_map(T, F, seed=41, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    if p16:
        m = ctx.pack_p16(m)
        _, _, deq = orc.quantize_p16(Y, s)
        om = orc.Map(deq, np.ones((T, F)))
    else:
        om = orc.Map(Y, s)
    th, K = _thetas(T, F, n, 3)
    z, g = ctx.grad(m, torch.from_numpy(th).cuda(), torch.from_numpy(K).cuda())
    z_only = ctx.smooth(m, torch.from_numpy(th).cuda(), torch.from_numpy(K).cuda())
    assert torch.equal(z, z_only)
    z, g = z.cpu().numpy(), g.cpu().numpy()
    zo = np.empty(n)
    go = np.empty((n, 6))
    for i in range(n):
        zo[i], go[i] = orc.smooth(om, th[i].astype(np.float64), int(K[i]))
    pm = deq if p16 else Y.astype(np.complex128) / s
    dmax = assert_smooth_close(z, zo, pm, th, K, what="smooth z")
    _say(f"smooth z max |dz| {dmax:.2e}")
    err = np.abs(g - go) / np.maximum(1.0, np.abs(go))
    assert err.max() < 2e-4, err.max()


def test_autograd_backward_is_the_gradient_kernel(stt, ctx):
    import torch
    from paper_1401_8060_amd.autograd import smooth_snr
    _say("autograd")
    T, F, n = 200, 150, 64
    Y, s = synth.noise_map(T, F, seed=42)
    m = stt.Map(*to_dev(Y, s))
    th, K = _thetas(T, F, n, 4)
    theta = torch.from_numpy(th).cuda().requires_grad_(True)
    Kt = torch.from_numpy(K).cuda()
    w = torch.linspace(-1, 2, n, device="cuda")
    z = smooth_snr(ctx, m, theta, Kt)
    (w * z).sum().backward()
    z2, g = ctx.grad(m, theta.detach(), Kt)
    assert torch.equal(z.detach(), z2)
    assert torch.allclose(theta.grad, w[:, None] * g, rtol=0, atol=0)


def test_refine_invariants_and_plain_rescore(orc, stt, ctx):
    import torch
    _say("refine")
    T, F, n, L = 300, 200, 256, 10
    Y, s = synth.noise_map(T, F, seed=43, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    om = orc.Map(Y, s)
    g = stt.Gen(seed=6, min_len=L, dtau_max=D10MS)
    tr0 = ctx.make_tracks(g, T, F, 0, n)
    th0, K = ctx.tracks_to_theta(tr0)
    z0 = ctx.smooth(m, th0, K)
    th, zs, tr, zp = ctx.refine(m, th0, K, L, D10MS, steps=50)
    th_h, zs_h, tr_h, zp_h = th.cpu().numpy(), zs.cpu().numpy(), tr.cpu().numpy(), zp.cpu().numpy()
    # the steps read the folded p, stt_smooth forms Y/sigma at each gather: the same values bit for bit
    assert torch.equal(zs, ctx.smooth(m, th, K))
    assert (zs_h >= z0.cpu().numpy() - 1e-6).all()
    assert (th_h[:, 0] >= 0).all() and (th_h[:, 1] <= T - 1).all() and (th_h[:, 1] - th_h[:, 0] >= L - 1 - 1e-4).all()
    assert (th_h[:, 2:5] >= 0).all() and (th_h[:, 2:5] < F).all() and (np.abs(th_h[:, 5]) <= 10.0 + 1e-5).all()
    # the kept iterate's z~ is the smooth statistic at the returned theta
    zo = np.array([orc.smooth(om, th_h[i].astype(np.float64), int(K[i]))[0] for i in range(n)])
    assert_smooth_close(zs_h, zo, Y.astype(np.complex128) / s, th_h, K.cpu().numpy(), what="best z~")
    # rounding to plain templates and their plain scores, exactly as the oracle defines them
    K_h = K.cpu().numpy()
    for i in range(n):
        want = orc.theta_to_track(th_h[i].astype(np.float64), T, F, L, D10MS)
        assert tuple(tr_h[i]) == tuple(int(x) for x in want.tolist())
    assert_close(zp_h, orc.score_list(om, tr_h.view(orc.TRACK_DTYPE).reshape(-1)), what="plain rescore")
    gain = zs_h - z0.cpu().numpy()
    _say(f"refine: mean z~ gain {gain.mean():.3f}, max {gain.max():.3f}")
    assert gain.mean() > 0.1


def test_refine_on_an_fp16_map(orc, stt, ctx):
    """Refinement on an FP16 map: the best z~ is stt_smooth's at the returned theta (bit for bit)
    and the oracle's on the dequantised map; the plain re-score matches the oracle there too."""
    import torch
    _say("refine fp16")
    T, F, n, L = 250, 180, 128, 10
    Y, s = synth.noise_map(T, F, seed=44, sigma=("loguniform", 0.5, 2.0))
    m16 = ctx.pack_p16(stt.Map(*to_dev(Y, s)))
    _, _, deq = orc.quantize_p16(Y, s)
    om = orc.Map(deq, np.ones((T, F)))
    g = stt.Gen(seed=8, min_len=L, dtau_max=D10MS)
    th0, K = ctx.tracks_to_theta(ctx.make_tracks(g, T, F, 0, n))
    th, zs, tr, zp = ctx.refine(m16, th0, K, L, D10MS, steps=30)
    assert torch.equal(zs, ctx.smooth(m16, th, K))
    th_h, K_h = th.cpu().numpy(), K.cpu().numpy()
    zo = np.array([orc.smooth(om, th_h[i].astype(np.float64), int(K_h[i]))[0] for i in range(n)])
    assert_smooth_close(zs.cpu().numpy(), zo, deq, th_h, K_h, what="fp16 best z~")
    assert_close(zp.cpu().numpy(), orc.score_list(om, tr.cpu().numpy().view(orc.TRACK_DTYPE).reshape(-1)),
                 what="fp16 plain rescore")


def test_refine_recovers_an_injection(orc, stt, ctx):
    """Noise-free map, one injected straight track: from a start a few pixels and 1 ms off,
    the GPU refinement ends within a pixel and 0.1 ms of it, like the oracle's."""
    import torch
    _say("refine injection")
    T, F = 100, 80
    Y = np.zeros((T, F), dtype=np.complex64)
    s = np.ones((T, F), dtype=np.float32)
    t0, t2, r0, r2, dt0 = 20, 79, 30.5, 50.5, 2.0
    k = np.arange(t2 - t0 + 1)
    rows = np.floor(r0 + (r2 - r0) * k / (t2 - t0)).astype(int)
    synth.add_pixels(Y, s, t0 + k, rows, 1.0, -(100.0 + rows) * dt0 * 1e-3)
    m = stt.Map(*to_dev(Y, s))
    th0 = np.array([[t0 + 1.5, t2 - 1.0, r0 + 1.5, 0.5 * (r0 + r2) - 1.0, r2 + 1.2, dt0 + 1.0]], dtype=np.float32)
    K = np.array([t2 - t0 + 1], dtype=np.int32)
    th, zs, _, _ = ctx.refine(m, torch.from_numpy(th0).cuda(), torch.from_numpy(K).cuda(), 10, D10MS, steps=50)
    th = th.cpu().numpy()[0]
    tho, zo = orc.refine(orc.Map(Y, s), th0[0].astype(np.float64), int(K[0]), 50, 10, 10.0)
    assert abs(th[5] - dt0) < 0.1 and np.abs(th[2:5] - [r0, 0.5 * (r0 + r2), r2]).max() < 1.0
    assert float(zs.item()) == pytest.approx(zo, rel=0.02)


# ---------------------------------------------------------------- the ascent step by step

DMS = D10MS * 1e3 / 2 ** 28  # the delay bound in ms, as the library converts it


def _clear_trace(orc, om, trace, K, first, delta=2e-4, dz=1e-4, dg=1e-3):
    """True when the oracle's trajectory has no near-decision for FP32 rounding to flip: samples
    of iterates >= first lie more than delta (px) from every grid line (where the bilinear
    gradient jumps), the delay derivative and the position gradient are clearly nonzero before
    each step (sign step, normalisation), and z~ rises by more than dz at every step (so the best
    iterate is the last)."""
    xi = np.arange(K) / (K - 1)
    b = np.stack([(1 - xi) ** 2, 2 * xi * (1 - xi), xi ** 2])
    for s, row in enumerate(trace):
        th = row[:6]
        if s >= first:
            u = th[0] + xi * (th[1] - th[0])
            v = b.T @ th[2:5] - 0.5
            if (np.abs(u - np.round(u)) <= delta).any() or (np.abs(v - np.round(v)) <= delta).any():
                return False
        if s < len(trace) - 1:
            _, g = orc.smooth(om, th, K)
            if abs(g[5]) <= dg or np.linalg.norm(g[:5]) <= 1e-2 or trace[s + 1][6] <= row[6] + dz:
                return False
    return True


@pytest.mark.parametrize("start", ["plain", "offgrid"])
def test_refine_step_by_step_matches_oracle(orc, stt, ctx, start):
    """k_refine after 1, 2 and 3 ascent steps against the oracle's iterates (each run has its own
    linear schedule: steps=1 moves 1 px and 0.5 ms; steps=2 moves 1 then 0.02 px; steps=3 1, 0.51,
    0.02). On templates whose trajectory has no near-decision (see _clear_trace) the returned
    point is the last iterate, and theta matches the oracle's to 1e-5 * max(1, |x|). z~ is checked
    at the returned point against the oracle's smooth statistic there (the FP32 forward bound of
    assert_smooth_close), and against the oracle's last iterate within that bound plus the first-
    order change of z~ over the two points' difference (|grad| . |d theta|, with a factor 2).
    'plain' starts from drawn templates (integer times: every start sample sits on a grid line,
    where both sides take the cell floor(u) of the same FP64 position); 'offgrid' from random
    real points."""
    import torch
    T, F, L, n = 200, 150, 10, 3000
    Y, s = synth.noise_map(T, F, seed=45, sigma=("loguniform", 0.5, 2.0))
    m = stt.Map(*to_dev(Y, s))
    om = orc.Map(Y, s)
    if start == "plain":
        tr = orc.draw_many(9, 0, 0, n, T, F, L, D10MS)
        th0 = np.stack([tr["t0"], tr["t2"], tr["f0"] / 256.0, tr["f1"] / 256.0, tr["f2"] / 256.0,
                        tr["dtau"] * (1e3 / 2 ** 28)], axis=1).astype(np.float32)
        K = (tr["t2"] - tr["t0"] + 1).astype(np.int32)
        first = 1
    else:
        sel = np.random.default_rng(3)
        K = sel.integers(10, 120, n).astype(np.int32)
        a = sel.uniform(0, T - 130, n)
        th0 = np.stack([a, a + K - 1 + sel.uniform(0, 8, n), *sel.uniform(1, F - 1, (3, n)),
                        sel.uniform(-9, 9, n)], axis=1).astype(np.float32)
        first = 0
    for steps in (1, 2, 3):
        _say(f"refine steps={steps} start={start}")
        th, zs, _, _ = ctx.refine(m, torch.from_numpy(th0).cuda(), torch.from_numpy(K).cuda(), L, D10MS,
                                  steps=steps, plain=False)
        th, zs = th.cpu().numpy().astype(np.float64), zs.cpu().numpy().astype(np.float64)
        picked = []
        for i in range(n):
            _, _, trc = orc.refine_trace(om, th0[i].astype(np.float64), int(K[i]), steps, L, DMS)
            if _clear_trace(orc, om, trc, int(K[i]), first):
                picked.append((i, trc[-1]))
        assert len(picked) >= 1000, len(picked)
        idx = np.array([i for i, _ in picked])
        want = np.array([r for _, r in picked])
        d_th = np.abs(th[idx] - want[:, :6]) / np.maximum(1.0, np.abs(want[:, :6]))
        _say(f"  {len(idx)} clear trajectories: max theta err {d_th.max():.2e}, "
             f"max z err {np.max(np.abs(zs[idx] - want[:, 6]) / np.maximum(1.0, np.abs(want[:, 6]))):.2e}")
        assert d_th.max() <= 1e-5, (int(idx[np.argmax(d_th.max(axis=1))]), d_th.max())
        p = Y.astype(np.complex128) / s
        z_at = np.array([orc.smooth(om, th[i], int(K[i]), grad=False)[0] for i in idx])
        assert_smooth_close(zs[idx], z_at, p, th[idx], K[idx], what=f"z~ at the returned point, {steps} steps")
        prop = np.array([2.0 * np.abs(orc.smooth(om, want[j, :6], int(K[i]))[1]) @ np.abs(th[i] - want[j, :6])
                         for j, i in enumerate(idx)])
        lim = np.array([1e-5 * max(1.0, abs(want[j, 6])) + smooth_fp32_bound(p, th[i], int(K[i]))
                        for j, i in enumerate(idx)]) + prop
        dz = np.abs(zs[idx] - want[:, 6])
        assert (dz <= lim).all(), (int(idx[np.argmax(dz / lim)]), float(dz.max()))
