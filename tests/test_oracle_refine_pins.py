"""Pins of the oracle's refinement rule (projected ascent of the smooth statistic), checked
against trajectories worked from closed forms, not against the oracle's own bilinear code.

The analytic map: p(t, r) = A(t, r) + i B(t, r) with A, B affine in (t, r) and integer
coefficients (exact in complex64), sigma = 1, and every row at the same frequency f (row spacing
0). Bilinear interpolation reproduces an affine function exactly, and the delay's phase factor
exp(2 pi i f dtau) is the same on every pixel, so for samples inside the map

    z~(theta) = K^-1/2 [cos(phi) SA - sin(phi) SB],   phi = 2 pi f dtau,
    SA = K a0 + a_t K (tau0 + tau2)/2 + a_r (S0 (phi0 + phi2) + S1 phi1 - K/2)   (SB alike),

with xi_k = k/(K-1), sum_k xi_k = sum_k (1 - xi_k) = K/2, S0 = sum (1-xi)^2 = sum xi^2 =
K(2K-1)/(6(K-1)) and S1 = sum 2 xi (1-xi) = K(K-2)/(3(K-1)). Its gradient is then

    d/dtau0 = d/dtau2 = K^-1/2 (K/2) (a_t cos - b_t sin),
    d/dphi0 = d/dphi2 = K^-1/2 S0 (a_r cos - b_r sin),  d/dphi1 = K^-1/2 S1 (a_r cos - b_r sin),
    d/d(dtau in ms) = -2 pi f 1e-3 K^-1/2 (sin SA + cos SB).

The rule being pinned (the build's reading of the refinement step): at step s of n, with
w = s/(n-1), the five positions move by eta_px = px0 + w (px1 - px0) along g_pos/|g_pos|
(|.| over the five positions only), the delay by eta_ms = ms0 + w (ms1 - ms0) times sign(g_dtau),
and then theta is projected; the start is projected first and the best iterate is kept. The
tests also show that each plausible slip -- the schedule run backwards, the delay inside the
position norm, a delay step proportional to its gradient, the projection taken before the move --
changes the worked trajectory far beyond the tolerance.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

A_COEF = (5.0, 1.0, 2.0)   # a0, a_t, a_r
B_COEF = (-3.0, -1.0, 1.0)  # b0, b_t, b_r
T_MAP, F_MAP = 60, 50


def _map(orc, fq4_lo, coefA=A_COEF, coefB=B_COEF):
    t = np.arange(T_MAP, dtype=np.float64)[:, None]
    r = np.arange(F_MAP, dtype=np.float64)[None, :]
    A = coefA[0] + coefA[1] * t + coefA[2] * r
    B = coefB[0] + coefB[1] * t + coefB[2] * r
    Y = (A + 1j * B).astype(np.complex64)
    assert np.array_equal(Y.real.astype(np.float64), A) and np.array_equal(Y.imag.astype(np.float64), B)
    return orc.Map(Y, np.ones((T_MAP, F_MAP), dtype=np.float32), fq4_lo=fq4_lo, dfq4=0)


def _sums(K):
    return K * (2 * K - 1) / (6 * (K - 1)), K * (K - 2) / (3 * (K - 1))


def _closed(th, K, f_hz, coefA=A_COEF, coefB=B_COEF):
    """(z~, gradient) of the affine map at theta, from the closed forms above."""
    S0, S1 = _sums(K)
    def s_of(c):
        return K * c[0] + c[1] * K * (th[0] + th[1]) / 2 + c[2] * (S0 * (th[2] + th[4]) + S1 * th[3] - K / 2)
    SA, SB = s_of(coefA), s_of(coefB)
    ph = 2 * math.pi * f_hz * th[5] * 1e-3
    c, s = math.cos(ph), math.sin(ph)
    k = 1 / math.sqrt(K)
    gt = k * K / 2 * (coefA[1] * c - coefB[1] * s)
    gr = k * (coefA[2] * c - coefB[2] * s)
    g = np.array([gt, gt, gr * S0, gr * S1, gr * S0, -2 * math.pi * f_hz * 1e-3 * k * (s * SA + c * SB)])
    return k * (c * SA - s * SB), g


def _project(th, L, dmax):
    a, b = th[0], th[1]
    if b - a < L - 1:
        mid = 0.5 * (a + b)
        a, b = mid - 0.5 * (L - 1), mid + 0.5 * (L - 1)
    if a < 0:
        b, a = b - a, 0.0
    if b > T_MAP - 1:
        a, b = a - (b - (T_MAP - 1)), float(T_MAP - 1)
    a = max(a, 0.0)
    out = np.array([a, b, *np.clip(th[2:5], 0.0, F_MAP - 2.0 ** -9), min(dmax, max(-dmax, th[5]))])
    return out


def _worked(th0, K, steps, L, dmax, f_hz, sched=(1.0, 0.02, 0.5, 0.01), slip=None, **coef):
    """Iterates (theta_s, z~_s) of the rule, worked from the closed forms; `slip` names one
    deliberate deviation from the rule."""
    th = _project(np.asarray(th0, dtype=np.float64), L, dmax)
    z, g = _closed(th, K, f_hz, **coef)
    out = [(th.copy(), z)]
    for s in range(steps):
        w = s / (steps - 1) if steps > 1 else 0.0
        if slip == "schedule_backwards":
            w = 1.0 - w
        epx = sched[0] + w * (sched[1] - sched[0])
        ems = sched[2] + w * (sched[3] - sched[2])
        if slip == "project_first":
            th = _project(th, L, dmax)
        nrm = np.linalg.norm(g if slip == "delay_in_norm" else g[:5])
        nxt = th.copy()
        nxt[:5] += epx * g[:5] / nrm
        nxt[5] += ems * g[5] if slip == "delay_proportional" else ems * np.sign(g[5])
        th = nxt if slip == "project_first" else _project(nxt, L, dmax)
        z, g = _closed(th, K, f_hz, **coef)
        out.append((th.copy(), z))
    return out


def _best(traj):
    zb, tb = traj[0][1], traj[0][0]
    for t, z in traj[1:]:
        if z > zb:
            zb, tb = z, t
    return tb, zb


def _inside(traj, K):
    """Every sample of every iterate lies strictly inside the map (no clamped coordinate)."""
    xi = np.arange(K) / (K - 1)
    for t, _ in traj:
        u = t[0] + xi * (t[1] - t[0])
        v = (1 - xi) ** 2 * t[2] + 2 * xi * (1 - xi) * t[3] + xi ** 2 * t[4] - 0.5
        if not ((u > 0) & (u < T_MAP - 1) & (v > 0) & (v < F_MAP - 1)).all():
            return False
    return True


def test_closed_forms_of_the_sample_sums():
    for K in (3, 4, 17, 300):
        xi = np.arange(K) / (K - 1)
        S0, S1 = _sums(K)
        assert ((1 - xi) ** 2).sum() == pytest.approx(S0, rel=1e-14) and (xi ** 2).sum() == pytest.approx(S0, rel=1e-14)
        assert (2 * xi * (1 - xi)).sum() == pytest.approx(S1, rel=1e-14)
        assert xi.sum() == pytest.approx(K / 2, rel=1e-14)


def test_smooth_statistic_and_gradient_on_the_affine_map(orc):
    rng = np.random.default_rng(71)
    for fq4 in (1600, 16000):
        m = _map(orc, fq4)
        for _ in range(20):
            K = int(rng.integers(3, 40))
            a = rng.uniform(1, 15)
            th = np.array([a, a + rng.uniform(K, 40), *rng.uniform(2, 45, 3), rng.uniform(-2, 2)])
            z, g = orc.smooth(m, th, K)
            zc, gc = _closed(th, K, fq4 / 16)
            assert z == pytest.approx(zc, rel=1e-12, abs=1e-10)
            np.testing.assert_allclose(g, gc, rtol=1e-11, atol=1e-10)


# A hand-worked case (f = 100 Hz, K = 3, so S0 = 5/4, S1 = 1/2; start inside every constraint).
# At theta0 = (10, 30, 12, 20, 16, 0): phi = 0, SA = 15 + 3 (40)/2 + 2 (5/4 * 28 + 10 - 3/2) = 162,
# SB = -9 - 3 (40)/2 + (5/4 * 28 + 10 - 3/2) = -25.5, so z~ = 162/sqrt(3); the position gradient
# is 3^-1/2 (3/2, 3/2, 5/2, 1, 5/2) with norm 3^-1/2 sqrt(18), the delay gradient
# -2 pi 100 1e-3 3^-1/2 (-25.5) > 0. Step 0 (eta_px = 1, eta_ms = 0.5) gives
# theta1 = theta0 + (1.5, 1.5, 2.5, 1, 2.5)/sqrt(18) + (0, 0, 0, 0, 0, 0.5).
def test_hand_worked_first_step(orc):
    m = _map(orc, 1600)
    th0 = [10.0, 30.0, 12.0, 20.0, 16.0, 0.0]
    z0, g0 = orc.smooth(m, th0, 3)
    assert z0 == pytest.approx(162 / math.sqrt(3), rel=1e-13)
    assert g0[5] == pytest.approx(2 * math.pi * 0.1 * 25.5 / math.sqrt(3), rel=1e-12)
    _, _, tr = orc.refine_trace(m, th0, 3, 2, 10, 10.0)
    want1 = np.array(th0) + np.array([1.5, 1.5, 2.5, 1.0, 2.5, 0.0]) / math.sqrt(18.0) + np.array([0, 0, 0, 0, 0, 0.5])
    np.testing.assert_allclose(tr[1, :6], want1, rtol=0, atol=1e-12)


CASES = [
    # (theta0, K, steps, L, dmax_ms, fq4_lo): interior; a delay bound that binds after a move; a start
    # shorter than L (the start's projection widens it); a high row frequency where the delay flips sign
    ((10.3, 40.7, 12.2, 20.9, 15.4, 0.12), 31, 3, 10, 10.0, 1600),
    ((8.1, 33.9, 14.6, 22.2, 19.7, 0.1), 20, 3, 10, 0.3, 1600),
    ((20.0, 24.5, 10.5, 18.0, 12.5, -0.05), 12, 2, 10, 10.0, 1600),
    ((12.6, 38.2, 16.1, 12.3, 21.0, 0.03), 25, 3, 10, 10.0, 16000),
]


@pytest.mark.parametrize("case", CASES)
def test_trajectory_matches_the_worked_one(orc, case):
    th0, K, steps, L, dmax, fq4 = case
    m = _map(orc, fq4)
    traj = _worked(th0, K, steps, L, dmax, fq4 / 16)
    assert _inside(traj, K)
    th, z, tr = orc.refine_trace(m, th0, K, steps, L, dmax)
    for s, (t, zs) in enumerate(traj):
        np.testing.assert_allclose(tr[s, :6], t, rtol=0, atol=1e-9, err_msg=f"iterate {s}")
        assert tr[s, 6] == pytest.approx(zs, rel=1e-12, abs=1e-10)
    tb, zb = _best(traj)
    np.testing.assert_allclose(th, tb, rtol=0, atol=1e-9)
    assert z == pytest.approx(zb, rel=1e-12)
    # the same through the plain entry point
    th2, z2 = orc.refine(m, th0, K, steps, L, dmax)
    assert np.array_equal(th2, th) and z2 == z


@pytest.mark.parametrize("slip", ["schedule_backwards", "delay_in_norm", "delay_proportional", "project_first"])
def test_each_slip_moves_the_worked_trajectory(slip):
    """Every deviation from the rule lands at least 1e-3 away from the rule's own iterates (the
    tolerance above is 1e-9) in at least one of the cases."""
    worst = 0.0
    for th0, K, steps, L, dmax, fq4 in CASES:
        good = _worked(th0, K, steps, L, dmax, fq4 / 16)
        bad = _worked(th0, K, steps, L, dmax, fq4 / 16, slip=slip)
        worst = max(worst, max(np.abs(a[0] - b[0]).max() for a, b in zip(good, bad)))
    assert worst > 1e-3, (slip, worst)


def test_delay_bound_binds_and_best_is_not_last(orc):
    """The second case ends with its delay on the bound (projection after the move), and the fourth
    keeps an earlier iterate: the delay overshoots at 1 kHz and the last step is not the best."""
    th0, K, steps, L, dmax, fq4 = CASES[1]
    traj = _worked(th0, K, steps, L, dmax, fq4 / 16)
    assert any(abs(t[5]) == dmax for t, _ in traj[1:])
    th0, K, steps, L, dmax, fq4 = CASES[3]
    traj = _worked(th0, K, steps, L, dmax, fq4 / 16)
    zs = [z for _, z in traj]
    assert int(np.argmax(zs)) != len(zs) - 1
    th, z, _ = orc.refine_trace(_map(orc, fq4), th0, K, steps, L, dmax)
    np.testing.assert_allclose(th, traj[int(np.argmax(zs))][0], rtol=0, atol=1e-9)
