"""Derive the polynomial the polar fold uses for arg p: atan(t) / (2 pi) on |t| <= tan(pi/8).

Method: weighted least squares on Chebyshev nodes of the interval (a standard near-minimax
construction, cf. Trefethen, "Approximation Theory and Approximation Practice", ch. 16), for
    atan(t) / (2 pi) ~ t * P(t^2)    (odd)
with P fitted in double precision on s = t^2 and its coefficients rounded to float32. The fold
reduces any (x, y) to this interval: octant symmetry, then atan(a) = pi/4 + atan((a - 1)/(a + 1))
for a = min(|x|, |y|) / max(|x|, |y|) above tan(pi/8); the eighth turns are added as integers.
Run it to print the coefficients and the float32 evaluation's error in units of 2^-32 turn.
"""
import numpy as np

T_MAX = np.tan(np.pi / 8)


def fit(nterms, n=4000):
    k = np.arange(n)
    t = np.cos(np.pi * (k + 0.5) / n) * T_MAX  # Chebyshev nodes on [-T_MAX, T_MAX]
    t = t[t != 0]
    target = np.arctan(t) / (2 * np.pi) / t    # atan(t) / (2 pi) = t P(t^2)
    A = np.vander(t * t, nterms, increasing=True)
    c, *_ = np.linalg.lstsq(A, target, rcond=None)
    return c


def evaluate_f32(c, t):
    t = t.astype(np.float32)
    s = (t * t).astype(np.float32)
    acc = np.float32(c[-1])
    for ci in c[-2::-1]:
        acc = (acc * s + np.float32(ci)).astype(np.float32)
    return (t * acc).astype(np.float32)


def main():
    ts = np.linspace(-T_MAX, T_MAX, 4_000_001)
    ref = np.arctan(ts) / (2 * np.pi)
    for nterms in (6, 7, 8):
        c = fit(nterms).astype(np.float32)
        err = np.abs(evaluate_f32(c, ts).astype(np.float64) - ref).max()
        print(f"// {nterms} terms: max error {err:.3e} turn = {err * 2.0 ** 32:.1f} units of 2^-32 turn")
        print(", ".join(f"{float(v):.9e}f" for v in c))


if __name__ == "__main__":
    main()
