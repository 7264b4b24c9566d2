"""Derive the polynomial coefficients the kernels use for sin and cos on [-pi/2, pi/2].

Method: weighted least squares on Chebyshev nodes of the interval (a standard
near-minimax construction, cf. Trefethen, "Approximation Theory and
Approximation Practice", ch. 16), for
    sin(x) ~ x + x^3 * P(x^2)      (odd; leading 1 kept exact)
    cos(x) ~ 1 + x^2 * Q(x^2)      (even; leading 1 kept exact)
with P, Q fitted in double precision on the variable s = x^2. The result is
printed as C float literals; run it to regenerate the table in dev_common.hpp.
"""
import numpy as np


def fit(kind, nterms, n=4000):
    k = np.arange(n)
    x = np.cos(np.pi * (k + 0.5) / n) * (np.pi / 2)      # Chebyshev nodes on [-pi/2, pi/2]
    x = x[x != 0]
    s = x * x
    if kind == "sin":
        target = (np.sin(x) - x) / x ** 3                # sin = x + x^3 P(s)
    else:
        target = (np.cos(x) - 1.0) / s                   # cos = 1 + s Q(s)
    A = np.vander(s, nterms, increasing=True)
    c, *_ = np.linalg.lstsq(A, target, rcond=None)
    return c


def evaluate_f32(kind, c, x):
    x = x.astype(np.float32)
    s = (x * x).astype(np.float32)
    acc = np.float32(c[-1])
    for ci in c[-2::-1]:
        acc = (acc * s + np.float32(ci)).astype(np.float32)
    if kind == "sin":
        return (x + (x * s).astype(np.float32) * acc).astype(np.float32)
    return (np.float32(1) + s * acc).astype(np.float32)


def main():
    xs = np.linspace(-np.pi / 2, np.pi / 2, 2_000_001)
    for kind, nterms in (("sin", 4), ("cos", 5)):
        c = fit(kind, nterms).astype(np.float32)
        ref = np.sin(xs) if kind == "sin" else np.cos(xs)
        err = np.abs(evaluate_f32(kind, c, xs).astype(np.float64) - ref).max()
        print(f"// {kind}: max abs error {err:.3e} in float32 evaluation")
        print(", ".join(f"{float(v):.9e}f" for v in c))


if __name__ == "__main__":
    main()
