"""Fits the float32 polynomials of the per-chain kernel's root solve.

    atan(t) = t + t^3 P(t^2),  t in [0, 1]     (P of degree 8)
    asin(s) = s + s w Q(w),    w = s^2 in [0, 1/2]   (Q of degree 7)

Near-minimax in absolute error: Lawson's iteratively reweighted least squares
on Chebyshev nodes, in float64; the coefficients are then rounded to float32.
Prints the two coefficient lists (lowest degree first) as they appear in
sample.hpp.  Run: python fit_angle_poly.py
"""
import numpy as np


def lawson(f, lo, hi, deg, n=4000, iters=30):
    x = 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos(np.pi * (np.arange(n) + 0.5) / n)
    y = f(x)
    V = np.vander(x, deg + 1, increasing=True)
    w = np.ones(n)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(V * sw[:, None], y * sw, rcond=None)
        e = np.abs(V @ c - y)
        w = w * e
        w /= w.sum()
    return c


def p_atan(u):
    """(atan(sqrt u) / sqrt u - 1) / u, with its series near 0."""
    s = np.sqrt(u)
    big = u > 1e-8
    return np.where(big, (np.arctan(s) / np.where(big, s, 1) - 1) / np.where(big, u, 1),
                    -1 / 3 + u / 5)


def q_asin(w):
    """(asin(sqrt w) / sqrt w - 1) / w, with its series near 0."""
    s = np.sqrt(w)
    big = w > 1e-8
    return np.where(big, (np.arcsin(s) / np.where(big, s, 1) - 1) / np.where(big, w, 1),
                    1 / 6 + 3 * w / 40)


def coefficients():
    pa = lawson(p_atan, 0.0, 1.0, 8).astype(np.float32)
    qa = lawson(q_asin, 0.0, 0.5, 7).astype(np.float32)
    return pa, qa


if __name__ == "__main__":
    pa, qa = coefficients()
    fmt = lambda c: ", ".join(f"{float(v)!r}f" for v in c)
    print("atan P:", fmt(pa))
    print("asin Q:", fmt(qa))
