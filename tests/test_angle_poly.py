"""The float32 angle polynomials of the per-chain kernel's root solve
(sample.hpp: kAtanP, kAsinQ), evaluated on the CPU in float32 arithmetic with
the kernel's operation order, against numpy's float64 arctan2 / arcsin.

The kernel's v_rcp_f32 (followed by one Newton step) and v_sqrt_f32 are
within one ulp; the emulation takes the correctly rounded value and its
neighbours on both sides, so the bounds hold for any result within that
ulp.  The coefficients must be the
ones fit_angle_poly.py prints (derived here, not taken from a library)."""
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_10449_amd", "csrc")
f32 = np.float32


def header_coeffs(name):
    text = open(os.path.join(CSRC, "sample.hpp")).read()
    m = re.search(r"constexpr float " + name + r"\[\d+\] = \{([^}]*)\}", text)
    assert m, name
    return np.array([float(v.strip().rstrip("f")) for v in m.group(1).split(",")], dtype=f32)


def fma32(a, b, c):
    # a * b is exact in float64 for float32 operands; one rounding to float32
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def horner(c, x):
    acc = np.full_like(x, c[-1])
    for k in range(len(c) - 2, -1, -1):
        acc = fma32(acc, x, np.full_like(x, c[k]))
    return acc


def atan2_poly(q, p, P, nudge=0):
    ax, ay = np.abs(p), np.abs(q)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    r0 = (f32(1) / mx).astype(f32)
    if nudge:
        r0 = np.nextafter(r0, f32(np.inf) if nudge > 0 else f32(0)).astype(f32)
    one = np.ones_like(mx)
    inv = fma32(r0, fma32(-mx, r0, one), r0)   # one Newton step
    t = (mn * inv).astype(f32)
    u = (t * t).astype(f32)
    r = fma32((t * u).astype(f32), horner(P, u), t).astype(np.float64)
    r = np.where(ay > ax, 0.5 * np.pi - r, r)      # reflections in float64
    r = np.where(p < 0, np.pi - r, r)
    return np.where(np.signbit(q), -r, r)


def asin_sqrt_poly(w, Q, nudge=0):
    s = np.sqrt(w.astype(np.float64)).astype(f32)
    if nudge:   # the root of 0 is 0 exactly
        s = np.where(s > 0, np.nextafter(s, f32(np.inf) if nudge > 0 else f32(0)), s).astype(f32)
    return fma32((s * w).astype(f32), horner(Q, w), s)


def test_coefficients_are_the_fit_scripts():
    sys.path.insert(0, CSRC)
    try:
        import fit_angle_poly
    finally:
        sys.path.remove(CSRC)
    pa, qa = fit_angle_poly.coefficients()
    assert np.array_equal(pa, header_coeffs("kAtanP"))
    assert np.array_equal(qa, header_coeffs("kAsinQ"))


@pytest.mark.parametrize("nudge", [-1, 0, 1])
def test_atan2_within_1_2e_7_rad(nudge):
    P = header_coeffs("kAtanP")
    rng = np.random.default_rng(11)
    n = 400_000
    p = np.concatenate([rng.standard_normal(n), np.cos(np.linspace(-np.pi, np.pi, n)),
                        rng.standard_normal(n) * 1e-30, [0.0, -0.0, 1.0, -1.0, 3.0]]).astype(f32)
    q = np.concatenate([rng.standard_normal(n), np.sin(np.linspace(-np.pi, np.pi, n)),
                        rng.standard_normal(n) * 1e-30, [1.0, -1.0, 0.0, -0.0, 3.0]]).astype(f32)
    # the kernel scales arguments below 2^-100 up by 2^100 first (exact)
    small = np.maximum(np.abs(p), np.abs(q)) < 2.0 ** -100
    ps = np.where(small, p * f32(2.0 ** 100), p).astype(f32)
    qs = np.where(small, q * f32(2.0 ** 100), q).astype(f32)
    got = atan2_poly(qs, ps, P, nudge).astype(np.float64)
    ref = np.arctan2(q.astype(np.float64), p.astype(np.float64))
    d = np.abs(got - ref)
    d = np.minimum(d, 2 * np.pi - d)
    assert d.max() < 1.2e-7, d.max()
    # the sign convention of atan2 on the negative axis: q = -0, p = -1
    assert got[-2] < 0 and abs(got[-2] + np.pi) < 1.2e-7


@pytest.mark.parametrize("nudge", [-1, 0, 1])
def test_asin_sqrt_within_1_5e_7(nudge):
    Q = header_coeffs("kAsinQ")
    rng = np.random.default_rng(12)
    w64 = np.concatenate([rng.uniform(0, 0.5, 600_000), np.logspace(-17, np.log10(0.5), 100_000),
                          [0.0, 0.5, 0.25]])
    w = w64.astype(f32)
    got = asin_sqrt_poly(w, Q, nudge).astype(np.float64)
    # against the float32 argument the kernel sees (its rounding of w is
    # part of the root solve's error budget, not of the polynomial's)
    ref = np.arcsin(np.sqrt(w.astype(np.float64)))
    assert np.abs(got - ref).max() < 1.5e-7, np.abs(got - ref).max()
    assert got[-3] == 0.0
