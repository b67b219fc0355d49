"""Planted mistakes in the oracle (on the CPU) must each break some pin.

Every mutation below is a plausible slip when writing the oracle from the
paper: a flipped sign or swapped argument in the root formula, a missing
cumulative max, an off-by-one in gamma, a wrong interpolation in the inverse
CDF, swapped ellipse terms, an inverted safeguard, a wrong Philox constant,
a likelihood test that reads one row or swaps inside and outside, a gap
tested at its end instead of its middle, a change of variables with the
wrong sign of A mu or without the mean, a trim that also moves the 0 / 2 pi
seam, trims by 2 eps or turns an empty candidate into a piece, and a
transition that never rejects or rejects a proposal on the boundary.
"""
import numpy as np
import pytest

import oracle_pins as P
from oracle import ess, philox

TWO_PI = ess.TWO_PI


def _roots_sign_flip(p, q, b):
    al, be, hit = ORIG["roots"](p, q, b)
    phi = 0.5 * (be - al)
    al2 = ess.wrap_2pi(al + 2 * phi)          # tau + phi taken as alpha
    return np.where(hit, np.minimum(al2, be), 0), np.where(hit, np.maximum(al2, be), 0), hit


def _roots_swapped_atan(p, q, b):
    return ORIG["roots"](q, p, b)             # atan2(p, q) instead of atan2(q, p)


def _roots_no_wrap(p, q, b):
    p = np.asarray(p, float); q = np.asarray(q, float); b = np.asarray(b, float)
    r = np.hypot(p, q)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = b / r
    hit = (r > 0) & (z < 1)
    z = np.clip(np.where(hit, z, 0), -1, 1)
    tau, phi = np.arctan2(q, p), np.arccos(z)
    al, be = tau - phi, tau + phi             # forgot the wrap into [0, 2 pi]
    return np.where(hit, al, 0), np.where(hit, be, 0), hit


def _alg3_no_cummax(alpha, beta):
    order = np.argsort(alpha, axis=-1, kind="stable")
    a_s = np.take_along_axis(np.asarray(alpha, float), order, -1)
    b_s = np.take_along_axis(np.asarray(beta, float), order, -1)
    lo = np.concatenate([np.zeros(a_s.shape[:-1] + (1,)), b_s], -1)   # beta, not cummax
    hi = np.concatenate([a_s, np.full(a_s.shape[:-1] + (1,), TWO_PI)], -1)
    return lo, hi


def _alg3_gamma_off_by_one(alpha, beta):
    lo, hi = ORIG["alg3_candidates"](alpha, beta)
    lo2 = lo.copy()
    lo2[..., 1:-1] = lo[..., 2:]              # gamma_k used where gamma_{k-1} belongs
    return lo2, hi


def _alg3_sort_beta(alpha, beta):
    order = np.argsort(beta, axis=-1, kind="stable")   # sorted by the wrong endpoint
    a_s = np.take_along_axis(np.asarray(alpha, float), order, -1)
    b_s = np.take_along_axis(np.asarray(beta, float), order, -1)
    g = np.maximum.accumulate(b_s, -1)
    lo = np.concatenate([np.zeros(a_s.shape[:-1] + (1,)), g], -1)
    hi = np.concatenate([a_s, np.full(a_s.shape[:-1] + (1,), TWO_PI)], -1)
    return lo, hi


def _sample_no_offset(lo, hi, u):
    ell = np.maximum(np.asarray(hi) - np.asarray(lo), 0)
    cum = np.cumsum(ell)
    if cum[-1] <= 0:
        return 0.0, 0.0
    s = u * cum[-1]
    k = min(int(np.searchsorted(cum, s, side="right")), len(ell) - 1)
    return min(float(lo[k]) + s, float(hi[k])), float(cum[-1])   # forgot "- cum_{k-1}"


def _transition_swapped(A, b, x, nu, u, eps=0.0, pq=None, store=np.float64):
    return ORIG["transition"](A, b, nu, x, u, eps, pq, store)    # x and nu swapped


def _transition_inverted_safeguard(A, b, x, nu, u, eps=0.0, pq=None, store=np.float64):
    out = ORIG["transition"](A, b, x, nu, u, eps, pq, store)
    viol = (out["x_prop"] @ np.asarray(A, float).T > np.asarray(b, float)[None, :]).any(axis=1)
    out["x_new"] = np.where(viol[:, None], out["x_prop"], x)    # keeps x when feasible
    return out


def _trim_seam_too(lo, hi, eps):
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    return lo + eps, hi - eps                                    # the seam moves as well


def _trim_twice(lo, hi, eps):
    return ORIG["trim"](lo, hi, 2.0 * eps)                       # 2 eps per end


def _trim_orders_ends(lo, hi, eps):
    tlo, thi = ORIG["trim"](lo, hi, eps)
    return np.minimum(tlo, thi), np.maximum(tlo, thi)            # empty candidates become pieces


def _transition_always_accept(A, b, x, nu, u, eps=0.0, pq=None, store=np.float64, method="alg3"):
    out = ORIG["transition"](A, b, x, nu, u, eps, pq, store, method)
    out["rejected"] = out["total"] <= 0.0                        # the safeguard dropped
    out["x_new"] = np.where(out["rejected"][:, None], np.asarray(x, float), out["x_prop"])
    return out


def _transition_rejects_boundary(A, b, x, nu, u, eps=0.0, pq=None, store=np.float64, method="alg3"):
    out = ORIG["transition"](A, b, x, nu, u, eps, pq, store, method)
    bb = np.asarray(b, float)
    bb = bb[None, :] if bb.ndim == 1 else bb
    viol = (out["x_prop"] @ np.asarray(A, float).T >= bb).any(axis=1)   # equality rejected
    out["rejected"] = viol | (out["total"] <= 0.0)
    out["x_new"] = np.where(out["rejected"][:, None], np.asarray(x, float), out["x_prop"])
    return out


def _philox_wrong_weyl(c0, c1, c2, c3, k0, k1):
    saved = philox.W1
    philox.W1 = np.uint64(0xBB67AE86)
    try:
        return ORIG["philox4x32_10"](c0, c1, c2, c3, k0, k1)
    finally:
        philox.W1 = saved


def _box_muller_cos_twice(u1, u2):
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(TWO_PI * u2), rad * np.cos(TWO_PI * u2)


def _likelihood_first_row_only(p, q, b, theta):
    return bool(p[0] * np.cos(theta) + q[0] * np.sin(theta) <= b[0])


def _likelihood_strict_reversed(p, q, b, theta):
    return bool(np.all(p * np.cos(theta) + q * np.sin(theta) >= b))   # inside / outside swapped


def _midpoint_tests_lower_end(p, q, b):
    alpha, beta, hit = ess.roots(p, q, b)
    ends = np.concatenate([[0.0], np.sort(np.concatenate([alpha[hit], beta[hit]])), [TWO_PI]])
    out = []
    for lo, hi in zip(ends[:-1], ends[1:]):
        if hi > lo and ess.likelihood(p, q, b, lo):     # the gap's end, not its middle
            out.append((float(lo), float(hi)))
    return out


def _whiten_shift_sign(A, b, mu, L):
    A = np.asarray(A, float)
    return A @ np.asarray(L, float), np.asarray(b, float) + A @ np.asarray(mu, float)   # + A mu


def _unwhiten_no_mean(U, L, mu):
    return np.asarray(U, float) @ np.asarray(L, float).T                               # forgot + mu


ORIG = {"roots": ess.roots, "alg3_candidates": ess.alg3_candidates,
        "transition": ess.transition, "philox4x32_10": philox.philox4x32_10,
        "trim": ess.trim}

MUTATIONS = [
    (ess, "roots", _roots_sign_flip),
    (ess, "roots", _roots_swapped_atan),
    (ess, "roots", _roots_no_wrap),
    (ess, "alg3_candidates", _alg3_no_cummax),
    (ess, "alg3_candidates", _alg3_gamma_off_by_one),
    (ess, "alg3_candidates", _alg3_sort_beta),
    (ess, "sample_theta", _sample_no_offset),
    (ess, "transition", _transition_swapped),
    (ess, "transition", _transition_inverted_safeguard),
    (philox, "philox4x32_10", _philox_wrong_weyl),
    (philox, "box_muller", _box_muller_cos_twice),
    (ess, "likelihood", _likelihood_first_row_only),
    (ess, "likelihood", _likelihood_strict_reversed),
    (ess, "midpoint_intervals", _midpoint_tests_lower_end),
    (ess, "whiten", _whiten_shift_sign),
    (ess, "unwhiten", _unwhiten_no_mean),
    (ess, "trim", _trim_seam_too),
    (ess, "trim", _trim_twice),
    (ess, "trim", _trim_orders_ends),
    (ess, "transition", _transition_always_accept),
    (ess, "transition", _transition_rejects_boundary),
]


@pytest.mark.parametrize("mod,name,bad", MUTATIONS, ids=lambda v: getattr(v, "__name__", ""))
def test_planted_mistake_is_caught(monkeypatch, mod, name, bad):
    monkeypatch.setattr(mod, name, bad)
    caught = []
    for pin in P.FAST_PINS + P.CHAIN_PINS:
        try:
            if pin():
                caught.append(pin.__name__)
        except Exception as e:  # a crash also counts as caught
            caught.append(f"{pin.__name__}:{type(e).__name__}")
        if caught:
            break
    print(bad.__name__, "caught by", caught)
    assert caught, f"mutation {bad.__name__} not caught by any pin"
