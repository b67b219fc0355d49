"""Appendix B's recommendation of the tau +- acos(b / r) root form, checked
on the CPU: evaluated in float32 (the storage precision of the float32
path) the paper's form stays within 2e-6 rad of the float64 roots everywhere
away from tangency, while the forms of Gessner et al. (2 atan(q / (r + p)))
and Benavoli et al. (tan of the half angle over b + p) lose accuracy where
r + p or b + p nears zero, and give NaN at those edges exactly."""
import math

import numpy as np

from oracle import ess

TWO_PI = 2 * math.pi


def paper_form(p, q, b, dtype):
    """tau +- acos(b / r) evaluated in dtype, wrapped as `ess.roots` wraps."""
    p, q, b = (np.asarray(v, np.float64).astype(dtype) for v in (p, q, b))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.sqrt(p * p + q * q)
        z = b / r
        hit = (r > 0) & (z < 1)
        phi = np.arccos(np.clip(np.where(hit, z, 0), -1, 1)).astype(np.float64)
        tau = np.arctan2(q, p).astype(np.float64)
    al = ess.wrap_2pi(tau - phi)
    be = np.minimum(al + 2 * phi, TWO_PI)
    return np.where(hit, al, 0.0), np.where(hit, be, 0.0), hit


def angle_error(al, be, a0, b0):
    d = lambda u, v: np.abs(np.mod(u - v + math.pi, TWO_PI) - math.pi)
    return np.maximum(d(al, a0), d(be, b0))


def sample(seed=0, n=400000):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(n) * 2
    q = rng.standard_normal(n) * 2
    r = np.hypot(p, q)
    b = np.maximum(p, 0) + rng.uniform(0, 1.5, n) * r      # x_t feasible: p <= b
    return p, q, b, r


def test_float32_errors_sit_at_each_forms_edge_cases():
    p, q, b, r = sample()
    a0, b0, h0 = ess.roots(p, q, b)
    away = h0 & (np.abs(b / r) < 0.99)          # acos amplifies rounding near tangency
    err = {}
    for name, f in (("paper", paper_form), ("gessner", ess.roots_gessner),
                    ("benavoli", ess.roots_benavoli)):
        al, be, hit = f(p, q, b, np.float32)
        assert np.array_equal(hit, h0), name
        err[name] = angle_error(al, be, a0, b0)
    assert err["paper"][away].max() < 2e-6
    rp, bp = (r + p) / r, np.abs(b + p) / r
    bad_g = away & (err["gessner"] > 1e-5)
    bad_b = away & (err["benavoli"] > 1e-5)
    assert bad_g.sum() > 10 and bad_b.sum() > 10       # the edge cases do occur
    assert rp[bad_g].max() < 1e-3                      # Gessner: only near r + p = 0
    assert bp[bad_b].max() < 5e-2                      # Benavoli: only near b + p = 0
    assert err["gessner"][away].max() > 100 * err["paper"][away].max()
    assert err["benavoli"][away].max() > 100 * err["paper"][away].max()


def test_exact_edges_break_the_alternative_forms_only():
    # r + p = 0: q = 0, p < 0 (Figure 2's geometry seen from the other side)
    p, q, b = np.array([-1.0]), np.array([0.0]), np.array([0.5])
    al, be, _ = ess.roots(p, q, b)
    assert np.allclose([al[0], be[0]], [2 * math.pi / 3, 4 * math.pi / 3])
    assert np.isnan(ess.roots_gessner(p, q, b)[0]).all()
    # b + p = 0: the constraint's boundary meets the ellipse at theta = pi
    p, q, b = np.array([-0.5]), np.array([1.0]), np.array([0.5])
    al, be, _ = ess.roots(p, q, b)
    assert np.isfinite([al[0], be[0]]).all() and abs(be[0] - math.pi) < 1e-12
    assert np.isnan(ess.roots_benavoli(p, q, b)[0]).all()


def test_box_chains_reach_the_benavoli_edge():
    """b + p = 0 is no rarity: for a box row a = e_j, b = c it holds whenever
    x_j = -c, i.e. as the chain approaches the opposite face of the box.  With
    x_j = -1 + delta, the half-angle form's float32 error reaches 1e-3 rad and
    more as delta shrinks, the paper's form stays at float32 rounding."""
    delta = 10.0 ** -np.arange(1, 7)
    p = -1 + delta
    q = np.full_like(p, 2.0)
    b = np.ones_like(p)
    a0, b0, _ = ess.roots(p, q, b)
    e_paper = angle_error(*paper_form(p, q, b, np.float32)[:2], a0, b0)
    e_ben = angle_error(*ess.roots_benavoli(p, q, b, np.float32)[:2], a0, b0)
    assert e_paper.max() < 1e-6
    assert e_ben[3] > 5e-4 and e_ben[-1] > 1e-2
