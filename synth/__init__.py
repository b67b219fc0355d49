"""Seeded synthetic workloads (whitened problems A, b, x0).

This module builds inputs only; it holds none of the sampler's arithmetic, so
both the HIP path and the CPU oracle may consume it.  Every generator is
deterministic in its `rng_seed` (numpy default_rng).

Workloads (the paper measures only on synthetic instances: the univariate
truncations of its Section 4.1 and the random d x d instances of Section 4.2):

* small_fp64      d=10,   m=20,   16 chains:  A_ij ~ N(0,1), b ~ U(0.5,1.5)
* box_halfspace   d=100,  m=200,  4096 chains: x_1..x_50 two-sided box bounds
                  |x_j| <= c_j, c_j ~ U(0.5,2) (100 rows), plus 100 random
                  halfspaces with rows N(0,1)/sqrt(d), b ~ U(0.5,1.5)
* gp_rbf          d=m/2=1000, m=2000, 1024 chains: A_top = S L with L the
                  Cholesky factor of an RBF kernel (lengthscale 0.2, unit
                  variance, jitter 1e-6) on 1000 points uniform in [0,1]^2,
                  S = diag(random +-1), b_top = 0.1; plus 1000 random
                  halfspaces as in box_halfspace
* batched_uneven  256 problems, d ~ round(exp(U(ln 16, ln 512))),
                  m = d * U{1..4}, rows N(0,1)/sqrt(d), b ~ U(0.5,1.5),
                  64 chains each
* warm_family     d=256, m=768, fixed A (rows N(0,1)/sqrt(d)), b0 ~ U(0.5,1.5),
                  b = b0 + delta, delta ~ N(0, 0.1^2 I), redrawn while
                  min(b) <= 0.05
* paper_highdim   Section 4.2: A d x d N(0,1), x0 ~ N(0,I), b = A x0 + U[0,1]^d
* univariate      Section 4.1: N(0,1) on [lo, hi] as two rows
* box             independent box truncation lo_j <= x_j <= hi_j
x0 = 0 is strictly feasible for every workload with b > 0.
"""
from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Problem:
    A: np.ndarray            # (m, d) float64
    b: np.ndarray            # (m,) float64
    x0: np.ndarray           # (d,) float64, strictly feasible
    n_chains: int
    n_steps: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def d(self):
        return self.A.shape[1]

    @property
    def m(self):
        return self.A.shape[0]


def _halfspaces(rng, n, d):
    A = rng.standard_normal((n, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, size=n)
    return A, b


def small_fp64(rng_seed=1, d=10, m=20, n_chains=16, n_steps=2000):
    rng = np.random.default_rng(rng_seed)
    A = rng.standard_normal((m, d))
    b = rng.uniform(0.5, 1.5, size=m)
    return Problem(A, b, np.zeros(d), n_chains, n_steps, "small_fp64")


def box_halfspace(rng_seed=2, d=100, n_box=50, n_half=100, n_chains=4096, n_steps=1000):
    rng = np.random.default_rng(rng_seed)
    c = rng.uniform(0.5, 2.0, size=n_box)
    Abox = np.zeros((2 * n_box, d))
    idx = np.arange(n_box)
    Abox[2 * idx, idx] = 1.0
    Abox[2 * idx + 1, idx] = -1.0
    bbox = np.repeat(c, 2)
    Ah, bh = _halfspaces(rng, n_half, d)
    return Problem(np.vstack([Abox, Ah]), np.concatenate([bbox, bh]), np.zeros(d),
                   n_chains, n_steps, "box_halfspace", {"box_c": c})


def gp_rbf(rng_seed=3, d=1000, n_half=1000, lengthscale=0.2, jitter=1e-6, shift=0.1,
           n_chains=1024, n_steps=500):
    rng = np.random.default_rng(rng_seed)
    pts = rng.uniform(0.0, 1.0, size=(d, 2))
    sq = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    K = np.exp(-sq / (2.0 * lengthscale ** 2)) + jitter * np.eye(d)
    L = np.linalg.cholesky(K)
    s = rng.choice([-1.0, 1.0], size=d)
    Atop = s[:, None] * L
    btop = np.full(d, shift)
    Ah, bh = _halfspaces(rng, n_half, d)
    return Problem(np.vstack([Atop, Ah]), np.concatenate([btop, bh]), np.zeros(d),
                   n_chains, n_steps, "gp_rbf")


def batched_uneven(rng_seed=4, n_problems=256, d_lo=16, d_hi=512, k_max=4,
                   chains_per_problem=64, n_steps=1000):
    rng = np.random.default_rng(rng_seed)
    probs = []
    for p in range(n_problems):
        d = int(round(math.exp(rng.uniform(math.log(d_lo), math.log(d_hi)))))
        k = int(rng.integers(1, k_max + 1))
        A, b = _halfspaces(rng, k * d, d)
        probs.append(Problem(A, b, np.zeros(d), chains_per_problem, n_steps,
                             f"batched_{p}", {"k": k}))
    return probs


def warm_family(rng_seed=5, d=256, m=768, delta_sd=0.1, min_b=0.05):
    """Returns (A, b0, draw) where draw(rng, n) gives n right-hand sides."""
    rng = np.random.default_rng(rng_seed)
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b0 = rng.uniform(0.5, 1.5, size=m)

    def draw(gen, n):
        out = np.empty((n, m))
        for i in range(n):
            while True:
                bb = b0 + delta_sd * gen.standard_normal(m)
                if bb.min() > min_b:
                    break
            out[i] = bb
        return out

    return A, b0, draw


def paper_highdim(rng_seed=6, d=1000, n_chains=1, n_steps=1000):
    rng = np.random.default_rng(rng_seed)
    A = rng.standard_normal((d, d))
    x0 = rng.standard_normal(d)
    b = A @ x0 + rng.uniform(0.0, 1.0, size=d)
    return Problem(A, b, x0, n_chains, n_steps, "paper_highdim")


def univariate(lo, hi, n_chains=2000, n_steps=1000):
    A = np.array([[1.0], [-1.0]])
    b = np.array([hi, -lo])
    x0 = np.array([0.5 * (lo + hi)])
    return Problem(A, b, x0, n_chains, n_steps, f"univariate[{lo},{hi}]")


def box(lo, hi, n_chains=256, n_steps=1000):
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    d = lo.size
    A = np.vstack([np.eye(d), -np.eye(d)])
    b = np.concatenate([hi, -lo])
    return Problem(A, b, 0.5 * (lo + hi), n_chains, n_steps, "box", {"lo": lo, "hi": hi})


def random_small(rng, d, m, n_chains=4):
    """Tiny random polytope with x0 = 0 strictly inside (for exhaustive checks)."""
    A = rng.standard_normal((m, d))
    b = rng.uniform(0.2, 1.5, size=m)
    return Problem(A, b, np.zeros(d), n_chains, 1, "random_small")


def random_states(rng, A, b, n, scale=1.0, margin=1e-3):
    """n points strictly inside {A x <= b} (needs b > margin, so that 0 is inside).

    Each point is a draw x ~ N(0, scale^2 I), kept as it is when it clears
    every constraint by `margin`, else pulled toward 0 along its own
    direction to a uniform fraction in [0.2, 0.9] of the distance at which it
    would reach the first constraint (less margin): a generic interior point
    in a random direction, never 0 itself."""
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64)
    assert (b > margin).all(), "0 must clear every constraint by the margin"
    d = A.shape[1]
    out = np.empty((n, d))
    for i in range(n):
        x = scale * rng.standard_normal(d)
        ax = A @ x
        if (ax <= b - margin).all():
            out[i] = x
            continue
        pos = ax > 0
        t_max = np.min((b[pos] - margin) / ax[pos])
        out[i] = rng.uniform(0.2, 0.9) * t_max * x
    return out
