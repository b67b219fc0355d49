"""Float64 CPU oracle for one linear elliptical slice sampling transition.

Test infrastructure only: nothing on the product path may import this file.
It follows Wu & Gardner, "A Fast, Robust Elliptical Slice Sampling
Implementation for Linearly Truncated Multivariate Normal Distributions"
(arXiv 2407.10449):

* target: N(0, I_d) restricted to {x : A x <= b} (Section 1);
* one transition (Algorithm 1): draw nu ~ N(0, I), form the ellipse
  x(theta) = x cos(theta) + nu sin(theta) (Section 2, eq. "ellipse"), build
  the active intervals I_act, draw theta uniformly on I_act, move;
* per-constraint roots of p cos(theta) + q sin(theta) = b (Section 2, eq.
  "trigonometry-equation"; Appendix B, eq. "roots"), and Appendix B's two
  alternative forms, for the ablation of the root formula;
* the active intervals by brute force (Algorithm 2), by sort + cumulative
  max (Algorithm 3 / Proposition 1), with the no-root padding of Section 3.2,
  and by likelihood testing at midpoints (Section 2.2, the quadratic method
  the paper compares against);
* the two safeguards of Section 3.3: trimming by epsilon and reject-and-stay;
* Appendix A's change of variables for N(mu, Sigma), Sigma = L L^T.

Readings taken where the paper is silent (each is listed with its reason in
the design notes):
* alpha = (tau - phi) wrapped into [0, 2 pi), beta = min(alpha + 2 phi, 2 pi);
* b / r >= 1 or r == 0 pads the row with alpha = beta = 0; b / r < -1 is
  clamped to -1;
* trimming moves only real endpoints: a lower end at 0 and an upper end at
  2 pi are the seam through x_t itself and stay;
* theta is drawn by inverse CDF over the candidate intervals in ascending
  order; zero total length means "stay" and counts as a rejection;
* a proposal is rejected when some a_i^T x' > b_i (equality accepted).

Everything is float64; x and nu may be handed in already rounded to the
storage precision of the code under test.
"""
import math

import numpy as np

from . import philox

TWO_PI = 6.283185307179586


# --------------------------------------------------------------------------
# Appendix B: roots of p cos(theta) + q sin(theta) = b
# --------------------------------------------------------------------------
def wrap_2pi(a):
    """a mod 2 pi into [0, 2 pi); a result that rounds to 2 pi becomes 0."""
    w = np.mod(a, TWO_PI)
    return np.where(w >= TWO_PI, 0.0, w)


def roots(p, q, b):
    """Intersection angles of each constraint with the ellipse (Appendix B).

    p = a_i^T x_t, q = a_i^T nu_t, b = b_i (broadcastable arrays).
    Returns (alpha, beta, hit) with I_i = [0, alpha] U [beta, 2 pi]; rows the
    ellipse never crosses (b / r > 1, Section 3.2, and r = 0) get the padding
    alpha = beta = 0 and hit = False.
    """
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = np.hypot(p, q)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = b / r
    hit = (r > 0) & (z < 1.0)
    z = np.clip(np.where(hit, z, 0.0), -1.0, 1.0)
    tau = np.arctan2(q, p)            # cos tau = p / r, sin tau = q / r
    phi = np.arccos(z)                # roots are tau +- phi
    alpha = wrap_2pi(tau - phi)
    beta = np.minimum(alpha + 2.0 * phi, TWO_PI)
    alpha = np.where(hit, alpha, 0.0)
    beta = np.where(hit, beta, 0.0)
    return alpha, beta, hit


# --------------------------------------------------------------------------
# Appendix B's two alternative root forms (for the ablation only)
# --------------------------------------------------------------------------
def roots_gessner(p, q, b, dtype=np.float64):
    """The form of Gessner et al. quoted in Appendix B:
    theta = +-acos(b / r) + 2 atan(q / (r + p)).  The half angle 2 atan(q /
    (r + p)) equals tau (tan(tau / 2) = sin tau / (1 + cos tau)), so the
    infeasible arc is again (2 atan(q / (r + p)) - phi, ... + phi) and the
    same wrap gives (alpha, beta, hit) as `roots` does.  Evaluated in `dtype`
    as written: nothing handles r + p = 0 (q = 0 with p < 0), where the
    quotient is 0 / 0."""
    p, q, b = (np.asarray(v, dtype=np.float64).astype(dtype) for v in (p, q, b))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        r = np.sqrt(p * p + q * q)
        z = b / r
        hit = (r > 0) & (z < 1)
        phi = np.arccos(np.clip(np.where(hit, z, 0), -1, 1)).astype(np.float64)
        tau = (2 * np.arctan(q / (r + p))).astype(np.float64)
    alpha = wrap_2pi(tau - phi)
    beta = np.minimum(alpha + 2.0 * phi, TWO_PI)
    return np.where(hit, alpha, 0.0), np.where(hit, beta, 0.0), hit


def roots_benavoli(p, q, b, dtype=np.float64):
    """The form of Benavoli et al. quoted in Appendix B:
    tan(theta / 2) = (q +- sqrt(r^2 - b^2)) / (b + p).  With t = tan(theta / 2)
    the constraint p cos + q sin <= b becomes g(t) = (b + p) t^2 - 2 q t +
    (b - p) >= 0, so for b + p > 0 the infeasible arc lies between the two
    roots and for b + p < 0 it runs through theta = pi; theta = 0 (x_t) is
    feasible either way.  Returns (alpha, beta, hit) as `roots` does,
    evaluated in `dtype` as written: nothing handles b + p = 0, where one
    root is at theta = pi and the quotient divides by zero."""
    p, q, b = (np.asarray(v, dtype=np.float64).astype(dtype) for v in (p, q, b))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        r2 = p * p + q * q
        hit = (r2 > 0) & (b * b < r2) | ((r2 > 0) & (b < 0))
        s = np.sqrt(np.maximum(r2 - b * b, 0))
        den = b + p
        t1 = 2 * np.arctan((q - s) / den)
        t2 = 2 * np.arctan((q + s) / den)
        lo = np.minimum(t1, t2).astype(np.float64)
        hi = np.maximum(t1, t2).astype(np.float64)
    inside = np.asarray(den, np.float64) > 0          # infeasible arc is (lo, hi)
    alpha = np.where(inside, wrap_2pi(lo), wrap_2pi(hi))
    width = np.where(inside, hi - lo, lo + TWO_PI - hi)
    beta = np.minimum(alpha + width, TWO_PI)
    return np.where(hit, alpha, 0.0), np.where(hit, beta, 0.0), hit


# --------------------------------------------------------------------------
# Algorithm 2: the definition, I_act = intersection of all I_i, one at a time
# --------------------------------------------------------------------------
def _intersect_lists(u, v):
    out = []
    for lo1, hi1 in u:
        for lo2, hi2 in v:
            lo, hi = max(lo1, lo2), min(hi1, hi2)
            if lo <= hi:
                out.append((lo, hi))
    out.sort()
    return out


def alg2_brute_force(alpha, beta):
    """Active intervals of one chain by sequential intersection (Algorithm 2).

    Closed intervals; the result may contain zero-length pieces.
    """
    acc = [(0.0, TWO_PI)]
    for a, b in zip(np.asarray(alpha, float), np.asarray(beta, float)):
        acc = _intersect_lists(acc, [(0.0, float(a)), (float(b), TWO_PI)])
    return acc


# --------------------------------------------------------------------------
# Algorithm 3 / Proposition 1: sort the alphas, cumulative max of the betas
# --------------------------------------------------------------------------
def alg3_candidates(alpha, beta):
    """The m + 1 candidate intervals of Proposition 1, for one or many chains.

    alpha, beta: (..., m).  Returns (lo, hi), each (..., m + 1):
      k = 0:          [0, alpha_(1)]
      k = 1 .. m - 1: [gamma_k, alpha_(k+1)]  with gamma_k = max of the first
                      k betas in alpha order (cumulative max)
      k = m:          [gamma_m, 2 pi]
    A candidate with hi < lo is the empty set.
    """
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    order = np.argsort(alpha, axis=-1, kind="stable")
    a_s = np.take_along_axis(alpha, order, axis=-1)
    b_s = np.take_along_axis(beta, order, axis=-1)
    gamma = np.maximum.accumulate(b_s, axis=-1)
    shape = alpha.shape[:-1] + (alpha.shape[-1] + 1,)
    lo = np.empty(shape)
    hi = np.empty(shape)
    lo[..., 0] = 0.0
    lo[..., 1:] = gamma
    hi[..., :-1] = a_s
    hi[..., -1] = TWO_PI
    return lo, hi


def nonempty(lo, hi, min_len=0.0):
    """Pieces of one chain's candidate list with length > min_len, in order."""
    return [(float(l), float(h)) for l, h in zip(lo, hi) if h - l > min_len]


# --------------------------------------------------------------------------
# Section 2.2: likelihood testing at midpoints (the quadratic comparator)
# --------------------------------------------------------------------------
def likelihood(p, q, b, theta):
    """Section 2.2's likelihood: 1 when x(theta) satisfies every constraint,
    evaluated from the cached projections p = A x_t and q = A nu_t."""
    return bool(np.all(p * math.cos(theta) + q * math.sin(theta) <= b))


def midpoint_intervals(p, q, b):
    """Active intervals of one chain by likelihood testing at midpoints
    (Section 2.2, the variant that tests the point halfway between two
    consecutive intersection angles instead of a fixed offset).

    The intersection angles of the crossing rows are sorted, with 0 and 2 pi
    as the outer ends; every gap of positive length whose midpoint has
    likelihood 1 is active, and touching active gaps merge.  Each test reads
    all m rows, so the whole is O(m^2).  Returns the list of (lo, hi).
    """
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    alpha, beta, hit = roots(p, q, b)
    ends = np.concatenate([[0.0], np.sort(np.concatenate([alpha[hit], beta[hit]])), [TWO_PI]])
    out = []
    for lo, hi in zip(ends[:-1], ends[1:]):
        if hi <= lo:
            continue
        if likelihood(p, q, b, 0.5 * (lo + hi)):
            if out and out[-1][1] == lo:
                out[-1] = (out[-1][0], float(hi))
            else:
                out.append((float(lo), float(hi)))
    return out


# --------------------------------------------------------------------------
# Section 3.3: trimming, then theta uniform on the active intervals
# --------------------------------------------------------------------------
def trim(lo, hi, eps):
    """[l, u] -> [l + eps, u - eps] at real endpoints; the 0 / 2 pi seam stays."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if eps == 0.0:
        return lo.copy(), hi.copy()
    return np.where(lo > 0.0, lo + eps, lo), np.where(hi < TWO_PI, hi - eps, hi)


def sample_theta(lo, hi, u):
    """theta uniform on the union of [lo_k, hi_k] (one chain) by inverse CDF.

    Returns (theta, total_length).  Zero total length returns theta = 0.
    """
    ell = np.maximum(np.asarray(hi) - np.asarray(lo), 0.0)
    cum = np.cumsum(ell)
    total = float(cum[-1])
    if total <= 0.0:
        return 0.0, 0.0
    s = float(u) * total
    k = int(np.searchsorted(cum, s, side="right"))   # first k with cum_k > s
    if k >= len(ell):                                 # s rounded up to total
        k = int(np.nonzero(ell > 0)[0][-1])
        return float(hi[k]), total
    before = float(cum[k - 1]) if k > 0 else 0.0
    theta = float(lo[k]) + (s - before)
    return min(theta, float(hi[k])), total


# --------------------------------------------------------------------------
# Algorithm 1: one transition for a batch of chains
# --------------------------------------------------------------------------
def transition(A, b, x, nu, u, eps=0.0, pq=None, store=np.float64, method="alg3"):
    """One transition for C chains.

    A (m, d), b (m,) or (C, m) (one polytope per chain), x (C, d), nu (C, d),
    u (C,).  If pq = (P, Q) (each
    (C, m)) is given, those projections are used instead of A x and A nu.
    The proposal is rounded to `store` before the feasibility check, as the
    code under test stores it.  method="midpoint" builds the active intervals
    by Section 2.2's likelihood testing and method="alg2" by Algorithm 2's
    sequential intersection instead of Algorithm 3.
    Returns a dict with x_new, rejected, theta, intervals (list per chain of
    the non-empty trimmed pieces), alpha, beta, p, q, x_prop.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    if pq is None:
        P, Q = x @ A.T, nu @ A.T
    else:
        P, Q = (np.asarray(t, dtype=np.float64) for t in pq)
    bb = b[None, :] if b.ndim == 1 else b
    alpha, beta, _ = roots(P, Q, bb)
    C = x.shape[0]
    if method == "alg3":
        lo, hi = alg3_candidates(alpha, beta)
        lo, hi = trim(lo, hi, eps)
        pieces = [(lo[c], hi[c]) for c in range(C)]
    elif method == "alg2":
        # Algorithm 2 over the rows the ellipse crosses (a row it does not
        # cross has I_i = [0, 2 pi], which leaves the intersection as it is)
        pieces = []
        for c in range(C):
            hit = beta[c] > 0.0
            ivs = alg2_brute_force(alpha[c][hit], beta[c][hit])
            lo_c = np.array([v[0] for v in ivs] or [0.0])
            hi_c = np.array([v[1] for v in ivs] or [0.0])
            pieces.append(trim(lo_c, hi_c, eps))
    else:
        pieces = []
        for c in range(C):
            ivs = midpoint_intervals(P[c], Q[c], bb[c if bb.shape[0] > 1 else 0])
            lo_c = np.array([v[0] for v in ivs] or [0.0])
            hi_c = np.array([v[1] for v in ivs] or [0.0])
            pieces.append(trim(lo_c, hi_c, eps))
    theta = np.zeros(C)
    total = np.zeros(C)
    intervals = []
    for c in range(C):
        theta[c], total[c] = sample_theta(pieces[c][0], pieces[c][1], u[c])
        intervals.append(nonempty(pieces[c][0], pieces[c][1]))
    ct, st = np.cos(theta), np.sin(theta)
    x_prop = x * ct[:, None] + nu * st[:, None]
    x_prop = x_prop.astype(store).astype(np.float64)
    viol = (x_prop @ A.T > bb).any(axis=1)
    rejected = viol | (total <= 0.0)
    x_new = np.where(rejected[:, None], x, x_prop)
    return dict(x_new=x_new, rejected=rejected, theta=theta, total=total,
                intervals=intervals, alpha=alpha, beta=beta, p=P, q=Q,
                x_prop=x_prop)


def run(A, b, x0, n_chains, n_steps, seed, eps=0.0, store=np.float64,
        start_step=0, thin=1, chain_offset=0, problem=0):
    """Run C chains for n_steps from x0 with the Philox stream.

    x0: (d,) broadcast to all chains or (C, d).  nu and the proposal are
    rounded to `store`.  Returns (trace (n_steps // thin, C, d), x_final,
    rejections per chain).
    """
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    x = np.broadcast_to(np.asarray(x0, dtype=np.float64), (n_chains, d)).astype(store).astype(np.float64)
    chains = np.arange(n_chains) + chain_offset
    rej = np.zeros(n_chains, dtype=np.int64)
    trace = []
    for t in range(n_steps):
        step = start_step + t
        nu = philox.normals(seed, step, chains, d, problem).astype(store).astype(np.float64)
        u = philox.uniforms(seed, step, chains, problem)
        out = transition(A, b, x, nu, u, eps=eps, store=store)
        x = out["x_new"]
        rej += out["rejected"]
        if (t + 1) % thin == 0:
            trace.append(x.copy())
    return np.array(trace).reshape(-1, n_chains, d), x, rej


# --------------------------------------------------------------------------
# Appendix A: a non-standard normal through the change of variables
# --------------------------------------------------------------------------
def whiten(A, b, mu, L):
    """x ~ N(mu, L L^T) truncated to {A x <= b} is x = L u + mu with
    u ~ N(0, I) truncated to {(A L) u <= b - A mu}: returns (A L, b - A mu)."""
    A = np.asarray(A, dtype=np.float64)
    return A @ np.asarray(L, dtype=np.float64), np.asarray(b, dtype=np.float64) - A @ np.asarray(mu, dtype=np.float64)


def unwhiten(U, L, mu):
    """x = L u + mu for every row u of U."""
    return np.asarray(U, dtype=np.float64) @ np.asarray(L, dtype=np.float64).T + np.asarray(mu, dtype=np.float64)


# --------------------------------------------------------------------------
# Independent check: feasibility of the ellipse on a dense theta grid
# --------------------------------------------------------------------------
def dense_grid_feasible(A, b, x, nu, n=20001):
    """theta grid on [0, 2 pi] and whether x(theta) satisfies A x <= b."""
    theta = np.linspace(0.0, TWO_PI, n)
    pts = np.outer(np.cos(theta), x) + np.outer(np.sin(theta), nu)
    return theta, (pts @ np.asarray(A, float).T <= np.asarray(b, float)[None, :]).all(axis=1)
