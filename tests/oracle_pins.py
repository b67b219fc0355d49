"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each pin returns a list of failure messages (empty = pinned).  They look up
the oracle's functions at call time, so the planted-mistake tests can swap a
function for a plausibly wrong one and check that some pin fails.

Sources of truth:
* the worked examples drawn in Figures 1 and 2 (golden files, cited there);
* Algorithm 2 (the definition of I_act) and a dense theta grid that tests
  feasibility of x(theta) directly (they pin Algorithm 3 and the midpoint
  likelihood testing of Section 2.2 alike);
* closed forms: Appendix D's worst case, the sorting reduction of Section 3.1,
  the residual of the trigonometric equation, rotation covariance;
* textbook distributions: uniformity of theta (Kolmogorov-Smirnov), moments
  of truncated normals (scipy.stats.truncnorm), Philox known answers.
"""
import math
import os

import numpy as np

from oracle import ess, philox

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PI = math.pi
TWO_PI = 2.0 * math.pi


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def line_through(x, nu, t1, t2):
    """Halfspace a^T y <= b whose boundary passes through x(t1), x(t2), x inside."""
    e = lambda t: x * math.cos(t) + nu * math.sin(t)
    p1, p2 = e(t1), e(t2)
    dv = p2 - p1
    a = np.array([dv[1], -dv[0]])
    b = float(a @ p1)
    if a @ x > b:
        a, b = -a, -b
    return a, b


def fig1_cases():
    rows = read_golden("fig1_worked_example.txt")
    x = nu = None
    cases, cur = [], None
    for r in rows:
        if r[0] == "x_t":
            x = np.array([float(v) for v in r[1:]])
        elif r[0] == "nu":
            nu = np.array([float(v) for v in r[1:]])
        elif r[0] == "variant":
            cur = {"name": r[1], "lines": [], "active": []}
            cases.append(cur)
        elif r[0] == "line":
            cur["lines"].append((float(r[1]) * PI, float(r[2]) * PI))
        elif r[0] == "active":
            cur["active"].append((float(r[1]) * PI, float(r[2]) * PI))
    return x, nu, cases


def fig1_problem(x, nu, lines):
    rows = [line_through(x, nu, t1, t2) for t1, t2 in lines]
    return np.array([r[0] for r in rows]), np.array([r[1] for r in rows])


# ---------------------------------------------------------------- pins
def pin_fig1():
    fails = []
    x, nu, cases = fig1_cases()
    for case in cases:
        A, b = fig1_problem(x, nu, case["lines"])
        al, be, hit = ess.roots(A @ x, A @ nu, b)
        for (t1, t2), a_, b_ in zip(case["lines"], al, be):
            if abs(a_ - t1) > 1e-12 or abs(b_ - t2) > 1e-12:
                fails.append(f"fig1 {case['name']}: roots {a_/PI:.6f},{b_/PI:.6f} vs {t1/PI},{t2/PI}")
        lo, hi = ess.alg3_candidates(al, be)
        got = ess.nonempty(lo, hi)
        want = case["active"]
        if len(got) != len(want) or any(abs(g[0] - w[0]) > 1e-12 or abs(g[1] - w[1]) > 1e-12
                                         for g, w in zip(got, want)):
            fails.append(f"fig1 {case['name']}: active {got} vs {want}")
    return fails


def pin_fig2():
    fails = []
    x = np.array([2.0, 0.0])
    nu = np.array([0.0, 1.0])
    a = np.array([-1.0, 0.0])
    for r in read_golden("fig2_edge_cases.txt"):
        c, ratio, case = float(r[0]), float(r[1]), r[2]
        b = -c
        p, q = float(a @ x), float(a @ nu)
        if abs(b / math.hypot(p, q) - ratio) > 1e-15:
            fails.append(f"fig2 c={c}: ratio")
        if case == "invalid":
            if p <= b:
                fails.append("fig2 invalid case has a feasible x_t")
            continue
        al, be, hit = ess.roots(np.array([p]), np.array([q]), np.array([b]))
        al, be, hit = float(al[0]), float(be[0]), bool(hit[0])
        if case in ("no_root", "single_root_tangent"):
            # b/r > 1: no root; b/r = 1: tangent, ignorable (Section 3.2) -> padding
            if hit or al != 0.0 or be != 0.0:
                fails.append(f"fig2 c={c}: expected padding, got {al},{be},{hit}")
        elif case == "two_roots":
            r1, r2 = float(r[3]) * PI, float(r[4]) * PI
            if not hit or abs(al - r1) > 1e-12 or abs(be - r2) > 1e-12:
                fails.append(f"fig2 c={c}: roots {al/PI},{be/PI}")
            lo, hi = ess.alg3_candidates(np.array([al]), np.array([be]))
            got = ess.nonempty(lo, hi)
            if len(got) != 2 or abs(got[0][1] - r1) > 1e-12 or abs(got[1][0] - r2) > 1e-12:
                fails.append(f"fig2 c={c}: active {got}")
        elif case == "single_root_boundary":
            # b/r = -1: the only feasible point of the ellipse is x_t itself
            lo, hi = ess.alg3_candidates(np.array([al]), np.array([be]))
            total = float(np.maximum(hi - lo, 0).sum())
            if not hit or total > 1e-12:
                fails.append(f"fig2 c={c}: boundary case has active length {total}")
    return fails


def pin_fig1_trimmed(eps_values=(1e-3, 0.05)):
    """Section 3.3's trim on Figure 1: every interval [l, u] becomes
    [l + eps, u - eps], except that an end at 0 or 2 pi is the seam through x_t
    itself and stays (the reading taken where the paper is silent).  From the
    figure's active arcs the trimmed set is written down by hand:
    [0, pi/8 - eps], [7 pi/8 + eps, 9 pi/8 - eps], [7 pi/4 + eps, 2 pi].  The
    figure's candidate list also holds an empty candidate (the inactive pair
    (2/5, 4/5) pi), which must stay empty; so must a piece shorter than 2 eps
    and one of zero length."""
    fails = []
    x, nu, cases = fig1_cases()
    for case in cases:
        A, b = fig1_problem(x, nu, case["lines"])
        al, be, _ = ess.roots(A @ x, A @ nu, b)
        lo, hi = ess.alg3_candidates(al, be)
        for eps in eps_values:
            tlo, thi = ess.trim(lo, hi, eps)
            got = ess.nonempty(tlo, thi)
            want = [(l + eps if l > 0 else l, h - eps if h < TWO_PI else h)
                    for l, h in case["active"]]
            if len(got) != len(want) or any(abs(g[0] - w[0]) > 1e-12 or abs(g[1] - w[1]) > 1e-12
                                             for g, w in zip(got, want)):
                fails.append(f"fig1 {case['name']} eps={eps}: trimmed {got} vs {want}")
            # the empty candidate of the inactive row stays empty
            n_empty = int((hi - lo < 0).sum())
            if int((thi - tlo < 0).sum()) < n_empty:
                fails.append(f"fig1 {case['name']} eps={eps}: trim made an empty candidate non-empty")
    # short pieces: zero length in the middle, length eps (< 2 eps), and the
    # seam pieces [0, 0] and [2 pi, 2 pi]
    eps = 1e-3
    lo = np.array([0.0, 1.0, 2.0, 3.0, TWO_PI])
    hi = np.array([0.0, 1.0, 2.0 + eps, 3.5, TWO_PI])
    tlo, thi = ess.trim(lo, hi, eps)
    got = ess.nonempty(tlo, thi)
    if len(got) != 1 or abs(got[0][0] - (3.0 + eps)) > 1e-15 or abs(got[0][1] - (3.5 - eps)) > 1e-15:
        fails.append(f"short pieces after the trim: {got}")
    th, total = ess.sample_theta(tlo, thi, 0.999999)
    if abs(total - (0.5 - 2 * eps)) > 1e-12 or not (3.0 + eps <= th <= 3.5 - eps):
        fails.append(f"theta {th} / total {total} outside the one trimmed piece")
    return fails


def pin_reject_and_stay():
    """Section 3.3's second safeguard: a proposal that violates a constraint is
    rejected and the chain stays at x_t; a proposal on the boundary (a^T x' = b)
    is accepted (the reading taken where the paper is silent).  To make the
    branch fire, the transition is handed projections that claim the row
    never meets the ellipse (q = 0), although the direction nu = (2, 0) does
    cross x_1 <= b: I_act is then the whole circle, theta = 2 pi u by the
    inverse CDF of one piece, and x' = (2 sin theta, 0) by hand.
      chain 0: u = 1/4, b = 1: theta = pi/2, x' = (2, 0) violates: reject, stay at 0
      chain 1: u = 1/20, b = 1: x'_1 = 2 sin(pi/10) < 1: accept
      chain 2: u = 1/4, b = 2: x' = (2, 0) lies on the boundary: accept
    (sin of the float64 nearest pi/2 rounds to 1 exactly, checked below)."""
    fails = []
    A = np.array([[1.0, 0.0]])
    u = np.array([0.25, 0.05, 0.25])
    theta = TWO_PI * u
    if float(np.sin(theta)[0]) != 1.0:
        return ["sin(pi/2) does not round to 1 on this host: the boundary case is not exact"]
    b = np.array([[1.0], [1.0], [2.0]])
    x = np.zeros((3, 2))
    nu = np.tile(np.array([2.0, 0.0]), (3, 1))
    pq = (np.zeros((3, 1)), np.zeros((3, 1)))
    out = ess.transition(A, b, x, nu, u, pq=pq)
    want_rej = [True, False, False]
    if [bool(v) for v in out["rejected"]] != want_rej:
        fails.append(f"rejected {list(out['rejected'])} vs {want_rej}")
    if np.abs(np.asarray(out["theta"]) - theta).max() > 1e-15:
        fails.append(f"theta {out['theta']} vs 2 pi u {theta}")
    if not np.array_equal(out["x_new"][0], x[0]):
        fails.append(f"rejected chain moved to {out['x_new'][0]}")
    for c in (1, 2):
        want = np.array([2.0 * math.sin(theta[c]), 0.0])
        if np.abs(out["x_new"][c] - want).max() > 1e-15:
            fails.append(f"chain {c}: x_new {out['x_new'][c]} vs {want}")
    return fails


def pin_root_residual(seed=11, n=2000):
    """p cos(theta) + q sin(theta) = b at both roots; the arc between them is
    infeasible and the arc through theta = 0 feasible."""
    fails = []
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(n) * 2
    q = rng.standard_normal(n) * 2
    r = np.hypot(p, q)
    b = np.maximum(p, 0) + rng.uniform(0, 1.5, n) * r   # x_t feasible: p <= b
    al, be, hit = ess.roots(p, q, b)
    for i in np.nonzero(hit)[0]:
        for t in (al[i], be[i]):
            res = p[i] * math.cos(t) + q[i] * math.sin(t) - b[i]
            if abs(res) > 1e-12 * (abs(b[i]) + r[i]):
                fails.append(f"residual {res} at row {i}")
                break
        if not (0.0 <= al[i] < be[i] <= TWO_PI):
            fails.append(f"ordering row {i}: {al[i]} {be[i]}")
            continue
        mid = 0.5 * (al[i] + be[i])
        if p[i] * math.cos(mid) + q[i] * math.sin(mid) <= b[i]:
            fails.append(f"midpoint of (alpha, beta) feasible at row {i}")
        outside = 0.5 * al[i] if al[i] > 1e-9 else 0.5 * (be[i] + TWO_PI)
        if p[i] * math.cos(outside) + q[i] * math.sin(outside) > b[i] + 1e-12:
            fails.append(f"point outside (alpha, beta) infeasible at row {i}")
        if len(fails) > 5:
            break
    nohit = ~hit
    # rows without roots: the whole ellipse satisfies the constraint
    t = np.linspace(0, TWO_PI, 64)
    vals = p[nohit, None] * np.cos(t) + q[nohit, None] * np.sin(t) - b[nohit, None]
    if vals.size and vals.max() > 1e-12 * max(1.0, np.abs(b).max()):
        fails.append("padded row is crossed by the ellipse")
    return fails


def pin_alternative_root_forms(seed=23, n=20000):
    """Appendix B's two other forms (Gessner et al., Benavoli et al.) solve the
    same equation: away from their edge cases (r + p and b + p both above
    1e-3 r) each root has residual p cos(theta) + q sin(theta) - b within
    1e-11 (b + r), the arc between alpha and beta is infeasible at its
    midpoint, and alpha, beta equal the tau +- acos form's to 1e-9."""
    fails = []
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(n) * 2
    q = rng.standard_normal(n) * 2
    r = np.hypot(p, q)
    b = np.maximum(p, 0) + rng.uniform(0, 1.5, n) * r
    ok = (r + p > 1e-3 * r) & (np.abs(b + p) > 1e-3 * r)
    p, q, b, r = p[ok], q[ok], b[ok], r[ok]
    a0, b0, h0 = ess.roots(p, q, b)
    for f in (ess.roots_gessner, ess.roots_benavoli):
        al, be, hit = f(p, q, b)
        if not np.array_equal(hit, h0):
            fails.append(f"{f.__name__}: {np.sum(hit != h0)} rows differ in crossing or not")
            continue
        for t in (al, be):
            res = np.abs(p * np.cos(t) + q * np.sin(t) - b)[hit]
            if res.size and res.max() > 1e-11 * (np.abs(b) + r)[hit].max():
                fails.append(f"{f.__name__}: residual {res.max():.3e}")
        mid = 0.5 * (al + be)
        if np.any((p * np.cos(mid) + q * np.sin(mid) <= b)[hit]):
            fails.append(f"{f.__name__}: an arc midpoint is feasible")
        d = np.abs(np.mod(np.concatenate([al - a0, be - b0])[np.tile(hit, 2)] + PI, TWO_PI) - PI)
        if d.size and d.max() > 1e-9:
            fails.append(f"{f.__name__}: differs from tau +- acos by {d.max():.3e}")
    return fails


def pin_rotation_covariance(seed=12, n=500):
    """Replacing (x, nu) by (x cos s + nu sin s, -x sin s + nu cos s) rotates
    every angle by -s (mod 2 pi)."""
    fails = []
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(n)
    q = rng.standard_normal(n)
    b = np.maximum(p, 0) + rng.uniform(0.05, 1.0, n) * np.hypot(p, q)
    s = 0.37
    al, be, hit = ess.roots(p, q, b)
    p2 = p * math.cos(s) + q * math.sin(s)
    q2 = -p * math.sin(s) + q * math.cos(s)
    keep = hit & (p2 < b)   # rotated start must stay feasible
    al2, be2, hit2 = ess.roots(p2, q2, b)
    d1 = np.mod(al[keep] - s - al2[keep] + PI, TWO_PI) - PI
    d2 = np.mod(be[keep] - s - be2[keep] + PI, TWO_PI) - PI
    if np.abs(d1).max(initial=0) > 1e-10 or np.abs(d2).max(initial=0) > 1e-10:
        fails.append(f"rotation covariance off by {np.abs(d1).max()} / {np.abs(d2).max()}")
    return fails


def _same_sets(a, b, tol=1e-12):
    a = [(l, h) for l, h in a if h - l > tol]
    b = [(l, h) for l, h in b if h - l > tol]
    return len(a) == len(b) and all(abs(x[0] - y[0]) <= tol and abs(x[1] - y[1]) <= tol
                                    for x, y in zip(a, b))


def random_interval_sets(rng, n_sets, m_max=8):
    """Random (alpha, beta) sets with forced ties, padding and shared ends."""
    for _ in range(n_sets):
        m = int(rng.integers(1, m_max + 1))
        al = rng.uniform(0, TWO_PI, m)
        be = np.minimum(al + rng.uniform(0, TWO_PI, m), TWO_PI)
        if m > 2 and rng.random() < 0.3:
            al[1] = al[0]                       # tie in alpha
        if m > 3 and rng.random() < 0.3:
            be[2] = al[3]                       # arc ends where another starts
        if rng.random() < 0.3:
            j = int(rng.integers(0, m))
            al[j] = be[j] = 0.0                 # padding row
        bad = be <= al
        be[bad & (al > 0)] = np.minimum(al[bad & (al > 0)] + 1e-3, TWO_PI)
        yield al, be


def pin_alg3_equals_alg2(seed=13, n_sets=3000):
    """Proposition 1: Algorithm 3 gives the same set as Algorithm 2."""
    rng = np.random.default_rng(seed)
    for al, be in random_interval_sets(rng, n_sets):
        lo, hi = ess.alg3_candidates(al, be)
        if not _same_sets(ess.nonempty(lo, hi), ess.alg2_brute_force(al, be)):
            return [f"alg3 != alg2 for alpha={al.tolist()} beta={be.tolist()}"]
    return []


def pin_midpoint_equals_alg2(seed=21, n_cases=400):
    """Section 2.2's likelihood testing at midpoints finds the set that
    Algorithm 2 defines, on random polytopes through random ellipses."""
    rng = np.random.default_rng(seed)
    for case in range(n_cases):
        d = int(rng.integers(1, 5))
        m = int(rng.integers(1, 12))
        A = rng.standard_normal((m, d))
        b = rng.uniform(0.05, 1.5, m)
        x = np.zeros(d)
        for _ in range(200):
            y = rng.standard_normal(d)
            if (A @ y < b).all():
                x = y
                break
        nu = rng.standard_normal(d)
        p, q = A @ x, A @ nu
        al, be, _ = ess.roots(p, q, b)
        want = [pc for pc in ess.alg2_brute_force(al, be) if pc[1] > pc[0]]
        got = ess.midpoint_intervals(p, q, b)
        if not _same_sets(got, want, 1e-12):
            return [f"midpoint != alg2 (case {case}): {got} vs {want}"]
    return []


def pin_dense_grid(seed=14, n_cases=150, n_grid=4001):
    """Active intervals agree with the feasibility of x(theta) on a dense grid."""
    rng = np.random.default_rng(seed)
    step = TWO_PI / (n_grid - 1)
    for case in range(n_cases):
        d = int(rng.integers(1, 5))
        m = int(rng.integers(1, 9))
        A = rng.standard_normal((m, d))
        b = rng.uniform(0.05, 1.5, m)
        x = np.zeros(d)
        for _ in range(200):
            y = rng.standard_normal(d)
            if (A @ y < b).all():
                x = y
                break
        nu = rng.standard_normal(d)
        al, be, _ = ess.roots(A @ x, A @ nu, b)
        lo, hi = ess.alg3_candidates(al, be)
        pieces = ess.nonempty(lo, hi)
        theta, feas = ess.dense_grid_feasible(A, b, x, nu, n_grid)
        inside = np.zeros(n_grid, bool)
        for l, h in pieces:
            inside |= (theta >= l) & (theta <= h)
        # grid points farther than one step from every endpoint must agree
        ends = np.array([e for pc in pieces for e in pc] + list(al) + list(be))
        far = np.min(np.abs(theta[:, None] - ends[None, :]), axis=1) > 2 * step
        if (inside[far] != feas[far]).any():
            return [f"dense grid disagrees (case {case}, d={d}, m={m})"]
    return []


def pin_appendix_d(m=12):
    """Appendix D worst case: I_i = [0, 3^-i] U [2 * 3^-i, 1] (scaled by 2 pi);
    the first k intersect to k + 1 intervals with closed-form ends."""
    fails = []
    for k in range(1, m + 1):
        i = np.arange(1, k + 1)
        al = TWO_PI * 3.0 ** -i
        be = TWO_PI * 2.0 * 3.0 ** -i
        want = [(0.0, TWO_PI * 3.0 ** -k)] + sorted(
            (TWO_PI * 2 * 3.0 ** -j, TWO_PI * 3.0 ** -(j - 1)) for j in range(1, k + 1))
        lo, hi = ess.alg3_candidates(al, be)
        got = ess.nonempty(lo, hi)
        if not _same_sets(got, want, 1e-12):
            fails.append(f"appendix D k={k}: {len(got)} pieces vs {len(want)}")
    return fails


def pin_sorting_reduction(seed=15, m=40):
    """Section 3.1 lower bound: I_i = [0, c_i] U [c_i + eps, 2 pi] reveals the
    sorted order of the c_i."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 6.0, m)
    eps = 0.5 * np.min(np.diff(np.sort(c)))
    lo, hi = ess.alg3_candidates(c, c + eps)
    got = ess.nonempty(lo, hi)
    cs = np.sort(c)
    want = [(0.0, cs[0])] + [(cs[k - 1] + eps, cs[k]) for k in range(1, m)] + [(cs[-1] + eps, TWO_PI)]
    return [] if _same_sets(got, want, 1e-12) else ["sorting reduction order lost"]


def pin_theta_uniform(seed=16, n=20000):
    """theta = F^-1(u) is uniform on I_act (Kolmogorov-Smirnov) and monotone in u."""
    from scipy import stats
    fails = []
    lo = np.array([0.0, 1.0, 2.5, 5.0, 6.0])
    hi = np.array([0.4, 0.9, 3.5, 5.5, TWO_PI])   # second piece empty
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=n)
    th = np.array([ess.sample_theta(lo, hi, v)[0] for v in u])
    ell = np.maximum(hi - lo, 0)
    cum = np.concatenate([[0], np.cumsum(ell)])

    def cdf(t):
        t = np.asarray(t)
        return np.sum(np.clip(t[..., None] - lo, 0, ell), axis=-1) / cum[-1]

    ks = stats.kstest(th, cdf)
    if ks.pvalue < 1e-3:
        fails.append(f"theta not uniform (KS p={ks.pvalue:.2e})")
    inside = np.zeros(n, bool)
    for l, h in zip(lo, hi):
        inside |= (th >= l) & (th <= h) & (h > l)
    if not inside.all():
        fails.append("theta outside the active intervals")
    us = np.sort(u)
    ths = np.array([ess.sample_theta(lo, hi, v)[0] for v in us[:2000]])
    if (np.diff(ths) < 0).any():
        fails.append("theta not monotone in u")
    return fails


def pin_philox_kat():
    fails = []
    for r in read_golden("philox4x32_10_kat.txt"):
        v = [int(t, 16) for t in r]
        out = philox.philox4x32_10(*v[:6])
        if [int(o) for o in out] != v[6:]:
            fails.append(f"philox KAT {r[:6]}")
    return fails


def pin_box_muller(seed=17, n=200000):
    """Normals from the stream: mean 0, variance 1, uncorrelated pair halves,
    Kolmogorov-Smirnov against N(0, 1)."""
    from scipy import stats
    z = philox.normals(seed, 3, np.arange(n // 8), 8)
    fails = []
    flat = z.ravel()
    if abs(flat.mean()) > 5 / math.sqrt(flat.size) or abs(flat.var() - 1) > 5 * math.sqrt(2 / flat.size):
        fails.append(f"normal moments {flat.mean()} {flat.var()}")
    if abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) > 5 / math.sqrt(z.shape[0]):
        fails.append("pair halves correlated")
    if stats.kstest(flat[:50000], "norm").pvalue < 1e-4:
        fails.append("normals fail KS")
    u = philox.uniforms(seed, 0, np.arange(50000))
    if not ((u > 0) & (u < 1)).all() or stats.kstest(u, "uniform").pvalue < 1e-4:
        fails.append("uniforms not U(0,1)")
    return fails


def truncnorm_moments(lo, hi):
    from scipy import stats
    return stats.truncnorm.mean(lo, hi), stats.truncnorm.var(lo, hi)


def pin_chain_box_moments(seed=18, n_chains=300, n_steps=120, burn=20):
    """Independent box truncation: per-coordinate mean and variance have closed
    forms; the chain must match them within Monte Carlo error, and every
    iterate must satisfy A x <= b."""
    import synth
    lo = np.array([-1.0, 0.3, -2.0])
    hi = np.array([3.0, 2.0, -0.5])
    pr = synth.box(lo, hi)
    trace, _, rej = ess.run(pr.A, pr.b, pr.x0, n_chains, n_steps, seed)
    fails = []
    if ((trace @ pr.A.T) > pr.b).any():
        fails.append("iterate violates A x <= b")
    if rej.sum() != 0:
        fails.append(f"float64 chain rejected {rej.sum()} proposals")
    s = trace[burn:]
    for j in range(3):
        mu, var = truncnorm_moments(lo[j], hi[j])
        cm = s[:, :, j].mean(axis=0)          # per-chain means: independent
        se = cm.std(ddof=1) / math.sqrt(n_chains)
        cv = ((s[:, :, j] - mu) ** 2).mean(axis=0)
        sev = cv.std(ddof=1) / math.sqrt(n_chains)
        if abs(cm.mean() - mu) > 5 * se:
            fails.append(f"coord {j}: mean {cm.mean():.4f} vs {mu:.4f} (se {se:.4f})")
        if abs(cv.mean() - var) > 5 * sev:
            fails.append(f"coord {j}: var {cv.mean():.4f} vs {var:.4f} (se {sev:.4f})")
    return fails


def pin_exp1_table(n_chains=400, n_steps=150, burn=30):
    """Section 4.1 table: the closed-form moments printed in the paper agree with
    scipy's truncated normal, and the chain reproduces them."""
    import synth
    fails = []
    for r in read_golden("exp1_univariate_moments.txt"):
        lo, hi, tmu, _, tvar, _, _ = (float(v) for v in r)
        mu, var = truncnorm_moments(lo, hi)
        if abs(mu - tmu) > 6e-5 or abs(var - tvar) > 6e-5:
            fails.append(f"printed moments [{lo},{hi}] disagree with closed form")
        pr = synth.univariate(lo, hi)
        trace, _, _ = ess.run(pr.A, pr.b, pr.x0, n_chains, n_steps, seed=21)
        s = trace[burn:, :, 0]
        cm = s.mean(axis=0)
        se = cm.std(ddof=1) / math.sqrt(n_chains)
        if abs(cm.mean() - tmu) > max(5 * se, 1e-4):
            fails.append(f"[{lo},{hi}] chain mean {cm.mean():.5f} vs {tmu}")
        cv = ((s - mu) ** 2).mean(axis=0)
        sev = cv.std(ddof=1) / math.sqrt(n_chains)
        if abs(cv.mean() - tvar) > max(5 * sev, 1e-4):
            fails.append(f"[{lo},{hi}] chain var {cv.mean():.5f} vs {tvar}")
    return fails


def pin_appendix_a_truncnorm(n_chains=400, n_steps=150, burn=30):
    """Appendix A's change of variables: N(1, 2^2) truncated to [0, 3], sampled
    as u ~ N(0, 1) on the whitened interval and mapped back, matches the
    truncated normal's mean and variance (scipy.stats.truncnorm)."""
    from scipy import stats
    mu, sd, lo, hi = 1.0, 2.0, 0.0, 3.0
    A = np.array([[1.0], [-1.0]])
    b = np.array([hi, -lo])
    L = np.array([[sd]])
    Aw, bw = ess.whiten(A, b, np.array([mu]), L)
    trace, _, _ = ess.run(Aw, bw, np.zeros(1), n_chains, n_steps, seed=31)
    x = ess.unwhiten(trace[burn:].reshape(-1, 1), L, np.array([mu]))[:, 0]
    ref = stats.truncnorm((lo - mu) / sd, (hi - mu) / sd, loc=mu, scale=sd)
    fails = []
    # chains are independent; steps within a chain are close to independent
    # here, and the bounds allow a few standard errors
    se = math.sqrt(ref.var() / (n_chains * 20))
    if abs(x.mean() - ref.mean()) > 5 * se:
        fails.append(f"mean {x.mean():.4f} vs {ref.mean():.4f}")
    if abs(x.var() - ref.var()) > 0.05 * ref.var():
        fails.append(f"variance {x.var():.4f} vs {ref.var():.4f}")
    if x.min() < lo - 1e-12 or x.max() > hi + 1e-12:
        fails.append("sample outside [0, 3]")
    return fails


def pin_rejection_sampling_reference(seed=19, n_chains=200, n_steps=100, burn=20):
    """A small polytope where plain rejection sampling from N(0, I) is exact:
    the chain's mean matches the i.i.d. reference within Monte Carlo error."""
    rng = np.random.default_rng(seed)
    A = np.array([[1.0, 1.0], [-1.0, 0.5], [0.3, -1.0], [0.0, 1.0]])
    b = np.array([0.8, 0.6, 0.9, 0.5])
    z = rng.standard_normal((400000, 2))
    keep = z[(z @ A.T <= b).all(axis=1)]
    ref = keep.mean(axis=0)
    ref_se = keep.std(axis=0) / math.sqrt(len(keep))
    trace, _, _ = ess.run(A, b, np.zeros(2), n_chains, n_steps, seed=22)
    cm = trace[burn:].mean(axis=0)
    se = cm.std(axis=0, ddof=1) / math.sqrt(n_chains)
    bad = np.abs(cm.mean(axis=0) - ref) > 5 * np.sqrt(se ** 2 + ref_se ** 2)
    return [f"mean {cm.mean(axis=0)} vs rejection sampling {ref}"] if bad.any() else []


FAST_PINS = [pin_fig1, pin_fig2, pin_fig1_trimmed, pin_reject_and_stay, pin_root_residual,
             pin_alternative_root_forms, pin_rotation_covariance,
             pin_alg3_equals_alg2, pin_midpoint_equals_alg2, pin_dense_grid, pin_appendix_d,
             pin_sorting_reduction,
             pin_theta_uniform, pin_philox_kat, pin_box_muller]
CHAIN_PINS = [pin_chain_box_moments, pin_exp1_table, pin_rejection_sampling_reference,
              pin_appendix_a_truncnorm]
