"""Comparison rules between the HIP path and the CPU oracle.

Floating-point bar (float32 storage, float64 roots and interval ends):
* interval ends: within TOL_ANG = 1e-5 * 2 pi, after dropping pieces shorter
  than TOL_ANG on either side (a piece that short can appear or vanish under
  float32 rounding of the projections);
* the new state: |x_gpu - x_ref|_inf <= 1e-5 * max(1, |x_ref|_inf);
* a differing accept/reject decision is allowed only where some slack
  b_i - a_i^T x' is within the float32 rounding bound of the dot product,
  2 d 2^-24 sum_j |a_ij x'_j|, widened by what the state tolerance moves it.
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi
TOL_ANG = 1e-5 * TWO_PI
TOL_X = 1e-5


def pieces(arr, n, min_len):
    return [(float(l), float(h)) for l, h in arr[:n] if h - l > min_len]


def intervals_match(gpu, ref, tol=TOL_ANG):
    """Every piece longer than tol on one side has a partner within tol."""
    g = [p for p in gpu if p[1] - p[0] > tol]
    r = [p for p in ref if p[1] - p[0] > tol]

    def covered(a, bs):
        return any(abs(a[0] - b[0]) <= tol and abs(a[1] - b[1]) <= tol for b in bs)

    return all(covered(a, ref) for a in g) and all(covered(a, gpu) for a in r)


def fp32_dot_bound(A, x):
    d = A.shape[1]
    return 2 * d * 2.0 ** -24 * (np.abs(A) @ np.abs(x).T).T   # (C, m)


def _state_check(A, b, c, x_gpu, rejected_gpu, ref, tol_x):
    """Chain c's accept/reject decision and new state against the oracle's
    transition `ref`: returns ("fail" message | None, excused)."""
    rg, rr = bool(rejected_gpu), bool(ref["rejected"][c])
    if rg != rr:
        xp = ref["x_prop"][c]
        slack = (b[c] if np.ndim(b) == 2 else b) - A @ xp
        # float32 dot-product rounding plus the state tolerance below
        bound = fp32_dot_bound(A, xp[None, :])[0] + tol_x * (np.abs(A) @ np.maximum(np.abs(xp), 1.0))
        if np.any(np.abs(slack) <= bound):
            return None, True
        return f"chain {c}: rejected gpu={rg} ref={rr}, min slack {slack.min():.3e}", False
    xr = ref["x_new"][c]
    err = np.max(np.abs(x_gpu - xr))
    if err > tol_x * max(1.0, np.max(np.abs(xr))):
        return f"chain {c}: |dx| = {err:.3e}", False
    return None, False


def compare_transition(A, b, x, nu, u, gpu, ref, tol_ang=TOL_ANG, tol_x=TOL_X):
    """Returns (failures, n_excused) for one explicit transition."""
    fails = []
    excused = 0
    n_int = gpu["n_intervals"]
    for c in range(x.shape[0]):
        gi = pieces(gpu["intervals"][c], n_int[c], 0.0)
        if not intervals_match(gi, ref["intervals"][c], tol_ang):
            fails.append(f"chain {c}: intervals {gi[:4]} vs {ref['intervals'][c][:4]}")
            continue
        msg, exc = _state_check(A, b, c, gpu["x_new"][c], gpu["rejected"][c], ref, tol_x)
        excused += exc
        if msg:
            fails.append(msg)
    return fails, excused


def compare_states(A, b, x_new, rejected, ref, tol_x=TOL_X):
    """The state part of a transition (the accept/reject decision and the new
    x) for every chain.  Returns (failures, n_excused)."""
    fails = []
    excused = 0
    for c in range(x_new.shape[0]):
        msg, exc = _state_check(A, b, c, x_new[c], rejected[c], ref, tol_x)
        excused += exc
        if msg:
            fails.append(msg)
    return fails, excused


def chain_states(A, b, n, store, x0=None, seed=20240714, pool=32, burn=3, span=8):
    """n strictly interior states of {A x <= b} taken from float64 oracle
    chains (Algorithm 1 run from x0, default 0, for burn + span steps; the
    states after the burn-in).  Rows of A and the states are rounded to
    `store`, as the code under test holds them, and every kept state clears
    each constraint by four times the float32 rounding bound of its dot
    product, so a float32 check cannot call it infeasible.  States are
    shuffled and repeated to fill n rows."""
    from oracle import ess as ref_ess

    A_s = np.asarray(A, np.float64).astype(store).astype(np.float64)
    b = np.asarray(b, np.float64)
    d = A_s.shape[1]
    x0 = np.zeros(d) if x0 is None else np.asarray(x0, np.float64)
    eps = 1e-6 if store == np.float32 else 0.0
    tr, _, _ = ref_ess.run(A_s, b, x0, pool, burn + span, seed, eps=eps, store=store)
    cand = tr[burn:].reshape(-1, d)
    slack = b[None, :] - cand @ A_s.T
    ok = (slack > 4.0 * fp32_dot_bound(A_s, cand) + 1e-12).all(axis=1)
    ok &= np.abs(cand).max(axis=1) > 0.0
    cand = cand[ok]
    assert len(cand) >= min(n, pool), f"only {len(cand)} usable chain states"
    rng = np.random.default_rng(seed)
    cand = cand[rng.permutation(len(cand))]
    reps = -(-n // len(cand))
    return np.tile(cand, (reps, 1))[:n].astype(store)
