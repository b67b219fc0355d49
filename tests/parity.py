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


def compare_transition(A, b, x, nu, u, gpu, ref, tol_ang=TOL_ANG, tol_x=TOL_X):
    """Returns (failures, n_excused) for one explicit transition."""
    fails = []
    excused = 0
    C = x.shape[0]
    n_int = gpu["n_intervals"]
    for c in range(C):
        gi = pieces(gpu["intervals"][c], n_int[c], 0.0)
        if not intervals_match(gi, ref["intervals"][c], tol_ang):
            fails.append(f"chain {c}: intervals {gi[:4]} vs {ref['intervals'][c][:4]}")
            continue
        rg, rr = bool(gpu["rejected"][c]), bool(ref["rejected"][c])
        if rg != rr:
            xp = ref["x_prop"][c]
            slack = (b[c] if np.ndim(b) == 2 else b) - A @ xp
            # float32 dot-product rounding plus the state tolerance below
            bound = fp32_dot_bound(A, xp[None, :])[0] + tol_x * (np.abs(A) @ np.maximum(np.abs(xp), 1.0))
            if np.any(np.abs(slack) <= bound):
                excused += 1
                continue
            fails.append(f"chain {c}: rejected gpu={rg} ref={rr}, min slack {slack.min():.3e}")
            continue
        xr = ref["x_new"][c]
        err = np.max(np.abs(gpu["x_new"][c] - xr))
        if err > tol_x * max(1.0, np.max(np.abs(xr))):
            fails.append(f"chain {c}: |dx| = {err:.3e}")
    return fails, excused
