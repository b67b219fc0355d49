"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X)."""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import ess as ref_ess
from oracle import philox as ref_philox
from parity import (TOL_ANG, chain_states, compare_states, compare_transition, pieces,
                    intervals_match)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_10449_amd as E
    E.lib()
    return E


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def explicit_case(E, A, b, C, precision, seed, eps, n_ref=None, rng_seed=0, x0=None):
    """One explicit transition on the GPU and in the oracle on identical inputs."""
    rng = np.random.default_rng(rng_seed)
    npdt = np.float32 if precision == 32 else np.float64
    # generic mid-chain states (x = 0 would make every p = a_i^T x zero)
    x = chain_states(A, b, C, npdt, x0=x0, seed=rng_seed)
    assert (np.abs(x).max(axis=1) == 0).mean() <= 0.05
    nu = rng.standard_normal(x.shape).astype(npdt)
    u = rng.uniform(size=C)
    s = E.Sampler(A, b, x, C, seed=seed, precision=precision, trim_eps=eps)
    out = s.transition_explicit(x, nu, u)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    s.close()
    idx = np.arange(C) if n_ref is None else np.linspace(0, C - 1, n_ref).astype(int)
    Ab = A.astype(npdt).astype(np.float64)
    sub = {k: (v[idx] if k != "pq" else v[:, idx]) for k, v in g.items()}
    ref = ref_ess.transition(Ab, b, x[idx].astype(np.float64), nu[idx].astype(np.float64), u[idx],
                             eps=eps, store=npdt)
    # second tier: the oracle fed the projections the kernels used
    ref2 = ref_ess.transition(Ab, b, x[idx].astype(np.float64), nu[idx].astype(np.float64), u[idx],
                              eps=eps, store=npdt, pq=(sub["pq"][0], sub["pq"][1]))
    return Ab, x[idx].astype(np.float64), nu[idx], u[idx], sub, ref, ref2


CASES = [
    # name, d, m, C, precision, eps
    ("ragged_f32", 37, 150, 300, 32, 1e-6),
    ("bm128_f32", 200, 1030, 600, 32, 1e-6),
    # d > 192 where 128 x 128 tiles would not fill the device: the split
    # bfloat16 projection on 64 x 64 tiles, ragged in rows, chains and K
    ("split64_ragged_f32", 229, 777, 333, 32, 1e-6),
    ("small_f64", 10, 20, 16, 64, 0.0),
    ("ragged_f64", 65, 300, 130, 64, 0.0),
    ("univariate_f32", 1, 2, 64, 32, 0.0),
    ("one_chain_f32", 50, 100, 1, 32, 1e-6),
    ("max_m_f32", 64, 4096, 64, 32, 1e-6),
    # more than 256 chains take the kernels tuned for occupancy; 256 or fewer
    # take the 512-thread kernels with bucket refinement
    ("many_m500_f64", 30, 500, 300, 64, 0.0),
    ("many_m1000_f32", 40, 1000, 300, 32, 1e-6),
    ("many_m3000_f32", 40, 3000, 270, 32, 1e-6),
    ("many_max_m_f64", 20, 4096, 260, 64, 0.0),
    # more than 4096 rows: chunked passes, keys-only full sort
    ("large_m_f32", 40, 6000, 24, 32, 1e-6),
    ("large_m_f64", 30, 9000, 8, 64, 0.0),
    ("large_m_many_f32", 30, 5000, 300, 32, 1e-6),
    ("max_large_m_f32", 20, 16384, 4, 32, 1e-6),
    # more than 16384 rows: the full sort's keys in device memory
    ("large_m_global_keys_f32", 12, 32768, 6, 32, 1e-6),
    ("large_m_global_keys_max_f64", 8, 65536, 2, 64, 0.0),
]
LARGE = [c for c in CASES if c[0].startswith("large_m")]


@pytest.mark.parametrize("name,d,m,C,precision,eps", CASES, ids=[c[0] for c in CASES])
def test_explicit_transition_matches_oracle(E, name, d, m, C, precision, eps):
    say(f"[explicit] {name} d={d} m={m} C={C} prec={precision}")
    rng = np.random.default_rng(d * 7 + m)
    x0 = None
    if name.startswith("univariate"):
        pr = synth.univariate(-1.0, 3.0)
        A, b, x0 = pr.A, pr.b, pr.x0
    else:
        A = rng.standard_normal((m, d)) / math.sqrt(d)
        b = rng.uniform(0.5, 1.5, m)
    Ab, x, nu, u, g, ref, ref2 = explicit_case(E, A, b, C, precision, seed=5, eps=eps,
                                               n_ref=min(C, 96), rng_seed=m, x0=x0)
    fails, excused = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, "\n".join(fails[:10])
    assert excused <= max(1, len(u) // 20)
    # tier 2: same projections -> intervals and theta agree to the root solve's
    # rounding: float64 trig in float64 mode; float32 trig away from tangency in
    # float32 mode (a few 1e-7 rad, bounded here by 1e-5)
    tol2 = 1e-9 if precision == 64 else 1e-5
    for c in range(len(u)):
        gi = pieces(g["intervals"][c], g["n_intervals"][c], 0.0)
        assert intervals_match(gi, ref2["intervals"][c], tol2), (c, gi, ref2["intervals"][c])
        assert abs(g["theta"][c] - ref2["theta"][c]) <= tol2 * max(1.0, len(gi)), c


def test_near_tangent_rows_cross_both_root_branches(E):
    """With x = 0 and per-chain b, every row's b / r is set in [0.97, 1.03], so
    the float32 root solve's miss pretest (b / r >= 1.01 in float32) and its
    angles near tangency (arcs down to zero length) are both exercised.
    Tier 1 against the oracle; tier 2 with the oracle fed the kernel's own
    projections: interval ends and theta within 2e-6 rad (float32 atan2 and
    the half-angle form of acos are within a few 1e-7 rad)."""
    say("[explicit] near-tangent rows")
    rng = np.random.default_rng(17)
    d, m, C = 32, 512, 64
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    A32 = A.astype(np.float32).astype(np.float64)
    x = np.zeros((C, d), np.float32)
    nu = rng.standard_normal((C, d)).astype(np.float32)
    q = nu.astype(np.float64) @ A32.T
    z = rng.uniform(0.97, 1.03, (C, m))
    b = np.maximum(z * np.abs(q), 1e-3)
    u = rng.uniform(size=C)
    s = E.Sampler(A, b, x, C, seed=1, precision=32, trim_eps=1e-6)
    g = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
    s.close()
    x64, nu64 = x.astype(np.float64), nu.astype(np.float64)
    ref = ref_ess.transition(A32, b, x64, nu64, u, eps=1e-6, store=np.float32)
    fails, excused = compare_transition(A32, b, x64, nu64, u, g, ref)
    assert not fails, "\n".join(fails[:10])
    assert excused <= 2
    ref2 = ref_ess.transition(A32, b, x64, nu64, u, eps=1e-6, store=np.float32,
                              pq=(g["pq"][0], g["pq"][1]))
    for c in range(C):
        gi = pieces(g["intervals"][c], g["n_intervals"][c], 0.0)
        assert intervals_match(gi, ref2["intervals"][c], 2e-6), (c, gi, ref2["intervals"][c])
        assert abs(g["theta"][c] - ref2["theta"][c]) <= 2e-6 * max(1.0, len(gi)), c


@pytest.mark.parametrize("roots", ["in_kernel", "prepass"])
def test_explicit_full_size_gp_rbf(E, monkeypatch, roots):
    """d=1000, m=2000, 1024 chains (the benchmarked shape and kernel), from
    mid-chain states: 128 sampled chains, tier 1 and tier 2.  `prepass`: the
    measured alternative with every root solved ahead of the per-chain kernel
    (ESS_ROOTS_PREPASS)."""
    if roots == "prepass":
        monkeypatch.setenv("ESS_ROOTS_PREPASS", "1")
    say(f"[explicit] gp_rbf full size, roots {roots}")
    pr = synth.gp_rbf()
    Ab, x, nu, u, g, ref, ref2 = explicit_case(E, pr.A, pr.b, pr.n_chains, 32, seed=0, eps=1e-6,
                                               n_ref=128, rng_seed=3)
    assert len(np.unique(x, axis=0)) >= 100
    fails, excused = compare_transition(Ab, pr.b, x, nu, u, g, ref)
    assert not fails, "\n".join(fails[:10])
    assert excused <= 3
    for c in range(len(u)):
        gi = pieces(g["intervals"][c], g["n_intervals"][c], 0.0)
        assert intervals_match(gi, ref2["intervals"][c], 1e-5), (c, gi, ref2["intervals"][c])
        assert abs(g["theta"][c] - ref2["theta"][c]) <= 1e-5 * max(1.0, len(gi)), c


def test_no_constraint_crosses_the_ellipse(E):
    """All rows padded (b / r > 1): the active set is the whole ellipse."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 8)) * 1e-3
    b = np.full(40, 10.0)
    Ab, x, nu, u, g, ref, _ = explicit_case(E, A, b, 32, 32, seed=1, eps=1e-6)
    assert (g["n_intervals"] == 1).all()
    assert np.allclose(g["intervals"][:, 0], [0.0, 2 * math.pi])
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails


def fig2_rows():
    import os
    rows = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fig2_edge_cases.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            if f[2] != "invalid":
                rows.append((float(f[0]), f[2]))
    return rows


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("c,case", fig2_rows(), ids=[r[1] for r in fig2_rows()])
def test_figure_2_edge_cases_on_the_gpu(E, precision, c, case):
    """Figure 2's cases through the kernels (x = (2, 0), nu = (0, 1), feasible
    side x_1 >= c), untrimmed: no root and the tangent leave the whole
    ellipse, and two roots cut out (2 pi / 3, 4 pi / 3).  With c = 2 the
    figure's x_t lies on the boundary (b / r = -1), which the library refuses:
    it requires a strictly interior state."""
    npdt = np.float32 if precision == 32 else np.float64
    A = np.array([[-1.0, 0.0]])
    b = np.array([-c])
    C = 4
    x = np.tile(np.array([2.0, 0.0], npdt), (C, 1))
    nu = np.tile(np.array([0.0, 1.0], npdt), (C, 1))
    u = (np.arange(C) + 0.5) / C
    s = E.Sampler(A, b, np.array([3.0, 0.0]), C, seed=0, precision=precision, trim_eps=0.0)
    if case == "single_root_boundary":
        with pytest.raises(E.EssError, match="not strictly feasible"):
            s.transition_explicit(x, nu, u)
        s.close()
        return
    g = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
    s.close()
    want = ([(0.0, 2 * math.pi)] if case != "two_roots"
            else [(0.0, 2 * math.pi / 3), (4 * math.pi / 3, 2 * math.pi)])
    tol = 1e-6 if precision == 32 else 1e-12
    for ch in range(C):
        got = pieces(g["intervals"][ch], g["n_intervals"][ch], 0.0)
        assert len(got) == len(want), (ch, got)
        for (lo, hi), (wlo, whi) in zip(got, want):
            assert abs(lo - wlo) <= tol and abs(hi - whi) <= tol, (ch, got)
    assert (g["rejected"] == 0).all()


@pytest.mark.parametrize("precision,gap,eps", [(64, 1e-7, 1e-6), (32, 1e-5, 1e-4)])
def test_trimmed_away_active_set_stays_and_counts_a_rejection(E, precision, gap, eps):
    """Two forbidden arcs leave only [0, gap/2] and [2 pi - gap/2, 2 pi] around
    the current state; trimming by eps > gap/2 empties both (Section 3.3), so
    the chain stays where it is, the step is reported as rejected, and each
    chain's rejection counter grows by one."""
    alpha = np.array([gap / 2, 3.0])
    beta = np.array([3.0, 2 * math.pi - gap / 2])
    A, b = arcs_problem(alpha, beta)
    npdt = np.float32 if precision == 32 else np.float64
    C = 8
    x = np.tile(np.array([1.0, 0.0], npdt), (C, 1))
    nu = np.tile(np.array([0.0, 1.0], npdt), (C, 1))
    u = (np.arange(C) + 0.5) / C
    s = E.Sampler(A, b, x, C, seed=0, precision=precision, trim_eps=eps)
    g = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
    assert (g["n_intervals"] == 0).all() and (g["rejected"] == 1).all()
    assert np.array_equal(g["x_new"], x)
    assert (s.rejections() == 1).all()
    ref = ref_ess.transition(A.astype(npdt).astype(np.float64), b, x.astype(np.float64),
                             nu.astype(np.float64), u, eps=eps, store=npdt)
    assert np.asarray(ref["rejected"]).all()
    s.close()


@pytest.mark.parametrize("precision", [32, 64])
def test_philox_stream_matches_oracle(E, precision):
    pr = synth.small_fp64(d=33, m=20, n_chains=70)
    s = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=0xDEADBEEF12345, precision=precision)
    for step in (0, 1, 12345):
        nu, u = s.draw(step)
        nu, u = nu.cpu().numpy(), u.cpu().numpy()
        rn = ref_philox.normals(0xDEADBEEF12345, step, np.arange(pr.n_chains), pr.d)
        ru = ref_philox.uniforms(0xDEADBEEF12345, step, np.arange(pr.n_chains))
        assert np.array_equal(u, ru)                 # integer path: bit-exact
        if precision == 64:
            assert np.max(np.abs(nu - rn) / np.maximum(np.abs(rn), 1e-300)) < 1e-14
        else:
            diff = nu != rn.astype(np.float32)
            assert diff.mean() < 1e-3                 # libm ulp ties only
            assert np.max(np.abs(nu - rn)) < 1e-6
    s.close()


def test_run_matches_oracle_fp64(E):
    """Seeded float64 runs follow the oracle's trajectories step by step."""
    pr = synth.small_fp64()
    T = 60
    s = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=0, precision=64, trim_eps=0.0)
    tr, nrej = s.run(T)
    tr = tr.cpu().numpy()
    rtr, _, rrej = ref_ess.run(pr.A, pr.b, pr.x0, pr.n_chains, T, seed=0)
    err = np.abs(tr - rtr).max(axis=(0, 2))
    assert (err < 1e-9).all(), err
    assert nrej == rrej.sum() == 0
    s.close()


def run_step_by_step(E, s, A, b, seed, T, idx, eps, store=np.float32):
    """T single-step runs of sampler s; after each, the sampled chains idx are
    compared with one oracle transition from the GPU's previous state with
    the step's Philox draws (so errors cannot accumulate): the decision and
    the new state to 1e-5.  Returns the number of excused decisions."""
    C, d = s.n_chains, s.d
    A_s = np.asarray(A, np.float64).astype(store).astype(np.float64)
    x_prev = s.state()[0].cpu().numpy().astype(np.float64)
    rej_prev = s.rejections()
    excused = 0
    moved = 0
    for t in range(T):
        _, step = s.state()
        s.run(1, keep_trace=False)
        x_next = s.state()[0].cpu().numpy().astype(np.float64)
        rej = s.rejections()
        nu = ref_philox.normals(seed, step, idx, d).astype(store).astype(np.float64)
        u = ref_philox.uniforms(seed, step, idx)
        bs = b[idx] if np.ndim(b) == 2 else b   # one b per chain, or shared
        ref = ref_ess.transition(A_s, bs, x_prev[idx], nu, u, eps=eps, store=store)
        fails, exc = compare_states(A_s, bs, x_next[idx], (rej - rej_prev)[idx], ref)
        assert not fails, (t, fails[:10])
        excused += exc
        moved += int((x_next[idx] != x_prev[idx]).any(axis=1).sum())
        x_prev, rej_prev = x_next, rej
    assert moved >= 0.9 * T * len(idx)
    return excused


@pytest.mark.parametrize("workload,C", [("box_halfspace", 300), ("gp_rbf", 1024)])
def test_run_matches_oracle_fp32_per_step(E, workload, C):
    """The production run path (graph replay, more than 256 chains, so the
    kernels tuned for occupancy; gp_rbf is the benchmarked shape and kernel),
    checked one step at a time from the states it reached."""
    say(f"[run] per-step {workload} C={C}")
    pr = getattr(synth, workload)(n_chains=C)
    s = E.Sampler(pr.A, pr.b, pr.x0, C, seed=0, precision=32, trim_eps=1e-6)
    idx = np.linspace(0, C - 1, 96).astype(int)
    excused = run_step_by_step(E, s, pr.A, pr.b, 0, 4, idx, 1e-6)
    assert excused <= 2
    s.close()


@pytest.mark.parametrize("d,m,C", [(1300, 700, 300), (2500, 1500, 300)])
def test_run_matches_oracle_per_step_wide(E, d, m, C):
    """d above twice the threads per chain (256 and 512 threads here), so each
    thread draws several of the next direction's element pairs: the first
    ahead of the move, the rest in the move's loop.  The run path hands each
    step's draw to the next, checked one step at a time against the oracle."""
    say(f"[run] per-step wide d={d} m={m} C={C}")
    rng = np.random.default_rng(d)
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, m)
    s = E.Sampler(A, b, np.zeros(d), C, seed=11, precision=32, trim_eps=1e-6)
    s.run(2, keep_trace=False)                  # generic states first
    idx = np.linspace(0, C - 1, 48).astype(int)
    excused = run_step_by_step(E, s, A, b, 11, 3, idx, 1e-6)
    assert excused <= 2
    s.close()


def test_run_matches_oracle_per_step_warm_family(E):
    """The warm-start family's shape (d=256, m=768, 32 right-hand sides x 64
    chains = 2048 chains with one b per chain), the context the batched +
    warm-start comparison runs, checked one step at a time against the
    oracle."""
    A, b0, draw = synth.warm_family()
    B = np.repeat(draw(np.random.default_rng(3), 32), 64, axis=0)
    C, d = B.shape[0], A.shape[1]
    s = E.Sampler(A, B, np.zeros(d), C, seed=7, precision=32, trim_eps=1e-6)
    s.run(3, keep_trace=False)                  # generic states first
    idx = np.linspace(0, C - 1, 96).astype(int)
    excused = run_step_by_step(E, s, A, B, 7, 3, idx, 1e-6)
    assert excused <= 2
    s.close()


def test_thin_trace_and_checkpoint_resume(E):
    pr = synth.box_halfspace(n_chains=300)
    a = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=9, precision=32)
    full, _ = a.run(12, thin=3)
    b = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=9, precision=32)
    half, _ = b.run(6, thin=3)
    x, step = b.state()
    assert step == 6
    c = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=9, precision=32)
    c.set_state(x, step)
    rest, _ = c.run(6, thin=3)
    assert torch.equal(full[:2], half) and torch.equal(full[2:], rest)
    # same seed, same trace; rerun is bit-identical
    d = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=9, precision=32)
    again, _ = d.run(12, thin=3)
    assert torch.equal(full, again)
    for s in (a, b, c, d):
        s.close()


def test_iterates_stay_feasible(E):
    pr = synth.box_halfspace(n_chains=512)
    s = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=2, precision=32)
    tr, nrej = s.run(50)
    X = tr.double().cpu().numpy()
    slack = pr.b - X @ pr.A.T
    bound = 2 * pr.d * 2.0 ** -24 * (np.abs(X) @ np.abs(pr.A).T)
    assert (slack >= -bound).all()
    assert s.rejections().sum() == nrej
    s.close()


def test_infeasible_set_state_keeps_the_state(E):
    """A state that fails the strict start check raises, and the context
    keeps its previous state, step and projections: it then runs exactly as a
    twin context that never saw the bad state."""
    pr = synth.box_halfspace(n_chains=300)
    a = E.Sampler(pr.A, pr.b, pr.x0, 300, seed=4, precision=32)
    b = E.Sampler(pr.A, pr.b, pr.x0, 300, seed=4, precision=32)
    a.run(3, keep_trace=False)
    b.run(3, keep_trace=False)
    x, step = a.state()
    bad = x.clone()
    bad[0, 0] = 1.0e6   # outside the box
    with pytest.raises(E.EssError) as ei:
        a.set_state(bad, step)
    assert ei.value.status == E.ESS_ERR_INFEASIBLE_START
    x2, step2 = a.state()
    assert torch.equal(x2, x) and step2 == step
    ta, _ = a.run(4)
    tb, _ = b.run(4)
    assert torch.equal(ta, tb)
    a.close()
    b.close()


def test_errors_are_reported(E):
    pr = synth.small_fp64()
    with pytest.raises(E.EssError) as ei:
        E.Sampler(pr.A, pr.b, np.full(pr.d, 50.0), 4, precision=64)
    assert ei.value.status == E.ESS_ERR_INFEASIBLE_START and "chain 0" in str(ei.value)
    with pytest.raises(E.EssError) as ei:
        E.Sampler(np.zeros((65537, 3)), np.ones(65537), np.zeros(3), 2)
    assert ei.value.status == E.ESS_ERR_UNSUPPORTED
    with pytest.raises(E.EssError) as ei:
        E.Sampler(pr.A, pr.b, pr.x0, 4, precision=16)
    assert ei.value.status == E.ESS_ERR_INVALID_ARG
    prob = E.EssProblem(3, 2, 4, 32, None, None, None, 0, 0.0, 0)
    with pytest.raises(E.EssError):
        E.ess_init(prob)


def arcs_problem(alpha, beta):
    """d = 2 rows whose forbidden arcs on the ellipse through x = e1, nu = e2
    are exactly (alpha_i, beta_i): a_i = (cos tau, sin tau), b_i = cos phi with
    tau, phi the arc's centre and half-width (Appendix B read backwards)."""
    tau = 0.5 * (alpha + beta)
    phi = 0.5 * (beta - alpha)
    A = np.stack([np.cos(tau), np.sin(tau)], axis=1)
    return A, np.cos(phi)


def run_arcs(E, alpha, beta, precision, full_sort=False, C=8, method="alg3"):
    A, b = arcs_problem(alpha, beta)
    npdt = np.float32 if precision == 32 else np.float64
    x = np.tile(np.array([1.0, 0.0], npdt), (C, 1))
    nu = np.tile(np.array([0.0, 1.0], npdt), (C, 1))
    u = (np.arange(C) + 0.5) / C
    s = E.Sampler(A, b, x, C, seed=0, precision=precision, trim_eps=0.0, full_sort=full_sort,
                  method=method)
    g = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
    s.close()
    Ab = A.astype(npdt).astype(np.float64)
    ref = ref_ess.transition(Ab, b, x.astype(np.float64), nu.astype(np.float64), u, store=npdt,
                             method=method)
    return Ab, b, x.astype(np.float64), nu, u, g, ref


@pytest.mark.parametrize("precision", [32, 64])
def test_sorting_reduction_takes_full_path(E, precision):
    """Section 3.1's reduction: every row ends a gap, so 300 survivors overflow
    the bucket path and the chain is sorted in full.  Arcs are kept wider than
    float32 rounding of A can blur (about 3.5e-4 rad)."""
    rng = np.random.default_rng(7)
    c = 0.1 + 5.9 * (np.arange(300) + rng.uniform(0.2, 0.4, 300)) / 300
    Ab, b, x, nu, u, g, ref = run_arcs(E, c, c + 0.005, precision)
    assert (g["n_intervals"] == 301).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, fails[:5]


@pytest.mark.parametrize("precision,n_arcs", [(32, 20), (32, 100), (64, 60)])
def test_many_survivors_stay_on_the_bucket_path(E, precision, n_arcs):
    """Section 3.1's construction with fewer gaps than the bucket path holds:
    every row is a survivor (20 to 100 of them), so the inverse CDF runs over
    many candidates on the bucket path (its parallel form from 16 on)."""
    rng = np.random.default_rng(11 + n_arcs)
    c = 0.1 + 5.9 * (np.arange(n_arcs) + rng.uniform(0.2, 0.4, n_arcs)) / n_arcs
    Ab, b, x, nu, u, g, ref = run_arcs(E, c, c + 0.005, precision)
    assert (g["n_intervals"] == n_arcs + 1).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, fails[:5]


@pytest.mark.parametrize("precision,m", [(32, 7), (64, 14)])
def test_appendix_d_nested_arcs_in_one_bucket(E, precision, m):
    """Appendix D's worst case, I_i = [0, 3^-i] U [2 3^-i, 1] (scaled by 2 pi),
    placed at pi / 2 so the arcs are well conditioned: the nested arcs share a
    bucket and the in-bucket refinement must recover all m + 1 intervals."""
    i = np.arange(1, m + 1)
    al = 2 * np.pi * 3.0 ** -i
    Ab, b, x, nu, u, g, ref = run_arcs(E, 0.5 * np.pi + al, 0.5 * np.pi + 2 * al, precision)
    assert (g["n_intervals"] == m + 1).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, fails[:5]


def coarse_survivors(alpha, beta, nb=2048):
    """Rows whose alpha reaches the running max of beta over all rows of
    earlier buckets, with nb equal buckets of [0, 2 pi) (counted per chain)."""
    out = []
    for a, be in zip(alpha, beta):
        hit = be > 0
        a, be = a[hit], be[hit]
        bk = np.minimum((a * nb / (2 * math.pi)).astype(int), nb - 1)
        top = np.zeros(nb)
        np.maximum.at(top, bk, be)
        g = np.concatenate([[0.0], np.maximum.accumulate(top)[:-1]])
        out.append(int((a >= g[bk]).sum()))
    return out


def assert_same_as_full_sort(E, A, b, x, nu, u, precision, eps):
    outs = []
    for full in (False, True):
        s = E.Sampler(A, b, x, x.shape[0], seed=5, precision=precision, trim_eps=eps,
                      full_sort=full)
        outs.append({k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()})
        s.close()
    a, f = outs
    assert np.array_equal(a["n_intervals"], f["n_intervals"])
    assert np.abs(a["intervals"] - f["intervals"]).max() <= 1e-13
    assert np.abs(a["theta"] - f["theta"]).max() <= 1e-12
    assert np.array_equal(a["rejected"], f["rejected"])
    return a


@pytest.mark.parametrize("precision", [32, 64])
def test_section_4_2_crowded_buckets_are_refined(E, precision):
    """Section 4.2's unnormalised instance at d = m = 4000 from its start x0:
    the state sits within [0, 1] of every constraint while |a_i| is about 63,
    so the alphas crowd the first buckets and about 300 rows survive the
    2048-bucket filter.  The chain leaves the fast kernel and the bucket path
    with refined buckets must give what the oracle and the full sort give."""
    pr = synth.paper_highdim(d=4000)
    C = 3
    npdt = np.float32 if precision == 32 else np.float64
    rng = np.random.default_rng(42)
    x = np.tile(pr.x0, (C, 1)).astype(npdt)
    nu = rng.standard_normal(x.shape).astype(npdt)
    u = rng.uniform(size=C)
    Ab = pr.A.astype(npdt).astype(np.float64)
    ref = ref_ess.transition(Ab, pr.b, x.astype(np.float64), nu.astype(np.float64), u,
                             eps=1e-6, store=npdt)
    surv = coarse_survivors(ref["alpha"], ref["beta"])
    say("coarse survivors", surv)
    assert min(surv) > 128
    g = assert_same_as_full_sort(E, pr.A, pr.b, x, nu, u, precision, 1e-6)
    fails, _ = compare_transition(Ab, pr.b, x.astype(np.float64), nu, u, g, ref)
    assert not fails, fails[:5]


@pytest.mark.parametrize("precision", [32, 64])
def test_large_m_overflow_takes_keys_only_full_sort(E, precision):
    """300 disjoint arcs (Section 3.1's reduction) among 6000 rows that never
    meet the ellipse (b / r = 5): more than 4096 rows, survivors spread over
    the circle, so refinement cannot help and the keys-only full sort runs."""
    rng = np.random.default_rng(17)
    c = 0.1 + 5.9 * (np.arange(300) + rng.uniform(0.2, 0.4, 300)) / 300
    A1, b1 = arcs_problem(c, c + 0.005)
    ang = rng.uniform(0, 2 * np.pi, 6000)
    A = np.vstack([A1, np.stack([np.cos(ang), np.sin(ang)], axis=1)])
    b = np.concatenate([b1, np.full(6000, 5.0)])
    perm = rng.permutation(len(b))
    A, b = A[perm], b[perm]
    C = 4
    npdt = np.float32 if precision == 32 else np.float64
    x = np.tile(np.array([1.0, 0.0], npdt), (C, 1))
    nu = np.tile(np.array([0.0, 1.0], npdt), (C, 1))
    u = (np.arange(C) + 0.5) / C
    Ab = A.astype(npdt).astype(np.float64)
    ref = ref_ess.transition(Ab, b, x.astype(np.float64), nu.astype(np.float64), u, store=npdt)
    g = assert_same_as_full_sort(E, Ab, b, x, nu, u, precision, 0.0)
    assert (g["n_intervals"] == 301).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x.astype(np.float64), nu, u, g, ref)
    assert not fails, fails[:5]


@pytest.mark.parametrize("C", [2, 10])
def test_section_4_2_at_d_8000(E, C):
    """Section 4.2's instance beyond 4096 rows (d = m = 8000) from x0: crowded
    buckets on the chunked path (refinement on the gathered rows), against
    the oracle and the full sort.  Ten chains take the row-parallel
    projection's two waves of six chains (A, 256 MB, exceeds what the caches
    hold)."""
    pr = synth.paper_highdim(d=8000)
    rng = np.random.default_rng(43)
    x = np.tile(pr.x0, (C, 1)).astype(np.float32)
    nu = rng.standard_normal(x.shape).astype(np.float32)
    u = rng.uniform(size=C)
    Ab = pr.A.astype(np.float32).astype(np.float64)
    ref = ref_ess.transition(Ab, pr.b, x.astype(np.float64), nu.astype(np.float64), u,
                             eps=1e-6, store=np.float32)
    say("coarse survivors", coarse_survivors(ref["alpha"], ref["beta"]))
    g = assert_same_as_full_sort(E, pr.A, pr.b, x, nu, u, 32, 1e-6)
    fails, _ = compare_transition(Ab, pr.b, x.astype(np.float64), nu, u, g, ref)
    assert not fails, fails[:5]


MID_CASES = [
    # method, name, d, m, C, precision, eps
    ("midpoint", "mid_ragged_f32", 37, 150, 40, 32, 1e-6),
    ("midpoint", "mid_f64", 20, 300, 16, 64, 0.0),
    ("midpoint", "mid_m2000_f32", 40, 2000, 8, 32, 1e-6),
    ("midpoint", "mid_max_m_f32", 30, 4096, 3, 32, 1e-6),
    ("alg2", "alg2_ragged_f32", 37, 150, 40, 32, 1e-6),
    ("alg2", "alg2_f64", 20, 300, 16, 64, 0.0),
    ("alg2", "alg2_many_m1000_f32", 40, 1000, 300, 32, 1e-6),
    ("alg2", "alg2_m2000_f32", 40, 2000, 8, 32, 1e-6),
    ("alg2", "alg2_max_m_f64", 30, 4096, 3, 64, 0.0),
]


@pytest.mark.parametrize("method,name,d,m,C,precision,eps", MID_CASES, ids=[c[1] for c in MID_CASES])
def test_quadratic_comparators_match_oracle_and_alg3(E, method, name, d, m, C, precision, eps):
    """The quadratic comparators, Section 2.2's likelihood testing at
    midpoints and Algorithm 2's sequential intersection, find the same
    pieces as Algorithm 3 from the same projections, and agree with the
    oracle's version of the same method."""
    say(f"[{method}] {name} d={d} m={m} C={C} prec={precision}")
    rng = np.random.default_rng(d * 5 + m)
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, m)
    npdt = np.float32 if precision == 32 else np.float64
    x = chain_states(A, b, C, npdt, seed=m)
    nu = rng.standard_normal(x.shape).astype(npdt)
    u = rng.uniform(size=C)
    outs = {}
    for meth in ("alg3", method):
        s = E.Sampler(A, b, x, C, seed=5, precision=precision, trim_eps=eps, method=meth)
        outs[meth] = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
        s.close()
    a, g = outs["alg3"], outs[method]
    assert np.array_equal(a["n_intervals"], g["n_intervals"])
    # float64: the same roots bit for bit.  float32: each kernel inlines its
    # own copy of the float32 atan2 / acos away from tangency, and the compiler
    # may contract them differently, so an angle can differ by a float ulp
    # (up to 2.4e-7 rad below pi)
    tol_same = 1e-13 if precision == 64 else 1e-6
    assert np.abs(a["intervals"] - g["intervals"]).max() <= tol_same
    assert np.abs(a["theta"] - g["theta"]).max() <= 10 * tol_same
    assert np.array_equal(a["rejected"], g["rejected"])
    Ab = A.astype(npdt).astype(np.float64)
    ref = ref_ess.transition(Ab, b, x.astype(np.float64), nu.astype(np.float64), u, eps=eps,
                             store=npdt, pq=(g["pq"][0], g["pq"][1]), method=method)
    # the root solve's rounding bounds the rest, as in the Algorithm 3 parity
    # cases: float64 trig in float64 mode, float32 trig away from tangency
    tol2 = 1e-9 if precision == 64 else 1e-5
    for c in range(C):
        gi = pieces(g["intervals"][c], g["n_intervals"][c], 0.0)
        assert intervals_match(gi, ref["intervals"][c], tol2), (c, gi, ref["intervals"][c])
        assert abs(g["theta"][c] - ref["theta"][c]) <= tol2 * max(1.0, len(gi)), c


@pytest.mark.parametrize("method", ["midpoint", "alg2"])
@pytest.mark.parametrize("precision", [32, 64])
def test_comparators_on_the_sorting_reduction(E, precision, method):
    """Section 3.1's reduction (100 disjoint arcs) through the comparators."""
    rng = np.random.default_rng(23)
    c = 0.1 + 5.9 * (np.arange(100) + rng.uniform(0.2, 0.4, 100)) / 100
    Ab, b, x, nu, u, g, ref = run_arcs(E, c, c + 0.005, precision, method=method)
    assert (g["n_intervals"] == 101).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, fails[:5]


@pytest.mark.parametrize("precision,m", [(32, 7), (64, 14)])
def test_alg2_on_appendix_d_worst_case(E, precision, m):
    """Appendix D's input, I_i = [0, 3^-i] U [2 3^-i, 1] scaled by 2 pi and
    placed at pi / 2: Algorithm 2's list grows by one piece per row and ends
    with all m + 1 intervals, as Algorithm 3 finds them."""
    i = np.arange(1, m + 1)
    al = 2 * np.pi * 3.0 ** -i
    Ab, b, x, nu, u, g, ref = run_arcs(E, 0.5 * np.pi + al, 0.5 * np.pi + 2 * al, precision,
                                       method="alg2")
    assert (g["n_intervals"] == m + 1).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, fails[:5]


@pytest.mark.parametrize("method,m", [("midpoint", 300), ("alg3", 6000)])
def test_per_chain_b_on_the_comparator_and_the_large_path(E, method, m):
    """One right-hand side per chain (ESS_PER_CHAIN_B) through the quadratic
    comparator and through the chunked path beyond 4096 rows."""
    rng = np.random.default_rng(m + 3)
    d, C = 25, 6
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, (C, m))
    x = np.zeros((C, d), np.float32)
    nu = rng.standard_normal(x.shape).astype(np.float32)
    u = rng.uniform(size=C)
    s = E.Sampler(A, b, x, C, seed=4, precision=32, trim_eps=1e-6, method=method)
    g = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
    s.close()
    Ab = A.astype(np.float32).astype(np.float64)
    ref = ref_ess.transition(Ab, b, x.astype(np.float64), nu.astype(np.float64), u, eps=1e-6,
                             store=np.float32, method=method)
    fails, _ = compare_transition(Ab, b, x.astype(np.float64), nu, u, g, ref)
    assert not fails, fails[:5]


def test_two_refinement_levels(E):
    """600 rows whose alphas lie within 6e-7 rad (one bucket, and still one
    sub-bucket after the first split) and whose arcs overlap: two levels of
    refinement leave a single survivor.  Float64 resolves the spacing."""
    n = 600
    al = 1.0 + 1e-9 * np.arange(n)
    Ab, b, x, nu, u, g, ref = run_arcs(E, al, al + 1.0, 64)
    assert coarse_survivors(ref["alpha"], ref["beta"])[0] == n
    assert (g["n_intervals"] == 2).all(), g["n_intervals"]
    fails, _ = compare_transition(Ab, b, x, nu, u, g, ref)
    assert not fails, fails[:5]
    assert_same_as_full_sort(E, Ab, b, x, nu, u, 64, 0.0)


@pytest.mark.parametrize("name,d,m,C,precision,eps", CASES[:4] + LARGE,
                         ids=[c[0] for c in CASES[:4] + LARGE])
def test_full_sort_path_matches_bucket_path(E, name, d, m, C, precision, eps):
    rng = np.random.default_rng(d * 7 + m)
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, m)
    npdt = np.float32 if precision == 32 else np.float64
    x = chain_states(A, b, C, npdt, seed=m)
    nu = rng.standard_normal(x.shape).astype(npdt)
    u = rng.uniform(size=C)
    outs = []
    for full in (False, True):
        s = E.Sampler(A, b, x, C, seed=5, precision=precision, trim_eps=eps, full_sort=full)
        outs.append({k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()})
        s.close()
    a, f = outs
    assert np.array_equal(a["n_intervals"], f["n_intervals"])
    assert np.abs(a["intervals"] - f["intervals"]).max() <= 1e-13
    assert np.abs(a["theta"] - f["theta"]).max() <= 1e-12
    assert np.array_equal(a["rejected"], f["rejected"])
    assert np.abs(a["x_new"] - f["x_new"]).max() <= 1e-6


def test_graph_cache_eviction_keeps_results(E):
    """Eleven runs, each into a new live trace buffer and without counting
    rejections (no synchronisation inside ess_run), so the library captures a
    graph per run and evicts the oldest beyond eight while earlier replays may
    still be queued: every trace equals an eager run's, bit for bit."""
    pr = synth.box_halfspace(n_chains=300)
    g = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=6, precision=32)
    parts = [g.run(2 + (k % 3), count_rejections=False)[0] for k in range(11)]
    torch.cuda.synchronize()
    e = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=6, precision=32, eager=True)
    want, _ = e.run(sum(p.shape[0] for p in parts))
    assert torch.equal(torch.cat(parts), want)
    g.close()
    e.close()


def test_graph_replay_equals_eager_launches(E):
    """Captured-graph runs (default) and kernel-by-kernel runs agree bit for bit,
    across repeated replays of one captured shape and a state reset."""
    pr = synth.box_halfspace(n_chains=700)            # two chain groups
    g = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=4, precision=32)
    e = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=4, precision=32, eager=True)
    trace = torch.empty(3, pr.n_chains, pr.d, device="cuda")
    parts = []
    for _ in range(3):                                 # same shape and trace buffer: replays
        E.ess_run(g.ctx, 6, 2, trace, False)
        parts.append(trace.clone())
    want, _ = e.run(18, thin=2)
    assert torch.equal(torch.cat(parts), want)
    x, step = g.state()
    assert step == 18
    g.set_state(x, 3)                                  # rewind the counter: replay uses it
    E.ess_run(g.ctx, 6, 2, trace, False)
    e2 = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=4, precision=32, eager=True)
    e2.set_state(x, 3)
    want2, _ = e2.run(6, thin=2)
    assert torch.equal(trace, want2)
    for s in (g, e, e2):
        s.close()


@pytest.mark.parametrize("workload,C,precision", [("box_halfspace", 640, 32),
                                                   ("gp_rbf", 1024, 32),
                                                   ("box_halfspace", 256, 64)])
def test_single_context_autotune(E, tmp_path, monkeypatch, workload, C, precision):
    """ess_autotune on a single-problem context times the projection kernels
    (split bfloat16 tiles, float32 tiles of four shapes, band heights) and
    puts the chains back: same state, step and rejection counts.  Afterwards
    the context runs exactly as a new context that loads the cached choice
    from that state, and its steps match the oracle."""
    monkeypatch.setenv("ESS_TUNE_CACHE", str(tmp_path / "tune.json"))
    pr = getattr(synth, workload)(n_chains=C)
    eps = 1e-6 if precision == 32 else 0.0
    a = E.Sampler(pr.A, pr.b, pr.x0, C, seed=8, precision=precision, trim_eps=eps)
    first, _ = a.run(5)
    rej0 = a.rejections()
    report = E.ess_autotune(a.ctx, 2)
    say(report)
    assert "chosen" in report and (tmp_path / "tune.json").exists()
    x, step = a.state()
    assert step == 5 and torch.equal(x, first[-1])
    assert np.array_equal(a.rejections(), rej0)
    rest, _ = a.run(5)
    c = E.Sampler(pr.A, pr.b, pr.x0, C, seed=8, precision=precision, trim_eps=eps)  # loads the cache
    c.set_state(first[-1], 5)
    again, _ = c.run(5)
    assert torch.equal(again, rest)
    c.close()
    idx = np.linspace(0, C - 1, 64).astype(int)
    excused = run_step_by_step(E, a, pr.A, pr.b, 8, 2, idx, eps,
                               store=np.float32 if precision == 32 else np.float64)
    assert excused <= 2
    a.close()


def test_single_context_autotune_with_few_chains_has_nothing_to_tune(E, tmp_path, monkeypatch):
    monkeypatch.setenv("ESS_TUNE_CACHE", str(tmp_path / "tune.json"))
    pr = synth.small_fp64()
    s = E.Sampler(pr.A, pr.b, pr.x0, 8, precision=64)
    assert "nothing to tune" in E.ess_autotune(s.ctx, 2)
    s.close()


def test_split_projections_are_as_accurate_as_float32_matrix_cores(E, monkeypatch):
    """The projections through exact three-piece bfloat16 splits (the default
    where 128 x 128 tiles fill the device) against float64 A x and A nu, next
    to the float32 matrix-core projections of the same inputs: per entry, the
    error relative to sum_j |a_ij y_j| stays within the float32 accumulation
    bound d 2^-24 and within twice the float32 kernel's own largest error
    (measured: 1.1e-6 against 1.9e-6 for the float32 kernel)."""
    pr = synth.gp_rbf()
    C = pr.n_chains
    x = chain_states(pr.A, pr.b, C, np.float32, seed=3)
    rng = np.random.default_rng(4)
    nu = rng.standard_normal(x.shape).astype(np.float32)
    u = rng.uniform(size=C)
    A32 = pr.A.astype(np.float32).astype(np.float64)
    rows = rng.choice(pr.m, 300, replace=False)
    chains = rng.choice(C, 64, replace=False)
    errs = {}
    for mode in ("split", "f32"):
        if mode == "f32":
            monkeypatch.setenv("ESS_PROJ", "f32")
        else:
            monkeypatch.delenv("ESS_PROJ", raising=False)
        s = E.Sampler(pr.A, pr.b, x, C, seed=0, precision=32, trim_eps=1e-6)
        pq = s.transition_explicit(x, nu, u)["pq"].cpu().numpy().astype(np.float64)
        s.close()
        e = []
        for k, y in enumerate((x, nu)):
            Y = y[chains].astype(np.float64)
            ref = Y @ A32[rows].T
            mag = np.abs(Y) @ np.abs(A32[rows]).T
            e.append(np.abs(pq[k][chains][:, rows] - ref) / mag)
        errs[mode] = max(v.max() for v in e)
    say("projection error / sum |a y|:", errs)
    assert errs["split"] <= pr.d * 2.0 ** -24
    assert errs["split"] <= 2 * errs["f32"]


def test_split_64_tiles_are_as_accurate_as_float32_matrix_cores(E, monkeypatch):
    """The same comparison on the split bfloat16 64 x 64 tiles (the default
    for d > 192 where 128 x 128 tiles do not fill the device) against the
    float32 matrix-core 64 x 64 tiles, at d = 300, m = 900, 512 chains."""
    rng = np.random.default_rng(8)
    d, m, C = 300, 900, 512
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, m)
    x = chain_states(A, b, C, np.float32, seed=5)
    nu = rng.standard_normal(x.shape).astype(np.float32)
    u = rng.uniform(size=C)
    A32 = A.astype(np.float32).astype(np.float64)
    rows = rng.choice(m, 300, replace=False)
    chains = rng.choice(C, 64, replace=False)
    errs = {}
    for mode in ("split", "f32"):
        if mode == "f32":
            monkeypatch.setenv("ESS_PROJ", "f32")
        else:
            monkeypatch.delenv("ESS_PROJ", raising=False)
        s = E.Sampler(A, b, x, C, seed=0, precision=32, trim_eps=1e-6)
        pq = s.transition_explicit(x, nu, u)["pq"].cpu().numpy().astype(np.float64)
        s.close()
        e = []
        for k, y in enumerate((x, nu)):
            Y = y[chains].astype(np.float64)
            ref = Y @ A32[rows].T
            mag = np.abs(Y) @ np.abs(A32[rows]).T
            e.append(np.abs(pq[k][chains][:, rows] - ref) / mag)
        errs[mode] = max(v.max() for v in e)
    say("64 x 64 tiles, projection error / sum |a y|:", errs)
    assert errs["split"] <= d * 2.0 ** -24
    assert errs["split"] <= 2 * errs["f32"]
