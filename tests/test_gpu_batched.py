"""Batched contexts: many uneven polytopes advanced by one launch per step."""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import ess as ref_ess
from oracle import philox as ref_philox
from parity import compare_states

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


def problems(n, chains, seed=4):
    probs = synth.batched_uneven(rng_seed=seed, n_problems=n, chains_per_problem=chains)
    return [dict(A=p.A, b=p.b, x0=p.x0, n_chains=p.n_chains, seed=100 + i, trim_eps=1e-6)
            for i, p in enumerate(probs)]


def test_batched_matches_oracle_per_step(E):
    """Every chain of every problem, one step at a time: from the state the
    batch reached, the oracle's transition with the step's Philox draws
    (problem word p) gives the decision and the new state to 1e-5.  Four
    steps, so the states are generic mid-chain states after the first."""
    per_step_against_oracle(E, problems(10, 16))


def test_batched_with_a_problem_above_2048_rows_per_step(E):
    """A problem of 3000 rows beside small ones (the chain kernels' widest
    variant, with every smaller chain in one class of its own), per step
    against the oracle as above."""
    rng = np.random.default_rng(41)
    probs = problems(5, 16, seed=41)
    d, m = 48, 3000
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    probs.insert(2, dict(A=A, b=rng.uniform(0.5, 1.5, m), x0=np.zeros(d), n_chains=16,
                         seed=777, trim_eps=1e-6))
    per_step_against_oracle(E, probs)


def test_batched_with_a_wide_problem_per_step(E):
    """A problem of 700 columns beside small ones: each of its chains' threads
    draws more than one of the next direction's element pairs (the first ahead
    of the move, the rest in the move's loop), and its projections take the
    split 64 x 64 tiles; per step against the oracle as above."""
    rng = np.random.default_rng(43)
    probs = problems(4, 16, seed=43)
    d, m = 700, 900
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    probs.insert(1, dict(A=A, b=rng.uniform(0.5, 1.5, m), x0=np.zeros(d), n_chains=16,
                         seed=778, trim_eps=1e-6))
    per_step_against_oracle(E, probs)


def per_step_against_oracle(E, probs):
    say("[batched] shapes", [(p["A"].shape, p["n_chains"]) for p in probs])
    s = E.BatchedSampler(probs)
    x_prev = [x.astype(np.float64) for x in s.split(s.state()[0].cpu().numpy())]
    rej_prev = s.rejections()
    starts = np.cumsum([0] + [p["n_chains"] for p in probs])
    excused = 0
    for t in range(4):
        _, step = s.state()
        s.run(1, keep_trace=False)
        x_next = [x.astype(np.float64) for x in s.split(s.state()[0].cpu().numpy())]
        rej = s.rejections()
        for p, pr in enumerate(probs):
            C, d = pr["n_chains"], pr["A"].shape[1]
            A32 = pr["A"].astype(np.float32).astype(np.float64)
            ch = np.arange(C)
            nu = ref_philox.normals(pr["seed"], step, ch, d, problem=p).astype(np.float32)
            u = ref_philox.uniforms(pr["seed"], step, ch, problem=p)
            ref = ref_ess.transition(A32, pr["b"], x_prev[p], nu.astype(np.float64), u,
                                     eps=pr["trim_eps"], store=np.float32)
            rj = (rej - rej_prev)[starts[p]:starts[p + 1]]
            fails, exc = compare_states(A32, pr["b"], x_next[p], rj, ref)
            assert not fails, (t, p, fails[:5])
            excused += exc
        x_prev, rej_prev = x_next, rej
    assert excused <= 2


def test_batched_checkpoint_and_determinism(E):
    probs = problems(6, 8, seed=7)
    a = E.BatchedSampler(probs)
    full, _ = a.run(8, thin=2)
    b = E.BatchedSampler(probs)
    half, _ = b.run(4, thin=2)
    x, step = b.state()
    c = E.BatchedSampler(probs)
    c.set_state(x, step)
    rest, _ = c.run(4, thin=2)
    assert torch.equal(full[:2], half) and torch.equal(full[2:], rest)
    d = E.BatchedSampler(probs)
    again, _ = d.run(8, thin=2)
    assert torch.equal(full, again)
    for s in (a, b, c, d):
        s.close()


def test_batched_full_workload_stays_feasible(E):
    """256 polytopes, d log-uniform in [16, 512], m = d U{1..4}, 64 chains each."""
    probs = problems(256, 64)
    s = E.BatchedSampler(probs)
    tr, nrej = s.run(20, thin=5)
    per = s.split(tr.double().cpu().numpy())
    s.close()
    for pr, g in zip(probs, per):
        slack = pr["b"] - g @ pr["A"].T
        bound = 2 * pr["A"].shape[1] * 2.0 ** -24 * (np.abs(g) @ np.abs(pr["A"]).T)
        assert (slack >= -bound).all()
    assert nrej <= 1e-4 * 256 * 64 * 20


def test_batched_graph_replay_equals_eager(E, monkeypatch):
    probs = problems(5, 8, seed=9)
    g = E.BatchedSampler(probs)
    tr1, _ = g.run(4)
    tr2, _ = g.run(4)
    g.close()
    monkeypatch.setenv("ESS_EAGER", "1")
    e = E.BatchedSampler(probs)
    want, _ = e.run(8)
    e.close()
    assert torch.equal(torch.cat([tr1, tr2]), want)


def test_batched_autotune_keeps_results(E, tmp_path, monkeypatch):
    monkeypatch.setenv("ESS_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs = problems(6, 16, seed=12)
    a = E.BatchedSampler(probs)
    first, _ = a.run(3)
    report = E.ess_autotune(a.ctx, 2)
    assert "chosen" in report
    rest, _ = a.run(3)
    b = E.BatchedSampler(probs)
    want, _ = b.run(6)
    assert torch.equal(torch.cat([first, rest]), want)
    a.close()
    b.close()


@pytest.mark.parametrize("launch,tile", [("split", "32x64"), ("split", "64x32"),
                                         ("split", "32x32"), ("fused", "64x64"),
                                         ("fused", "32x32")])
def test_batched_launch_forms_and_tiles_give_identical_chains(E, monkeypatch, launch, tile):
    """Every tile shape sums each projection in the same order, and the fused
    and split launches run the same arithmetic, so the chains are
    bit-identical to the default (split launch, 64x64 tiles)."""
    probs = problems(12, 16, seed=21)
    monkeypatch.setenv("ESS_BATCH_TILE", "64x64")
    monkeypatch.setenv("ESS_BATCH_LAUNCH", "split")
    a = E.BatchedSampler(probs)
    want, _ = a.run(5)
    a.close()
    monkeypatch.setenv("ESS_BATCH_TILE", tile)
    monkeypatch.setenv("ESS_BATCH_LAUNCH", launch)
    b = E.BatchedSampler(probs)
    got, _ = b.run(5)
    b.close()
    assert torch.equal(got, want)


def test_batched_problem_zero_equals_its_own_context(E):
    """The first problem of a batch draws with problem word 0, as a
    single-problem context does, and every projection sums in the same order
    whatever the tile: its chains are bit-identical to the same problem run
    alone."""
    probs = problems(7, 16, seed=31)
    a = E.BatchedSampler(probs)
    tr, _ = a.run(6)
    first = a.split(tr)[0]
    a.close()
    p = probs[0]
    s = E.Sampler(p["A"], p["b"], p["x0"], p["n_chains"], seed=p["seed"], precision=32,
                  trim_eps=p["trim_eps"])
    alone, _ = s.run(6)
    s.close()
    assert torch.equal(first, alone)


def test_batched_problem_sets_give_identical_chains(E, monkeypatch):
    """Problem sets advanced on streams of their own change only which
    launches may overlap: one, two and four sets give bit-identical chains."""
    probs = problems(12, 16, seed=21)
    outs = []
    for n in ("1", "2", "4"):
        monkeypatch.setenv("ESS_BATCH_SETS", n)
        s = E.BatchedSampler(probs)
        tr, _ = s.run(5)
        s.close()
        outs.append(tr)
    assert torch.equal(outs[0], outs[1])
    assert torch.equal(outs[0], outs[2])


def test_batched_infeasible_set_state_keeps_the_state(E):
    """A state that fails the strict start check raises, and the batch keeps
    its previous state, step and projections: it then runs exactly as a twin
    batch that never saw the bad state."""
    probs = problems(6, 16, seed=51)
    a = E.BatchedSampler(probs)
    b = E.BatchedSampler(probs)
    a.run(3)
    b.run(3)
    x, step = a.state()
    bad = x.clone()
    bad[0] = 1.0e6   # far outside every polytope's rows that weigh coordinate 0
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
