"""The learned warm start end to end: data from the plain sampler, training on
the GPU kernels, the feasibility gate, and its effect on burn-in."""
import sys

import numpy as np
import pytest

import synth

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


def test_warm_start_cuts_burn_in_without_changing_the_law(E):
    from paper_2407_10449_amd import warmstart as W
    A, b0, draw = synth.warm_family()
    m, d = A.shape
    rng = np.random.default_rng(11)
    train_b = draw(rng, 10000)
    eval_b = draw(rng, 32)
    X, Y, t_gen = W.generate_pairs(E, A, train_b, chains_per_b=1, burn=200, n_keep=10, thin=10)
    say(f"[warm] {X.shape[0]} pairs in {t_gen:.2f} s")
    net = E.Mlp((m, 512, 512, d), seed=0)
    hist, t_train = W.train(net, X, Y, epochs=15, batch=1024, lr=1e-3)
    say(f"[warm] mse by epoch {[round(h, 4) for h in hist]} ({t_train:.1f} s)")
    assert hist[-1] < 0.9 * hist[0]      # hist[0] is the untrained network

    ref_mean, ref_sd = W.reference_moments(E, A, eval_b, chains=64, burn=300, steps=1200, thin=4)
    xhat = net.forward(torch.tensor(eval_b, dtype=torch.float32, device="cuda")).cpu().numpy()
    err_net = ((xhat - ref_mean) ** 2).mean()
    err_zero = (ref_mean ** 2).mean()
    say(f"[warm] mean-squared distance to E[x|b]: network {err_net:.5f}, zero start {err_zero:.5f}")
    # E[x | b] lies close to 0 for this family (the gain is small by nature);
    # the network must still be closer to it than the plain start
    assert err_net < 0.9 * err_zero

    chains, T = 64, 60
    B = np.repeat(eval_b, chains, axis=0)
    curves, accepted = {}, None
    for kind in ("plain", "warm"):
        s = E.Sampler(A, B, np.zeros(d), B.shape[0], seed=5, precision=32)
        if kind == "warm":
            cand = np.repeat(xhat, chains, axis=0)
            accepted = s.set_state_gated(cand, np.zeros_like(cand))
        tr, _ = s.run(T)
        s.close()
        x = np.concatenate([np.zeros((1,) + tr.shape[1:]) if kind == "plain" else
                            np.repeat(xhat, chains, axis=0)[None] * accepted[None, :, None],
                            tr.double().cpu().numpy()])
        curves[kind] = W.burn_in_curve(x, len(eval_b), chains, ref_mean, ref_sd)
    tb = {k: W.burn_in_steps(v) for k, v in curves.items()}
    say(f"[warm] gate accepted {accepted.mean():.3f}; burn-in steps plain {tb['plain']} warm {tb['warm']}")
    say(f"[warm] D_0 plain {curves['plain'][0]:.1f} warm {curves['warm'][0]:.1f}; "
        f"D_5 plain {curves['plain'][5]:.2f} warm {curves['warm'][5]:.2f}")
    assert accepted.mean() > 0.9
    assert curves["warm"][0] < curves["plain"][0]
    assert tb["warm"] <= tb["plain"]
    # after burn-in both starts sample the same law
    assert curves["warm"][-10:].mean() < 2.5 and curves["plain"][-10:].mean() < 2.5
    net.close()
