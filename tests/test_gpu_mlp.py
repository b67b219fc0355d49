"""Warm-start network kernels vs the float64 reference (identical bfloat16
operands) and the gated start."""
import math

import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_10449_amd as E
    E.lib()
    return E


def _net(E, widths, seed=0):
    net = E.Mlp(widths, seed=seed)
    flat = net.params().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    flat[:] += 0.05 * rng.standard_normal(flat.size)        # non-zero biases too
    net.set_params(flat.astype(np.float32))
    return net, net.unflatten(flat.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("widths,B", [((24, 40, 33, 10), 37), ((768, 512, 512, 256), 256)])
def test_forward_and_gradients_match_reference(E, widths, B):
    net, params = _net(E, widths)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((B, widths[0])).astype(np.float32)
    y = rng.standard_normal((B, widths[-1])).astype(np.float32)
    out = net.forward(x).cpu().numpy()
    g, loss = net.gradients(x, y)
    g = g.cpu().numpy()
    r_out, cache = ref.forward(params, x.astype(np.float64), rnd=ref.bf16)
    r_grads, _ = ref.backward(params, cache, r_out, y.astype(np.float64), rnd=ref.bf16)
    scale = np.abs(r_out).max()
    assert np.abs(out - r_out).max() <= 1e-2 * scale
    assert abs(loss - ref.mse(r_out, y)) <= 1e-2 * ref.mse(r_out, y)
    # every gradient element: within 1e-2 of its layer's largest gradient
    # (weights and biases separately); bfloat16 operands are identical on
    # both sides, so only float32 against float64 accumulation and the
    # rounding of recomputed activations to bfloat16 differ
    for (W, c), (gW, gc), off in zip(params, r_grads, np.cumsum([0] + [W.size + c.size for W, c in params])[:-1]):
        gw = g[off:off + W.size]
        assert np.abs(gw - gW.ravel()).max() <= 1e-2 * np.abs(gW).max(), off
        gb = g[off + W.size: off + W.size + c.size]
        assert np.abs(gb - gc).max() <= 1e-2 * np.abs(gc).max() + 1e-7, off
    net.close()


def test_adam_step_matches_reference(E):
    widths = (16, 32, 8)
    net, params = _net(E, widths, seed=3)
    flat0 = net.params().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((20, 16)).astype(np.float32)
    y = rng.standard_normal((20, 8)).astype(np.float32)
    g, _ = net.gradients(x, y)
    g = g.cpu().numpy().astype(np.float64)
    import paper_2407_10449_amd as P
    P.ess_mlp_adam(net.net, 1e-2)
    flat1 = net.params().cpu().numpy().astype(np.float64)
    want, _, _ = ref.adam_step(flat0, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-2)
    assert np.abs(flat1 - want).max() <= 1e-6
    net.close()


def test_training_on_gpu_reduces_the_loss(E):
    widths = (8, 64, 64, 4)
    net = E.Mlp(widths, seed=1)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1024, 8)).astype(np.float32)
    Y = np.stack([X[:, 0] * X[:, 1], np.sin(X[:, 2]), X[:, 3] ** 2, X[:, 4]], 1).astype(np.float32)
    Xd, Yd = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    _, first = net.gradients(Xd, Yd)
    for _ in range(300):
        net.train_step(Xd, Yd, 3e-3)
    _, last = net.gradients(Xd, Yd)
    assert last < 0.2 * first, (first, last)
    net.close()


def test_gated_start_takes_feasible_candidates_only(E):
    rng = np.random.default_rng(0)
    d, m, C = 12, 30, 64
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, m)
    cand = (rng.standard_normal((C, d)) * np.where(np.arange(C) % 2 == 0, 0.1, 5.0)[:, None]).astype(np.float32)
    fallback = np.zeros((C, d), np.float32)
    s = E.Sampler(A, b, np.zeros(d), C, precision=32)
    acc = s.set_state_gated(cand, fallback)
    x, step = s.state()
    x = x.cpu().numpy()
    feasible = (cand.astype(np.float64) @ A.astype(np.float32).astype(np.float64).T < b - 1e-5).all(axis=1)
    infeasible = (cand.astype(np.float64) @ A.T > b + 1e-5).any(axis=1)
    assert acc[feasible].all() and not acc[infeasible].any()
    assert np.array_equal(x[acc == 1], cand[acc == 1]) and (x[acc == 0] == 0).all()
    s.run(5)
    s.close()
