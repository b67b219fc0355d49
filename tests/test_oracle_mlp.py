"""The float64 warm-start network reference against finite differences and
closed forms (no GPU)."""
import math

import numpy as np
import pytest

from oracle import mlp


def small_net(rng, widths=(7, 5, 6, 3)):
    return [(rng.standard_normal((o, i)) / math.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(widths[:-1], widths[1:])]


def test_gelu_known_values():
    # GELU(z) = z Phi(z): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert abs(mlp.gelu(np.array(40.0)) - 40.0) < 1e-12
    assert abs(mlp.gelu_grad(np.array(0.0)) - 0.5) < 1e-15


def test_gelu_grad_matches_central_differences():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-8


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    params = small_net(rng)
    x = rng.standard_normal((4, 7))
    y = rng.standard_normal((4, 3))
    out, cache = mlp.forward(params, x)
    grads, d_in = mlp.backward(params, cache, out, y)

    def loss(ps, inp):
        return mlp.mse(mlp.forward(ps, inp)[0], y)

    h = 1e-6
    for li, (W, c) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (c, grads[li][1])):
            for idx in list(np.ndindex(arr.shape))[:12]:
                old = arr[idx]
                arr[idx] = old + h
                lp = loss(params, x)
                arr[idx] = old - h
                lm = loss(params, x)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - g[idx]) < 1e-7 * max(1, abs(g[idx])), (li, idx)
    for idx in list(np.ndindex(x.shape))[:10]:
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        assert abs((loss(params, xp) - loss(params, xm)) / (2 * h) - d_in[idx]) < 1e-7


def test_adam_closed_forms():
    # beta1 = beta2 = 0: the step is lr * g / (|g| + eps)
    w, g = np.array([1.0, -2.0, 0.5]), np.array([0.3, -4.0, 1e-3])
    w1, _, _ = mlp.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.1, b1=0.0, b2=0.0, eps=0.0)
    assert np.allclose(w1, w - 0.1 * np.sign(g), atol=1e-15)
    # a constant gradient: bias correction makes every step lr * g / (|g| + eps)
    m = v = np.zeros(3)
    ww = w.copy()
    for t in range(1, 6):
        ww, m, v = mlp.adam_step(ww, g, m, v, t, lr=0.01, eps=0.0)
    assert np.allclose(ww, w - 5 * 0.01 * np.sign(g), atol=1e-12)


def test_bf16_rounding():
    # 1 + 2^-8 is halfway between bfloat16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    x = np.random.default_rng(1).standard_normal(1000).astype(np.float32)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-38)


def test_training_reduces_the_loss():
    rng = np.random.default_rng(2)
    params = small_net(rng, (4, 16, 16, 2))
    X = rng.standard_normal((256, 4))
    Y = np.stack([X[:, 0] * X[:, 1], np.sin(X[:, 2])], axis=1)
    state = [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(c), np.zeros_like(c)) for W, c in params]
    first = None
    for t in range(1, 301):
        out, cache = mlp.forward(params, X)
        loss = mlp.mse(out, Y)
        first = first if first is not None else loss
        grads, _ = mlp.backward(params, cache, out, Y)
        new = []
        for (W, c), (gW, gc), (mW, vW, mc, vc) in zip(params, grads, state):
            W, mW, vW = mlp.adam_step(W, gW, mW, vW, t, 1e-2)
            c, mc, vc = mlp.adam_step(c, gc, mc, vc, t, 1e-2)
            new.append(((W, c), (mW, vW, mc, vc)))
        params = [p for p, _ in new]
        state = [s for _, s in new]
    assert loss < 0.3 * first
