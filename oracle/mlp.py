"""Float64 reference for the warm-start network (test infrastructure only).

A fully connected network x_hat = W_L g(... g(W_1 b + c_1) ...) + c_L with
the exact GELU g(z) = z Phi(z) (Hendrycks & Gimpel, 2016), the mean squared
error over all outputs, its gradients written out layer by layer, and one Adam
step (Kingma & Ba, 2015: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
w <- w - lr m_hat / (sqrt(v_hat) + eps) with the bias corrections
m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t)).

`rnd` (default: none) is applied wherever the code under test feeds a value
to a matrix product in reduced precision, so the same operand rounding can be
reproduced; `bf16` rounds float32 values to bfloat16 (nearest, ties to even).
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32).copy()
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + np.uint64(0x7FFF) + ((bits >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def ident(x):
    return np.asarray(x, dtype=np.float64)


def gelu(z):
    return z * 0.5 * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def forward(params, inp, rnd=ident):
    """params: list of (W (out, in), c (out,)).  Returns (output, cache)."""
    h = rnd(inp)
    cache = [h]
    L = len(params)
    for li, (W, c) in enumerate(params):
        z = h @ rnd(W).T + c
        if li < L - 1:
            cache.append(z)
            h = rnd(gelu(z))
            cache.append(h)
        else:
            return z, cache
    raise ValueError("empty network")


def mse(out, target):
    return float(np.mean((out - target) ** 2))


def backward(params, cache, out, target, rnd=ident):
    """Gradients of the mean squared error: list of (dW, dc), and d input."""
    n = out.size
    dz = 2.0 * (out - target) / n
    grads = [None] * len(params)
    L = len(params)
    for li in range(L - 1, -1, -1):
        W, _ = params[li]
        h_in = cache[2 * li]
        dzr = rnd(dz)
        grads[li] = (dzr.T @ h_in, dz.sum(axis=0))
        dh = dzr @ rnd(W)
        if li > 0:
            z_prev = cache[2 * li - 1]
            dz = dh * gelu_grad(z_prev)
        else:
            d_in = dh
    return grads, d_in


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step count t >= 1; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
