"""Learned warm start for a family of polytopes {x : A x <= b} sharing A.

1. Training data: the plain sampler (ESS_PER_CHAIN_B, one right-hand side
   per chain) runs chains for many b's; after a burn-in, thinned states give
   (b, x) pairs.
2. The network (768 -> 512 -> 512 -> 256 for the 256-dimensional family,
   GELU, bfloat16 matrix cores, float32 masters) is trained on those pairs
   with the mean squared error and Adam, so it predicts roughly E[x | b].
3. For new b's, every chain starts at the prediction when it is strictly
   feasible (A x_hat < b), and at the plain start otherwise
   (ess_set_state_gated).

The sampler's stationary law does not depend on the start; the burn-in and
effective-sample-size diagnostics of the plain chain judge the effect.
This module only sequences library calls; the computation runs in libess.
"""
import time

import numpy as np


def _per_chain_b(bs, chains_per_b):
    return np.repeat(np.asarray(bs, dtype=np.float64), chains_per_b, axis=0)


def generate_pairs(E, A, bs, chains_per_b=10, burn=200, n_keep=10, thin=10, seed=0):
    """Plain-sampler (b, x) pairs: len(bs) * chains_per_b * n_keep of them.

    Returns (inputs (N, m) float32, targets (N, d) float32) as device tensors
    and the generation time in seconds."""
    import torch
    m, d = A.shape
    B = _per_chain_b(bs, chains_per_b)
    C = B.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = E.Sampler(A, B, np.zeros(d), C, seed=seed, precision=32)
    s.run(burn, keep_trace=False, count_rejections=False)
    tr, _ = s.run(n_keep * thin, thin=thin, count_rejections=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    x = tr.reshape(-1, d)                                   # (n_keep * C, d), sample-major
    b = torch.as_tensor(B, dtype=torch.float32, device="cuda").repeat(n_keep, 1)
    return b.contiguous(), x.contiguous(), dt


def train(net, inputs, targets, epochs=20, batch=1024, lr=1e-3, seed=0, log=None):
    """Adam on contiguous minibatches of a once-permuted copy of the data.
    Returns the mean squared error on a probe set before training and after
    every epoch, and the training time.  Each target is one posterior draw, so
    the error cannot fall below the mean posterior variance."""
    import torch
    n = inputs.shape[0]
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(n), device=inputs.device)
    X, Y = inputs[perm].contiguous(), targets[perm].contiguous()
    nb = n // batch
    probe = slice(0, batch * min(nb, 8))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    history = [net.gradients(X[probe], Y[probe])[1]]   # before training
    for ep in range(epochs):
        for i in range(nb):
            sl = slice(i * batch, (i + 1) * batch)
            net.train_step(X[sl], Y[sl], lr)
        _, loss = net.gradients(X[probe], Y[probe])
        history.append(loss)
        if log:
            log(f"epoch {ep}: mse {loss:.5f}")
    torch.cuda.synchronize()
    return history, time.perf_counter() - t0


def reference_moments(E, A, bs, chains=64, burn=500, steps=2000, thin=4, seed=1):
    """Long plain runs: per b, the mean and sd of every coordinate."""
    m, d = A.shape
    B = _per_chain_b(bs, chains)
    s = E.Sampler(A, B, np.zeros(d), B.shape[0], seed=seed, precision=32)
    s.run(burn, keep_trace=False, count_rejections=False)
    tr, _ = s.run(steps, thin=thin, count_rejections=False)
    s.close()
    x = tr.double().cpu().numpy().reshape(tr.shape[0], len(bs), chains, d)
    flat = x.transpose(1, 0, 2, 3).reshape(len(bs), -1, d)
    return flat.mean(axis=1), flat.std(axis=1)


def burn_in_curve(trace, bs_count, chains, ref_mean, ref_sd):
    """D_t = mean over problems and coordinates of z^2, with
    z = (mean over a problem's chains at step t - reference mean) / (sd / sqrt(chains)).
    At stationarity D_t is about 1."""
    T, C, d = trace.shape
    x = trace.reshape(T, bs_count, chains, d).mean(axis=2)
    z = (x - ref_mean[None]) / (ref_sd[None] / np.sqrt(chains))
    return (z ** 2).mean(axis=(1, 2))


def burn_in_steps(curve, level=2.0):
    """First step from which the curve stays at or below `level`."""
    above = np.nonzero(curve > level)[0]
    return 0 if above.size == 0 else int(above[-1] + 1)
