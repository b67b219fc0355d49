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


def reference_moments(E, A, bs, chains=64, burn=500, steps=2000, thin=4, seed=1, segment=2000):
    """Long plain runs: per b, the mean and sd of every coordinate over all
    chains and recorded steps (float64 sums on the device, `segment` steps at
    a time, so the trace never has to be held whole)."""
    import torch
    m, d = A.shape
    nb = len(bs)
    B = _per_chain_b(bs, chains)
    s = E.Sampler(A, B, np.zeros(d), B.shape[0], seed=seed, precision=32)
    s.run(burn, keep_trace=False, count_rejections=False)
    s1 = torch.zeros(nb, d, dtype=torch.float64, device="cuda")
    s2 = torch.zeros_like(s1)
    n = 0
    left = steps
    while left > 0:
        k = min(segment, left)
        k -= k % thin
        if k == 0:
            break
        tr, _ = s.run(k, thin=thin, count_rejections=False)
        x = tr.double().reshape(tr.shape[0], nb, chains, d)
        s1 += x.sum(dim=(0, 2))
        s2 += (x * x).sum(dim=(0, 2))
        n += tr.shape[0] * chains
        left -= k
    s.close()
    mean = s1 / n
    var = (s2 / n - mean * mean).clamp_min(0.0)
    return mean.cpu().numpy(), var.sqrt().cpu().numpy()


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


def burn_in_excess(curve):
    """Threshold-free initialisation bias: sum over steps of max(D_t - 1, 0)."""
    return float(np.maximum(np.asarray(curve) - 1.0, 0.0).sum())


def _device_curve(tr, x0, nb, chains, ref_mean, ref_sd):
    """burn_in_curve for a device trace (T, C, d) and start x0 (C, d), computed
    on the device; returns a host float64 array of length T + 1."""
    import torch
    mu = torch.as_tensor(ref_mean, device=tr.device)
    se = torch.as_tensor(ref_sd, device=tr.device) / np.sqrt(chains)
    out = []
    for x in [x0[None]] + [tr[i:i + 256] for i in range(0, tr.shape[0], 256)]:
        m = x.double().reshape(x.shape[0], nb, chains, -1).mean(dim=2)
        out.append((((m - mu) / se) ** 2).mean(dim=(1, 2)))
    return torch.cat(out).cpu().numpy()


def compare(E, A, eval_b, net, chains=64, steps=12000, thin=4, level=2.0, ref=None, seed=0,
            log=None):
    """ESS/s at equal accuracy for three ways to sample the posteriors of `eval_b`:
      plain_per_problem  one context per b (`chains` chains each), started at 0
      batched_plain      one context over all b's (a b per chain), started at 0
      batched_warm       the same context started at the gated network prediction
    Every arm runs `steps` steps recorded every `thin` steps.  Its burn-in is
    the first recorded step from which the curve D_t (`burn_in_curve`, against
    long reference runs) stays at or below `level`; the draws after it give the
    ESS (bulk ESS, minimum over 64 monitored coordinates and |x|^2, summed over
    problems).  Wall time covers inference, gating and every step of the arm.
    Accuracy: the largest |posterior mean - reference| / MCSE over problems and
    the first 16 monitored coordinates."""
    import torch
    from . import diagnostics as D
    m, d = A.shape
    nb = len(eval_b)
    if ref is None:
        ref = reference_moments(E, A, eval_b, chains=chains, burn=3 * steps, steps=5 * steps,
                                thin=10, seed=seed + 1)
    ref_mean, ref_sd = ref
    mon = np.sort(np.random.default_rng(seed).choice(d, min(d, 64), replace=False))
    mon_t = torch.as_tensor(mon, device="cuda")
    B = np.repeat(eval_b, chains, axis=0)
    marks = [k for k in (0, 100, 250, 500, 1000, 2000, 4000, 8000, 16000) if k <= steps]
    out = {"reference": f"{chains} chains per b, {3 * steps} burn-in + {5 * steps} steps",
           "burn_in_level": level}

    def finish(name, tr, x0, wall):
        curve = _device_curve(tr, x0, nb, chains, ref_mean, ref_sd)
        tb = burn_in_steps(curve, level)           # in recorded steps
        sub = tr.index_select(2, mon_t).double()
        sq = (tr.double() ** 2).sum(dim=2, keepdim=True)
        x = torch.cat([sub, sq], dim=2)[max(tb - 1, 0):].cpu().numpy()
        ess, worst, zmax = 0.0, 1e30, 0.0
        if x.shape[0] >= 8:
            for j in range(nb):
                xj = x[:, j * chains:(j + 1) * chains, :]
                e = min(D.ess(xj[:, :, k]) for k in range(xj.shape[2]))
                ess += e
                worst = min(worst, e)
                for k in range(16):
                    se = D.mcse_mean(xj[:, :, k])
                    zmax = max(zmax, abs(xj[:, :, k].mean() - ref_mean[j, mon[k]]) / max(se, 1e-12))
        else:
            worst = 0.0
        out[name] = {"burn_in_steps": tb * thin, "burn_in_excess": burn_in_excess(curve) * thin,
                     "D_at_step": {str(k): round(float(curve[k // thin]), 3) for k in marks},
                     "ess": ess, "min_ess_per_problem": worst, "wall_s": wall,
                     "ess_per_s": ess / wall, "max_z_mean_vs_reference": float(zmax)}
        if log:
            log(f"{name}: {out[name]}")

    ctxs = [E.Sampler(A, b, np.zeros(d), chains, seed=seed + 100 + j, precision=32)
            for j, b in enumerate(eval_b)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trs = [q.run(steps, thin=thin, count_rejections=False)[0] for q in ctxs]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for q in ctxs:
        q.close()
    tr = torch.cat(trs, 1)
    del trs
    finish("plain_per_problem", tr, torch.zeros(B.shape[0], d, device="cuda"), wall)
    del tr

    for name in ("batched_plain", "batched_warm"):
        s = E.Sampler(A, B, np.zeros(d), B.shape[0], seed=seed + 7, precision=32)
        bdev = torch.tensor(eval_b, dtype=torch.float32, device="cuda")
        zeros = torch.zeros(B.shape[0], d, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x0 = zeros
        if name == "batched_warm":
            xhat = net.forward(bdev).repeat_interleave(chains, dim=0)
            acc = s.set_state_gated(xhat, zeros)
        tr, _ = s.run(steps, thin=thin, count_rejections=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if name == "batched_warm":
            x0 = xhat * torch.as_tensor(acc, device="cuda", dtype=xhat.dtype)[:, None]
            out["gate_accepted"] = float(np.mean(acc))
        s.close()
        finish(name, tr, x0, wall)
        del tr
    out["ess_per_s_batched_warm_over_plain_per_problem"] = (
        out["batched_warm"]["ess_per_s"] / max(out["plain_per_problem"]["ess_per_s"], 1e-30))
    out["ess_per_s_batched_warm_over_batched_plain"] = (
        out["batched_warm"]["ess_per_s"] / max(out["batched_plain"]["ess_per_s"], 1e-30))
    return out
