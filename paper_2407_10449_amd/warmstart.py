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


def reference_moments(E, A, bs, chains=64, burn=500, steps=2000, thin=4, seed=1, segment=2000,
                      log=None):
    """Long plain runs: per b, the mean and sd of every coordinate over all
    chains and recorded steps.  Runs `segment` steps at a time into one reused
    buffer (one captured graph), with float64 sums kept on the device."""
    import torch
    m, d = A.shape
    nb = len(bs)
    B = _per_chain_b(bs, chains)
    s = E.Sampler(A, B, np.zeros(d), B.shape[0], seed=seed, precision=32)
    segment = min(segment, steps, burn if burn > 0 else segment)
    segment = max(thin, segment - segment % thin)
    buf = torch.empty(segment // thin, B.shape[0], d, device="cuda")
    for _ in range(burn // segment):
        s.run(segment, thin=thin, count_rejections=False, out=buf)
    s1 = torch.zeros(nb, d, dtype=torch.float64, device="cuda")
    s2 = torch.zeros_like(s1)
    n = 0
    for k in range(max(1, steps // segment)):
        s.run(segment, thin=thin, count_rejections=False, out=buf)
        if log and k % 50 == 49:
            torch.cuda.synchronize()
            log(f"reference: {(k + 1) * segment} of {steps} steps")
        x = buf.double().reshape(buf.shape[0], nb, chains, d)
        s1 += x.sum(dim=(0, 2))
        s2 += (x * x).sum(dim=(0, 2))
        n += buf.shape[0] * chains
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


def compare(E, A, eval_b, net, chains=64, steps=48000, thin=20, level=2.0, ref=None, seed=0,
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
    Accuracy: |posterior mean - reference| / MCSE over problems and the first
    16 monitored coordinates (largest value, and the share within 3); runs are
    at equal accuracy when every arm reaches `min_ess_per_problem` >= 400."""
    import torch
    from . import diagnostics as D
    m, d = A.shape
    nb = len(eval_b)
    if ref is None:
        ref = reference_moments(E, A, eval_b, chains=chains, burn=max(20000, steps // 2),
                                steps=4 * steps, thin=20, seed=seed + 1, log=log)
    ref_mean, ref_sd = ref
    mon = np.sort(np.random.default_rng(seed).choice(d, min(d, 64), replace=False))
    mon_t = torch.as_tensor(mon, device="cuda")
    B = np.repeat(eval_b, chains, axis=0)
    marks = [k for k in (0, 100, 500, 1000, 2000, 4000, 8000, 16000, 32000) if k <= steps]
    out = {"reference": f"{chains} chains per b, {max(20000, steps // 2)} burn-in + {4 * steps} steps",
           "burn_in_level": level}

    def finish(name, tr, x0, wall):
        curve = _device_curve(tr, x0, nb, chains, ref_mean, ref_sd)
        tb = burn_in_steps(curve, level)           # in recorded steps
        x = tr[max(tb - 1, 0):]
        T = x.shape[0]
        if T >= 8:
            sq = torch.cat([(x[i:i + 512].double() ** 2).sum(dim=2, keepdim=True)
                            for i in range(0, T, 512)]).to(x.dtype)
            q = torch.cat([x.index_select(2, mon_t), sq], dim=2)      # (T, C, 65)
            Qn = q.shape[2]
            qb = q.reshape(T, nb, chains, Qn).permute(0, 2, 1, 3).reshape(T, chains, nb * Qn)
            step = max(Qn, (1 << 27) // max(1, T * chains) // Qn * Qn)   # bounded memory
            e = torch.cat([D.ess_batch(qb[:, :, i:i + step]) for i in range(0, nb * Qn, step)])
            e_all = e.reshape(nb, Qn)
            e = e_all.min(dim=1).values                                 # per problem
            ess, worst = float(e.sum()), float(e.min())
            c16 = qb.reshape(T, chains, nb, Qn)[:, :, :, :16].reshape(T, chains, nb * 16)
            se = D.mcse_mean_batch(c16)
            mean = c16.double().mean(dim=(0, 1))
            want = torch.as_tensor(ref_mean[:, mon[:16]].reshape(-1), device=mean.device)
            zs = ((mean - want).abs() / se.clamp_min(1e-12)).cpu().numpy()
        else:
            ess, worst, zs = 0.0, 0.0, np.zeros(1)
        out[name] = {"burn_in_steps": tb * thin, "burn_in_excess": burn_in_excess(curve) * thin,
                     "median_ess_coordinates": float(e_all[:, :-1].median()) if T >= 8 else 0.0,
                     "median_ess_sq_norm": float(e_all[:, -1].median()) if T >= 8 else 0.0,
                     "D_at_step": {str(k): round(float(curve[k // thin]), 3) for k in marks},
                     "ess": ess, "min_ess_per_problem": worst, "wall_s": wall,
                     "ess_per_s": ess / wall, "max_z_mean_vs_reference": float(zs.max()),
                     "share_z_within_3": float((zs <= 3.0).mean())}
        if log:
            log(f"{name}: {out[name]}")

    seg = min(steps, 2000)
    steps -= steps % seg

    def timed_run(samplers, start, name):
        """Every sampler runs `steps` steps in segments of `seg` into a buffer
        of its own, so each captures its graph once, before the clock starts
        (a capture run, then the state is reset).  `start(i, s)` sets sampler
        i's start state inside the timed region.  Returns the trace
        (steps / thin, total chains, d) and the wall time."""
        bufs = [torch.empty(seg // thin, q.n_chains, d, device="cuda") for q in samplers]
        for q, buf in zip(samplers, bufs):
            q.run(seg, thin=thin, count_rejections=False, out=buf)
            q.set_state(torch.zeros(q.n_chains, d, device="cuda"), 0)
        full = torch.empty(steps // thin, sum(q.n_chains for q in samplers), d, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, q in enumerate(samplers):
            start(i, q)
        for k in range(steps // seg):
            rows = slice(k * (seg // thin), (k + 1) * (seg // thin))
            c0 = 0
            for q, buf in zip(samplers, bufs):
                q.run(seg, thin=thin, count_rejections=False, out=buf)
                full[rows, c0:c0 + q.n_chains].copy_(buf)
                c0 += q.n_chains
            if log and k % 10 == 9 and len(samplers) > 1:
                torch.cuda.synchronize()   # progress of the slow arm (its wall time includes this)
                log(f"{name}: {(k + 1) * seg} of {steps} steps")
        torch.cuda.synchronize()
        return full, time.perf_counter() - t0

    zeros = torch.zeros(B.shape[0], d, device="cuda")
    ctxs = [E.Sampler(A, b, np.zeros(d), chains, seed=seed + 100 + j, precision=32)
            for j, b in enumerate(eval_b)]
    tr, wall = timed_run(ctxs, lambda i, q: None, "plain_per_problem")
    for q in ctxs:
        q.close()
    finish("plain_per_problem", tr, zeros, wall)
    del tr

    bdev = torch.tensor(eval_b, dtype=torch.float32, device="cuda")
    for name in ("batched_plain", "batched_warm"):
        s = E.Sampler(A, B, np.zeros(d), B.shape[0], seed=seed + 7, precision=32)
        gate = {}

        def start(i, q):
            if name == "batched_warm":
                gate["xhat"] = net.forward(bdev).repeat_interleave(chains, dim=0)
                gate["acc"] = q.set_state_gated(gate["xhat"], zeros)

        tr, wall = timed_run([s], start, name)
        x0 = zeros
        if name == "batched_warm":
            acc = gate["acc"]
            x0 = gate["xhat"] * torch.as_tensor(acc, device="cuda", dtype=torch.float32)[:, None]
            out["gate_accepted"] = float(np.mean(acc))
        s.close()
        finish(name, tr, x0, wall)
        del tr
    out["equal_accuracy"] = all(out[k]["min_ess_per_problem"] >= 400 for k in
                                ("plain_per_problem", "batched_plain", "batched_warm"))
    out["ess_per_s_batched_warm_over_plain_per_problem"] = (
        out["batched_warm"]["ess_per_s"] / max(out["plain_per_problem"]["ess_per_s"], 1e-30))
    out["ess_per_s_batched_warm_over_batched_plain"] = (
        out["batched_warm"]["ess_per_s"] / max(out["batched_plain"]["ess_per_s"], 1e-30))
    return out
