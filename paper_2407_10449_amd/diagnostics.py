"""Convergence and efficiency diagnostics for traces (host-side numpy).

Effective sample size and split-R-hat follow Vehtari, Gelman, Simpson,
Carpenter & Buerkner, "Rank-normalization, folding, and localization: an
improved R-hat for assessing convergence of MCMC" (Bayesian Analysis, 2021):
chains are split in halves, draws are rank-normalised (bulk), the
autocorrelation is estimated from the multi-chain variogram, and the sum of
autocorrelations is truncated with Geyer's initial monotone sequence.

These read sampler output after the run; they are not part of the sampler.
"""
import numpy as np
from scipy import stats


def _split(x):
    """(draws, chains) -> (draws // 2, 2 chains)."""
    n = x.shape[0] // 2
    return np.concatenate([x[:n], x[x.shape[0] - n:]], axis=1)


def _rank_normalise(x):
    flat = x.ravel()
    r = stats.rankdata(flat, method="average").reshape(x.shape)
    return stats.norm.ppf((r - 0.375) / (flat.size + 0.25))


def _autocov(x):
    """Autocovariance of each column via FFT, lags 0..n-1."""
    n = x.shape[0]
    xc = x - x.mean(axis=0)
    f = np.fft.rfft(xc, n=2 * n, axis=0)
    ac = np.fft.irfft(f * np.conj(f), axis=0)[:n]
    return ac / n


def ess(x, rank=True):
    """Bulk effective sample size of draws x with shape (draws, chains)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    xs = _split(x)
    if rank:
        xs = _rank_normalise(xs)
    n, m = xs.shape
    if n < 4:
        return float(n * m)
    acov = _autocov(xs)
    chain_mean = xs.mean(axis=0)
    chain_var = acov[0] * n / (n - 1.0)
    w = chain_var.mean()
    b_over_n = chain_mean.var(ddof=1) if m > 1 else 0.0
    var_plus = w * (n - 1.0) / n + b_over_n
    if var_plus <= 0:
        return float(n * m)
    rho = 1.0 - (w - acov.mean(axis=1)) / var_plus
    rho[0] = 1.0
    # Geyer: sums of adjacent pairs, kept while positive, made monotone
    k = (n - 1) // 2 * 2
    pairs = rho[0:k:2] + rho[1:k:2] if k else np.zeros(0)
    bad = np.nonzero(pairs <= 0)[0]
    if bad.size:
        pairs = pairs[:bad[0]]
    pairs = np.minimum.accumulate(pairs) if pairs.size else np.array([1.0])
    tau = -1.0 + 2.0 * pairs.sum()
    tau = max(tau, 1.0 / np.log10(n * m))
    return float(n * m / tau)


def rhat(x):
    """Rank-normalised split-R-hat (max of bulk and folded)."""
    x = np.asarray(x, dtype=np.float64)
    xs = _split(x)

    def _r(z):
        n = z.shape[0]
        w = z.var(axis=0, ddof=1).mean()
        bn = z.mean(axis=0).var(ddof=1)
        return np.sqrt(((n - 1.0) / n * w + bn) / w)

    z = _rank_normalise(xs)
    zf = _rank_normalise(np.abs(xs - np.median(xs)))
    return float(max(_r(z), _r(zf)))


def min_ess(trace, functionals=None):
    """Minimum bulk ESS over monitored functionals of a trace (draws, chains, d):
    every coordinate (or the given subset) and the squared norm."""
    trace = np.asarray(trace, dtype=np.float64)
    cols = range(trace.shape[2]) if functionals is None else functionals
    vals = [ess(trace[:, :, j]) for j in cols]
    vals.append(ess((trace ** 2).sum(axis=2)))
    return float(min(vals))


def mcse_mean(x):
    """Monte Carlo standard error of the mean of draws (draws, chains)."""
    x = np.asarray(x, dtype=np.float64)
    return float(x.std(ddof=1) / np.sqrt(ess(x, rank=False)))


def ess_batch(x, rank=True):
    """Bulk ESS of many quantities at once: x is a torch tensor of shape
    (draws, chains, quantities) on any device; returns a float64 tensor of
    length `quantities`.  The same estimator as `ess` (split chains,
    rank-normalisation with average ranks for ties, multi-chain
    autocorrelation, Geyer's initial monotone sequence), evaluated with torch
    so that thousands of quantities take milliseconds on the GPU."""
    import torch
    x = x.to(torch.float64)
    T, M, Q = x.shape
    n = T // 2
    xs = torch.cat([x[:n], x[T - n:]], dim=1)            # (n, 2M, Q)
    m = xs.shape[1]
    N = n * m
    if not rank:
        return _ess_from(xs, n, N)
    flat = xs.permute(2, 0, 1).reshape(Q, N)             # one row per quantity
    sv, si = torch.sort(flat, dim=1)
    pos = torch.arange(1, N + 1, device=x.device, dtype=torch.float64).expand(Q, N)
    # average rank over runs of equal values: run start / end positions by
    # a forward cummax of run starts and a backward cummin of run ends
    new_run = torch.ones_like(sv, dtype=torch.bool)
    new_run[:, 1:] = sv[:, 1:] != sv[:, :-1]
    end_run = torch.ones_like(sv, dtype=torch.bool)
    end_run[:, :-1] = new_run[:, 1:]
    first = torch.where(new_run, pos, torch.zeros_like(pos)).cummax(dim=1).values
    last = torch.where(end_run, pos, torch.full_like(pos, float(N + 1)))
    last = last.flip(1).cummin(dim=1).values.flip(1)
    ranks = torch.empty_like(pos)
    ranks.scatter_(1, si, 0.5 * (first + last))
    z = torch.special.ndtri((ranks - 0.375) / (N + 0.25))
    return _ess_from(z.reshape(Q, n, m).permute(1, 2, 0), n, N)


def _ess_from(z, n, N):
    """ESS from split draws z of shape (n, chains, quantities)."""
    import torch
    zc = z - z.mean(dim=0, keepdim=True)
    f = torch.fft.rfft(zc, n=2 * n, dim=0)
    acov = torch.fft.irfft(f * f.conj(), n=2 * n, dim=0)[:n] / n   # (n, 2M, Q)
    chain_mean = z.mean(dim=0)                           # (2M, Q)
    chain_var = acov[0] * n / (n - 1.0)
    w = chain_var.mean(dim=0)                            # (Q,)
    b_over_n = chain_mean.var(dim=0, unbiased=True)
    var_plus = w * (n - 1.0) / n + b_over_n
    rho = 1.0 - (w[None] - acov.mean(dim=1)) / var_plus[None]   # (n, Q)
    rho[0] = 1.0
    k = (n - 1) // 2 * 2
    pairs = rho[0:k:2] + rho[1:k:2]                      # (k / 2, Q)
    alive = (pairs > 0).to(torch.int64).cumprod(dim=0).bool()
    mono = pairs.cummin(dim=0).values
    tau = -1.0 + 2.0 * torch.where(alive, mono, torch.zeros_like(mono)).sum(dim=0)
    tau = torch.where(alive[0], tau, torch.ones_like(tau))   # no positive pair: as `ess`
    tau = torch.clamp(tau, min=1.0 / np.log10(N))
    return torch.where(var_plus > 0, N / tau, torch.full_like(tau, float(N)))


def mcse_mean_batch(x):
    """Monte Carlo standard error of the mean of every quantity of a torch
    tensor (draws, chains, quantities), as `mcse_mean`."""
    x = x.to(dtype=__import__("torch").float64)
    sd = x.reshape(-1, x.shape[2]).std(dim=0, unbiased=True)
    return sd / ess_batch(x, rank=False).sqrt()
