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
    # Geyer: sums of adjacent pairs, positive and monotone
    t = 0
    pairs = []
    while t + 1 < n:
        p = rho[t] + rho[t + 1]
        if p <= 0:
            break
        pairs.append(p)
        t += 2
    pairs = np.minimum.accumulate(np.array(pairs)) if pairs else np.array([1.0])
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
