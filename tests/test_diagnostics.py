"""Effective sample size against closed forms (no GPU)."""
import numpy as np

from paper_2407_10449_amd import diagnostics as D


def ar1(rng, rho, n, m):
    x = np.empty((n, m))
    x[0] = rng.standard_normal(m) / np.sqrt(1 - rho ** 2)
    e = rng.standard_normal((n, m))
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    return x


def test_iid_draws_have_full_ess():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2000, 8))
    assert 0.85 * x.size < D.ess(x) < 1.15 * x.size


def test_ar1_ess_matches_closed_form():
    # AR(1): integrated autocorrelation time (1 + rho) / (1 - rho)
    rng = np.random.default_rng(1)
    for rho in (0.5, 0.9):
        x = ar1(rng, rho, 4000, 8)
        want = x.size * (1 - rho) / (1 + rho)
        got = D.ess(x, rank=False)
        assert 0.75 * want < got < 1.3 * want, (rho, got, want)


def test_rhat_detects_unmixed_chains():
    rng = np.random.default_rng(2)
    good = rng.standard_normal((1000, 4))
    bad = good + np.array([0, 0, 0, 3.0])
    assert D.rhat(good) < 1.01
    assert D.rhat(bad) > 1.1


def test_mcse_of_iid_mean():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4000, 4))
    assert abs(D.mcse_mean(x) - 1 / np.sqrt(x.size)) < 0.15 / np.sqrt(x.size)


def test_batched_estimators_equal_the_reference_ones():
    """The torch versions reproduce ess / mcse_mean, including ties, constant
    draws and random walks."""
    torch = __import__("pytest").importorskip("torch")
    rng = np.random.default_rng(5)
    T, M, Q = 401, 12, 6
    x = rng.standard_normal((T, M, Q)).cumsum(0) * 0.05 + rng.standard_normal((T, M, Q))
    x[:, :, 2] = np.round(x[:, :, 2], 1)
    x[:, :, 3] = 2.5
    x[:, :, 4] = rng.standard_normal((T, M)).cumsum(0)
    x[:, :, 5] = ar1(rng, 0.9, T, M)
    got = D.ess_batch(torch.as_tensor(x)).numpy()
    want = np.array([D.ess(x[:, :, q]) for q in range(Q)])
    np.testing.assert_allclose(got, want, rtol=1e-9)
    got = D.ess_batch(torch.as_tensor(x), rank=False).numpy()
    want = np.array([D.ess(x[:, :, q], rank=False) for q in range(Q)])
    np.testing.assert_allclose(got, want, rtol=1e-9)
    keep = [0, 1, 2, 4, 5]
    got = D.mcse_mean_batch(torch.as_tensor(x[:, :, keep])).numpy()
    want = np.array([D.mcse_mean(x[:, :, q]) for q in keep])
    np.testing.assert_allclose(got, want, rtol=1e-9)
